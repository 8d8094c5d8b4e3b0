// Device-wide exclusive scan and stable LSD radix sort (see hln_prim.hpp).
#include "hln_prim.hpp"

#include <algorithm>

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

constexpr int kSortBlock = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortBlock * kSortRounds;
constexpr int kRadix = 256;

template <typename T>
__device__ __forceinline__ T shfl_up_t(T x, int off) {
    if constexpr (sizeof(T) == 8) {
        int lo = __shfl_up(static_cast<int>(static_cast<unsigned long long>(x) & 0xffffffffull), off, 64);
        int hi = __shfl_up(static_cast<int>(static_cast<unsigned long long>(x) >> 32), off, 64);
        return static_cast<T>((static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                              static_cast<unsigned>(lo));
    } else {
        return __shfl_up(x, off, 64);
    }
}

// Inclusive scan of one value per thread over a block of kScanBlock
// threads; returns the inclusive prefix and writes the block total.
template <typename T>
__device__ __forceinline__ T block_inclusive_scan(T x, T* s_wave, T& total) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T y = shfl_up_t(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    T before = 0;
    T all = 0;
    for (int w = 0; w < kScanBlock / 64; ++w) {
        if (w < wave) before += s_wave[w];
        all += s_wave[w];
    }
    __syncthreads();
    total = all;
    return x + before;
}

template <typename T>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const T* __restrict__ in, long long count, T* sums) {
    __shared__ T s_wave[kScanBlock / 64];
    const long long base = static_cast<long long>(blockIdx.x) * kScanTile + static_cast<long long>(threadIdx.x) * kScanItems;
    T x = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < count) x += in[base + i];
    T total;
    block_inclusive_scan<T>(x, s_wave, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block: exclusive scan of the block sums in place; total to *total_out.
template <typename T>
__global__ __launch_bounds__(kScanBlock) void k_scan_sums(T* sums, long long nb, T* total_out) {
    __shared__ T s_wave[kScanBlock / 64];
    T carry = 0;
    for (long long c = 0; c < nb; c += kScanBlock) {
        const long long i = c + threadIdx.x;
        const T x = i < nb ? sums[i] : T(0);
        T total;
        const T inc = block_inclusive_scan<T>(x, s_wave, total);
        if (i < nb) sums[i] = carry + inc - x;
        carry += total;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

template <typename T>
__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const T* in, T* out, long long count, const T* offs) {
    __shared__ T s_wave[kScanBlock / 64];
    const long long base = static_cast<long long>(blockIdx.x) * kScanTile + static_cast<long long>(threadIdx.x) * kScanItems;
    T v[kScanItems];
    T x = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < count ? in[base + i] : T(0);
        x += v[i];
    }
    T total;
    const T inc = block_inclusive_scan<T>(x, s_wave, total);
    T run = offs[blockIdx.x] + inc - x;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < count) out[base + i] = run;
        run += v[i];
    }
}

__global__ __launch_bounds__(kSortBlock) void k_sort_hist(const unsigned long long* __restrict__ keys, long long count,
                                                          int shift, int nb, int32_t* hist) {
    __shared__ int s_h[kRadix];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const long long base = static_cast<long long>(blockIdx.x) * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const long long i = base + r * kSortBlock + threadIdx.x;
        if (i < count) atomicAdd(&s_h[(keys[i] >> shift) & (kRadix - 1)], 1);
    }
    __syncthreads();
    hist[static_cast<long long>(threadIdx.x) * nb + blockIdx.x] = s_h[threadIdx.x];
}

// Stable scatter of one tile: the tile is taken in rounds of kSortBlock keys
// in index order; inside a round, lanes holding the same digit are ranked by
// lane index (ballots over the digit bits) and waves in wave order.
__global__ __launch_bounds__(kSortBlock) void k_sort_scatter(const unsigned long long* __restrict__ kin,
                                                             const int32_t* __restrict__ vin,
                                                             unsigned long long* __restrict__ kout,
                                                             int32_t* __restrict__ vout, long long count, int shift,
                                                             int nb, const int32_t* __restrict__ offs) {
    constexpr int kWaves = kSortBlock / 64;
    __shared__ int s_base[kRadix];
    __shared__ int s_wcnt[kWaves][kRadix];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    s_base[threadIdx.x] = offs[static_cast<long long>(threadIdx.x) * nb + blockIdx.x];
    const unsigned long long lt = (1ull << lane) - 1ull;
    const long long base = static_cast<long long>(blockIdx.x) * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        for (int i = threadIdx.x; i < kWaves * kRadix; i += kSortBlock) (&s_wcnt[0][0])[i] = 0;
        __syncthreads();
        const long long idx = base + r * kSortBlock + threadIdx.x;
        const bool valid = idx < count;
        const unsigned long long key = valid ? kin[idx] : 0ull;
        const int32_t val = valid ? vin[idx] : 0;
        const int d = static_cast<int>((key >> shift) & (kRadix - 1));
        const unsigned long long live = __ballot(valid);
        unsigned long long same = live;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int bit = (d >> b) & 1;
            const unsigned long long bal = __ballot(valid && bit);
            same &= bit ? bal : (live & ~bal);
        }
        const int rank = __popcll(same & lt);
        if (valid && rank == 0) s_wcnt[wave][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            int pre = 0;
            for (int w = 0; w < wave; ++w) pre += s_wcnt[w][d];
            const int pos = s_base[d] + pre + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        int add = 0;
        for (int w = 0; w < kWaves; ++w) add += s_wcnt[w][threadIdx.x];
        s_base[threadIdx.x] += add;
        __syncthreads();
    }
}

__global__ void k_copy_pairs(const unsigned long long* kin, const int32_t* vin, unsigned long long* kout,
                             int32_t* vout, long long count) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        kout[i] = kin[i];
        vout[i] = vin[i];
    }
}

long long scan_blocks(long long count) { return std::max<long long>(1, (count + kScanTile - 1) / kScanTile); }

}  // namespace

namespace hln {
namespace prim {

size_t scan_workspace(long long count) { return Arena::round(static_cast<size_t>(scan_blocks(count) + 1) * 8); }

template <typename T>
hln_status scan_exclusive(const T* in, T* out, long long count, void* ws, size_t ws_bytes, hipStream_t st) {
    const long long nb = scan_blocks(count);
    if (ws_bytes < scan_workspace(count)) return fail(HLN_ENOMEM, "scan workspace too small");
    T* sums = static_cast<T*>(ws);
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3(static_cast<unsigned>(nb)), dim3(kScanBlock), 0, st, in, count, sums);
    hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(kScanBlock), 0, st, sums, nb, out + count);
    hipLaunchKernelGGL(k_scan_apply<T>, dim3(static_cast<unsigned>(nb)), dim3(kScanBlock), 0, st, in, out, count,
                       sums);
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

template hln_status scan_exclusive<int32_t>(const int32_t*, int32_t*, long long, void*, size_t, hipStream_t);
template hln_status scan_exclusive<int64_t>(const int64_t*, int64_t*, long long, void*, size_t, hipStream_t);

size_t sort_workspace(long long count) {
    const long long nb = std::max<long long>(1, (count + kSortTile - 1) / kSortTile);
    const long long hist = nb * kRadix;
    return Arena::round(static_cast<size_t>(count) * 8) + Arena::round(static_cast<size_t>(count) * 4) +
           Arena::round(static_cast<size_t>(hist + 1) * 4) + scan_workspace(hist);
}

hln_status sort_pairs(unsigned long long* keys, int32_t* vals, long long count, int key_bits, void* ws,
                      size_t ws_bytes, hipStream_t st) {
    if (count <= 1) return HLN_OK;
    if (ws_bytes < sort_workspace(count)) return fail(HLN_ENOMEM, "sort workspace too small");
    const long long nb = (count + kSortTile - 1) / kSortTile;
    if (nb * kRadix >= (1ll << 31)) return fail(HLN_EUNSUPPORTED, "sort too large");
    Arena ar{static_cast<char*>(ws), ws_bytes};
    unsigned long long* kalt = ar.take<unsigned long long>(count);
    int32_t* valt = ar.take<int32_t>(count);
    int32_t* hist = ar.take<int32_t>(nb * kRadix + 1);
    void* sws = ar.base + ar.off;
    const size_t sws_bytes = ws_bytes - ar.off;
    unsigned long long* ka = keys;
    int32_t* va = vals;
    unsigned long long* kb = kalt;
    int32_t* vb = valt;
    const int passes = std::max(1, (key_bits + 7) / 8);
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_sort_hist, dim3(static_cast<unsigned>(nb)), dim3(kSortBlock), 0, st, ka, count, shift,
                           static_cast<int>(nb), hist);
        hln_status s = scan_exclusive<int32_t>(hist, hist, nb * kRadix, sws, sws_bytes, st);
        if (s != HLN_OK) return s;
        hipLaunchKernelGGL(k_sort_scatter, dim3(static_cast<unsigned>(nb)), dim3(kSortBlock), 0, st, ka, va, kb, vb,
                           count, shift, static_cast<int>(nb), hist);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        const unsigned grid = static_cast<unsigned>(std::min<long long>((count + 255) / 256, 4096));
        hipLaunchKernelGGL(k_copy_pairs, dim3(grid), dim3(256), 0, st, ka, va, keys, vals, count);
    }
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

}  // namespace prim
}  // namespace hln
