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

// Histogram of one tile's digits, keys [begin, end).
__device__ __forceinline__ void hist_tile(const unsigned long long* __restrict__ keys, long long begin, long long end,
                                          int shift, int* s_h) {
    s_h[threadIdx.x] = 0;
    __syncthreads();
    for (int r = 0; r < kSortRounds; ++r) {
        const long long i = begin + r * kSortBlock + threadIdx.x;
        if (i < end) atomicAdd(&s_h[(keys[i] >> shift) & (kRadix - 1)], 1);
    }
    __syncthreads();
}

// Stable scatter of one tile, keys [begin, end) (at most kSortTile), whose
// digit d goes to s_base[d] onwards.  The tile is taken in rounds of
// kSortBlock keys in index order; inside a round, lanes holding the same
// digit are ranked by lane index (ballots over the digit bits) and waves in
// wave order.  kVals: values move with their keys.
template <bool kVals>
__device__ __forceinline__ void scatter_tile(const unsigned long long* __restrict__ kin,
                                             const int32_t* __restrict__ vin, unsigned long long* __restrict__ kout,
                                             int32_t* __restrict__ vout, long long begin, long long end, int shift,
                                             int* s_base, int (*s_wcnt)[kRadix]) {
    constexpr int kWaves = kSortBlock / 64;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int r = 0; r < kSortRounds; ++r) {
        for (int i = threadIdx.x; i < kWaves * kRadix; i += kSortBlock) (&s_wcnt[0][0])[i] = 0;
        __syncthreads();
        const long long idx = begin + r * kSortBlock + threadIdx.x;
        const bool valid = idx < end;
        const unsigned long long key = valid ? kin[idx] : 0ull;
        int32_t val = 0;
        if constexpr (kVals) val = valid ? vin[idx] : 0;
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
            if constexpr (kVals) vout[pos] = val;
        }
        __syncthreads();
        int add = 0;
        for (int w = 0; w < kWaves; ++w) add += s_wcnt[w][threadIdx.x];
        s_base[threadIdx.x] += add;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kSortBlock) void k_sort_hist(const unsigned long long* __restrict__ keys, long long count,
                                                          int shift, int nb, int32_t* hist) {
    __shared__ int s_h[kRadix];
    const long long base = static_cast<long long>(blockIdx.x) * kSortTile;
    hist_tile(keys, base, count, shift, s_h);
    hist[static_cast<long long>(threadIdx.x) * nb + blockIdx.x] = s_h[threadIdx.x];
}

__global__ __launch_bounds__(kSortBlock) void k_sort_scatter(const unsigned long long* __restrict__ kin,
                                                             const int32_t* __restrict__ vin,
                                                             unsigned long long* __restrict__ kout,
                                                             int32_t* __restrict__ vout, long long count, int shift,
                                                             int nb, const int32_t* __restrict__ offs) {
    __shared__ int s_base[kRadix];
    __shared__ int s_wcnt[kSortBlock / 64][kRadix];
    s_base[threadIdx.x] = offs[static_cast<long long>(threadIdx.x) * nb + blockIdx.x];
    const long long base = static_cast<long long>(blockIdx.x) * kSortTile;
    scatter_tile<true>(kin, vin, kout, vout, base, count, shift, s_base, s_wcnt);
}

// Segmented sort: segment s holds keys [key_off[s], key_off[s+1]) and tiles
// [tile_off[s], tile_off[s+1]), one tile per kSortTile keys.  Its histogram
// block starts at kRadix * tile_off[s], digit-major (d * tiles + tile), so
// one exclusive scan over all histograms places every segment's keys in its
// own range.  Largest s in [0, nseg) with off[s] <= x (empty segments are
// skipped: a later segment with the same offset wins).
__device__ __forceinline__ int seg_of(const long long* __restrict__ off, int nseg, long long x) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct SegTile {
    long long begin, end;      // keys of this tile: [begin, min(end, begin + kSortTile))
    long long hist_base;       // kRadix * tile_off[s]
    long long nb, t;           // tiles of the segment, this tile's index in it
};

__device__ __forceinline__ SegTile seg_tile(const long long* __restrict__ key_off,
                                            const long long* __restrict__ tile_off, int nseg) {
    const long long b = blockIdx.x;
    const int s = seg_of(tile_off, nseg, b);
    SegTile T;
    const long long t0 = tile_off[s];
    T.nb = tile_off[s + 1] - t0;
    T.t = b - t0;
    T.begin = key_off[s] + T.t * kSortTile;
    T.end = key_off[s + 1];
    T.hist_base = static_cast<long long>(kRadix) * t0;
    return T;
}

__global__ __launch_bounds__(kSortBlock) void k_seg_hist(const unsigned long long* __restrict__ keys,
                                                         const long long* __restrict__ key_off,
                                                         const long long* __restrict__ tile_off, int nseg, int shift,
                                                         int32_t* hist) {
    __shared__ int s_h[kRadix];
    const SegTile T = seg_tile(key_off, tile_off, nseg);
    hist_tile(keys, T.begin, T.end, shift, s_h);
    hist[T.hist_base + static_cast<long long>(threadIdx.x) * T.nb + T.t] = s_h[threadIdx.x];
}

template <bool kVals>
__global__ __launch_bounds__(kSortBlock) void k_seg_scatter(const unsigned long long* __restrict__ kin,
                                                            const int32_t* __restrict__ vin,
                                                            unsigned long long* __restrict__ kout,
                                                            int32_t* __restrict__ vout,
                                                            const long long* __restrict__ key_off,
                                                            const long long* __restrict__ tile_off, int nseg,
                                                            int shift, const int32_t* __restrict__ offs) {
    __shared__ int s_base[kRadix];
    __shared__ int s_wcnt[kSortBlock / 64][kRadix];
    const SegTile T = seg_tile(key_off, tile_off, nseg);
    s_base[threadIdx.x] = offs[T.hist_base + static_cast<long long>(threadIdx.x) * T.nb + T.t];
    scatter_tile<kVals>(kin, vin, kout, vout, T.begin, T.end, shift, s_base, s_wcnt);
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

long long seg_sort_tiles(long long count) { return (count + kSortTile - 1) / kSortTile; }

size_t seg_sort_workspace(long long tiles) {
    const long long hist = tiles * kRadix;
    return Arena::round(static_cast<size_t>(hist + 1) * 4) + scan_workspace(hist);
}

hln_status sort_segmented(unsigned long long* keys, unsigned long long* alt, int32_t* vals, int32_t* valt,
                          const long long* key_off, const long long* tile_off, int nseg, long long tiles, int key_bits,
                          void* ws, size_t ws_bytes, hipStream_t st, bool* in_alt) {
    *in_alt = false;
    if (tiles <= 0 || nseg <= 0) return HLN_OK;
    if (ws_bytes < seg_sort_workspace(tiles)) return fail(HLN_ENOMEM, "sort workspace too small");
    if (tiles * kRadix >= (1ll << 31) || tiles >= (1ll << 31)) return fail(HLN_EUNSUPPORTED, "sort too large");
    Arena ar{static_cast<char*>(ws), ws_bytes};
    int32_t* hist = ar.take<int32_t>(tiles * kRadix + 1);
    void* sws = ar.base + ar.off;
    const size_t sws_bytes = ws_bytes - ar.off;
    unsigned long long* ka = keys;
    unsigned long long* kb = alt;
    int32_t* va = vals;
    int32_t* vb = valt;
    const int passes = std::max(1, (key_bits + 7) / 8);
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_seg_hist, dim3(static_cast<unsigned>(tiles)), dim3(kSortBlock), 0, st, ka, key_off,
                           tile_off, nseg, shift, hist);
        hln_status s = scan_exclusive<int32_t>(hist, hist, tiles * kRadix, sws, sws_bytes, st);
        if (s != HLN_OK) return s;
        if (vals)
            hipLaunchKernelGGL(k_seg_scatter<true>, dim3(static_cast<unsigned>(tiles)), dim3(kSortBlock), 0, st, ka, va,
                               kb, vb, key_off, tile_off, nseg, shift, hist);
        else
            hipLaunchKernelGGL(k_seg_scatter<false>, dim3(static_cast<unsigned>(tiles)), dim3(kSortBlock), 0, st, ka,
                               nullptr, kb, nullptr, key_off, tile_off, nseg, shift, hist);
        std::swap(ka, kb);
        std::swap(va, vb);
        *in_alt = !*in_alt;
    }
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

}  // namespace prim
}  // namespace hln
