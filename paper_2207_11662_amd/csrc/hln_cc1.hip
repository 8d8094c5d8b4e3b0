// Heuristic CC1 of the composition step (Sec. 5.1, Eq. 2-3).  The paper
// describes CC1 in words only; the readings taken (the same in the test
// oracle):
//   - sumDist is the penalised distance sum P = S + n(n - R): a vertex that
//     cannot be reached counts at distance n (Sec. 5.1);
//   - Eq. 2 over r layers: ratio_l(u) = P_l(u) / m(u), where m(u) is the
//     smallest degree of u over the layers (an upper bound on u's degree in
//     the AND graph); a vertex with m(u) = 0 has no ratio, is never central
//     and is left out of the averages;
//   - avg_l = mean of ratio_l over the vertices with m > 0, summed in a
//     fixed shape (sequentially within id-chunks of 1024, chunk sums in
//     order); Eq. 3: the AND graph's average is the largest avg_l;
//   - a vertex is central in layer l when its ratio is strictly below that
//     average;
//   - CH_l = the above-average closeness set of layer l (Sec. 4, Eq. 1 in
//     the Wasserman-Faust form, the same fixed-shape mean);
//   - a vertex c in every CH_l is a CC1 node when its central neighbour sets
//     C_l(c) = { v in N_l(c) : v central in l } overlap significantly: with
//     I the intersection of the C_l(c) and s the smallest |C_l(c)|, s > 0
//     and |I| * tau_den >= tau_num * s.
//
// Kernels: per-vertex degree bound; per-(layer, chunk) sums of the ratios
// and closeness values; per-layer means and Eq. 3 (one thread per layer);
// per-vertex central bits (one bit per layer) and the common-CC flag; one
// wave per common CC node for the overlap (lanes stride over the node's
// rows, neighbour membership by binary search in the sorted rows of the
// other layers); scan and compaction of the kept ids.
#include "hln_internal.hpp"
#include "hln_prim.hpp"

#include <algorithm>

namespace {

constexpr int kMaxLayers = 64;
constexpr int kChunk = 1024;

struct Layers {
    int r;
    long long nnz[kMaxLayers];
    const int32_t* row_ptr[kMaxLayers];
    const int32_t* col_idx[kMaxLayers];
    const int64_t* S[kMaxLayers];
    const int32_t* R[kMaxLayers];
};

__device__ __forceinline__ double closeness_wf(int n, int64_t s, int32_t r) {
    if (r > 1 && s > 0 && n > 1) {
        const double reach = static_cast<double>(r - 1);
        const double q1 = reach / static_cast<double>(s);
        const double q2 = reach / static_cast<double>(n - 1);
        return q1 * q2;
    }
    return 0.0;
}

__device__ __forceinline__ double ratio_of(int n, const Layers& L, int l, int u, int32_t m) {
    const int64_t P = L.S[l][u] + static_cast<int64_t>(n) * static_cast<int64_t>(n - L.R[l][u]);
    return static_cast<double>(P) / static_cast<double>(m);
}

__global__ void k_cc1_degree_bound(int n, Layers L, int32_t* m) {
    for (long long uu = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; uu < n;
         uu += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int u = static_cast<int>(uu);
        int32_t best = 0;
        for (int l = 0; l < L.r; ++l) {
            const int32_t d = L.row_ptr[l][u + 1] - L.row_ptr[l][u];
            if (l == 0 || d < best) best = d;
        }
        m[u] = best;
    }
}

// thread (l, c): sequential sums over chunk c of layer l's ratios (m > 0)
// and closeness values; layer 0's threads also count the vertices with m > 0
__global__ void k_cc1_chunks(int n, Layers L, const int32_t* __restrict__ m, int chunks, double* part_ratio,
                             double* part_cc, int32_t* part_valid) {
    const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<long long>(chunks) * L.r) return;
    const int l = static_cast<int>(t / chunks);
    const int c = static_cast<int>(t % chunks);
    const int lo = c * kChunk;
    const int hi = min(lo + kChunk, n);
    double sr = 0.0, sc = 0.0;
    int valid = 0;
    for (int u = lo; u < hi; ++u) {
        const int32_t mu = m[u];
        if (mu > 0) {
            sr += ratio_of(n, L, l, u, mu);
            ++valid;
        }
        sc += closeness_wf(n, L.S[l][u], L.R[l][u]);
    }
    part_ratio[t] = sr;
    part_cc[t] = sc;
    if (l == 0) part_valid[c] = valid;
}

// one thread per layer: the layer's averages; then thread 0 takes Eq. 3
__global__ void k_cc1_means(int n, int r, int chunks, const double* __restrict__ part_ratio,
                            const double* __restrict__ part_cc, const int32_t* __restrict__ part_valid,
                            double* mean_cc, double* avg_l, double* avg, double* avg_out) {
    const int l = threadIdx.x;
    if (l < r) {
        double tr = 0.0, tc = 0.0;
        long long valid = 0;
        for (int c = 0; c < chunks; ++c) {
            tr += part_ratio[static_cast<long long>(l) * chunks + c];
            tc += part_cc[static_cast<long long>(l) * chunks + c];
            valid += part_valid[c];
        }
        avg_l[l] = valid > 0 ? tr / static_cast<double>(valid) : 0.0;
        mean_cc[l] = tc / static_cast<double>(n);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int k = 0; k < r; ++k)
            if (k == 0 || avg_l[k] > a) a = avg_l[k];
        *avg = a;
        if (avg_out) *avg_out = a;
    }
}

// central bits per vertex and the common-CC flag
__global__ void k_cc1_central(int n, Layers L, const int32_t* __restrict__ m, const double* __restrict__ mean_cc,
                              const double* __restrict__ avg, unsigned long long* central, int32_t* flag) {
    const double a = *avg;
    for (long long uu = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; uu < n;
         uu += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int u = static_cast<int>(uu);
        const int32_t mu = m[u];
        unsigned long long bits = 0;
        int common = 1;
        for (int l = 0; l < L.r; ++l) {
            if (mu > 0 && ratio_of(n, L, l, u, mu) < a) bits |= 1ull << l;
            common &= closeness_wf(n, L.S[l][u], L.R[l][u]) >= mean_cc[l] ? 1 : 0;
        }
        central[u] = bits;
        flag[u] = common;
    }
}

__device__ __forceinline__ bool row_has(const int32_t* __restrict__ col, int lo, int hi, int v) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int x = col[mid];
        if (x == v) return true;
        if (x < v) lo = mid + 1;
        else hi = mid;
    }
    return false;
}

__device__ __forceinline__ long long wave_sum(long long x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// row bounds of u in layer l, clamped to the declared arc count so that a
// malformed row pointer cannot send a read outside col_idx
__device__ __forceinline__ int2 row_of(const Layers& L, int l, int u) {
    const long long e0 = min(max(static_cast<long long>(L.row_ptr[l][u]), 0ll), L.nnz[l]);
    const long long e1 = min(max(static_cast<long long>(L.row_ptr[l][u + 1]), e0), L.nnz[l]);
    return make_int2(static_cast<int>(e0), static_cast<int>(e1));
}

// one wave per vertex (grid-stride over waves); only common CC nodes work.
// Column ids outside [0, n) are skipped (they cannot index the central bits).
__global__ __launch_bounds__(256) void k_cc1_overlap(int n, Layers L, const unsigned long long* __restrict__ central,
                                                     int tau_num, int tau_den, int32_t* flag) {
    const int lane = threadIdx.x & 63;
    const long long wave = (static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const long long waves = (static_cast<long long>(gridDim.x) * blockDim.x) >> 6;
    const unsigned long long all = L.r >= 64 ? ~0ull : ((1ull << L.r) - 1ull);
    for (long long cc = wave; cc < n; cc += waves) {
        const int c = static_cast<int>(cc);
        if (!flag[c]) continue;                              // wave-uniform
        long long smallest = -1;
        for (int l = 0; l < L.r; ++l) {
            const int2 rw = row_of(L, l, c);
            long long size = 0;
            for (int e = rw.x + lane; e < rw.y; e += 64) {
                const int v = L.col_idx[l][e];
                if (static_cast<unsigned>(v) < static_cast<unsigned>(n)) size += (central[v] >> l) & 1ull;
            }
            size = wave_sum(size);
            if (smallest < 0 || size < smallest) smallest = size;
        }
        long long inter = 0;
        const int2 r0 = row_of(L, 0, c);
        for (int e = r0.x + lane; e < r0.y; e += 64) {
            const int v = L.col_idx[0][e];
            bool ok = static_cast<unsigned>(v) < static_cast<unsigned>(n) && (central[v] & all) == all;
            for (int l = 1; l < L.r && ok; ++l) {
                const int2 rl = row_of(L, l, c);
                ok = row_has(L.col_idx[l], rl.x, rl.y, v);
            }
            inter += ok ? 1 : 0;
        }
        inter = wave_sum(inter);
        if (lane == 0)
            flag[c] = (smallest > 0 && inter * tau_den >= static_cast<long long>(tau_num) * smallest) ? 1 : 0;
    }
}

__global__ void k_cc1_compact(int n, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos, int32_t* ids,
                              int32_t* count) {
    for (long long u = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; u < n;
         u += static_cast<long long>(gridDim.x) * blockDim.x)
        if (flag[u]) ids[pos[u]] = static_cast<int32_t>(u);
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = pos[n];
}

struct Carve {
    int32_t* m;
    unsigned long long* central;
    int32_t* flag;
    int32_t* pos;
    double* part_ratio;
    double* part_cc;
    int32_t* part_valid;
    double* means;      // mean_cc[r], avg_l[r], avg
    void* scan_ws;
    size_t scan_bytes;
};

size_t carve(int32_t n, int32_t r, char* base, size_t bytes, Carve* out) {
    using hln::Arena;
    const size_t chunks = (static_cast<size_t>(n) + kChunk - 1) / kChunk;
    const size_t scan = hln::prim::scan_workspace(n);
    size_t need = 0;
    need += Arena::round(static_cast<size_t>(n) * 4);                 // m
    need += Arena::round(static_cast<size_t>(n) * 8);                 // central
    need += 2 * Arena::round((static_cast<size_t>(n) + 1) * 4);       // flag, pos
    need += 2 * Arena::round(chunks * r * 8);                         // part_ratio, part_cc
    need += Arena::round(chunks * 4);                                 // part_valid
    need += Arena::round((2 * static_cast<size_t>(r) + 1) * 8);       // means
    need += Arena::round(scan);
    if (!base || !out) return need;
    if (bytes < need) return 0;
    Arena ar{base, bytes};
    out->m = ar.take<int32_t>(n);
    out->central = ar.take<unsigned long long>(n);
    out->flag = ar.take<int32_t>(static_cast<size_t>(n) + 1);
    out->pos = ar.take<int32_t>(static_cast<size_t>(n) + 1);
    out->part_ratio = ar.take<double>(chunks * r);
    out->part_cc = ar.take<double>(chunks * r);
    out->part_valid = ar.take<int32_t>(chunks);
    out->means = ar.take<double>(2 * static_cast<size_t>(r) + 1);
    out->scan_ws = ar.take<char>(scan);
    out->scan_bytes = scan;
    return need;
}

int grid_for(long long items, int block, int cus) {
    const long long g = (items + block - 1) / block;
    return static_cast<int>(std::max<long long>(1, std::min<long long>(g, static_cast<long long>(cus) * 16)));
}

}  // namespace

extern "C" {

size_t hln_compose_cc1_workspace_size(int32_t n, int32_t r) {
    if (n < 1 || r < 1 || r > kMaxLayers) return 0;
    return carve(n, r, nullptr, 0, nullptr);
}

hln_status hln_compose_cc1(const hln_csr* layers, int32_t r, const int64_t* const* S, const int32_t* const* R,
                           int32_t tau_num, int32_t tau_den, int32_t* ids, int32_t* count, double* avg,
                           void* workspace, size_t workspace_bytes, void* stream) {
    using hln::fail;
    hln::clear_error();
    if (!layers || !S || !R) return fail(HLN_EINVAL, "layers, S and R are required");
    if (r < 1 || r > kMaxLayers) return fail(HLN_EINVAL, "r must be in [1, %d] (got %d)", kMaxLayers, r);
    if (tau_num < 0 || tau_den < 1) return fail(HLN_EINVAL, "tau must be tau_num >= 0 over tau_den >= 1");
    if (!ids || !count) return fail(HLN_EINVAL, "ids and count are required");
    const int n = layers[0].n;
    if (n < 1) return fail(HLN_EINVAL, "n must be >= 1");
    Layers L{};
    L.r = r;
    for (int l = 0; l < r; ++l) {
        if (layers[l].n != n) return fail(HLN_EINVAL, "layer %d has n = %d, layer 0 has %d", l, layers[l].n, n);
        if (!layers[l].row_ptr || (layers[l].nnz > 0 && !layers[l].col_idx) || !S[l] || !R[l])
            return fail(HLN_EINVAL, "layer %d: NULL array", l);
        L.nnz[l] = layers[l].nnz;
        L.row_ptr[l] = layers[l].row_ptr;
        L.col_idx[l] = layers[l].col_idx;
        L.S[l] = S[l];
        L.R[l] = R[l];
    }
    if (!workspace) return fail(HLN_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % hln::Arena::kAlign) return fail(HLN_EINVAL, "workspace not 256-byte aligned");
    Carve w{};
    const size_t need = carve(n, r, nullptr, 0, nullptr);
    if (workspace_bytes < need) return fail(HLN_ENOMEM, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
    carve(n, r, static_cast<char*>(workspace), workspace_bytes, &w);
    const hln::DeviceInfo* di = hln::device_info();
    if (!di) return HLN_EDEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int chunks = (n + kChunk - 1) / kChunk;
    double* mean_cc = w.means;
    double* avg_l = w.means + r;
    double* avg_dev = w.means + 2 * r;

    hipLaunchKernelGGL(k_cc1_degree_bound, dim3(grid_for(n, 256, di->cus)), dim3(256), 0, st, n, L, w.m);
    const long long threads = static_cast<long long>(chunks) * r;
    hipLaunchKernelGGL(k_cc1_chunks, dim3(static_cast<int>((threads + 63) / 64)), dim3(64), 0, st, n, L, w.m, chunks,
                       w.part_ratio, w.part_cc, w.part_valid);
    hipLaunchKernelGGL(k_cc1_means, dim3(1), dim3(64), 0, st, n, r, chunks, w.part_ratio, w.part_cc, w.part_valid,
                       mean_cc, avg_l, avg_dev, avg);
    hipLaunchKernelGGL(k_cc1_central, dim3(grid_for(n, 256, di->cus)), dim3(256), 0, st, n, L, w.m, mean_cc, avg_dev,
                       w.central, w.flag);
    hipLaunchKernelGGL(k_cc1_overlap, dim3(grid_for(static_cast<long long>(n) * 64, 256, di->cus)), dim3(256), 0, st, n,
                       L, w.central, tau_num, tau_den, w.flag);
    HLN_TRY_HIP(hipGetLastError());
    hln_status s = hln::prim::scan_exclusive<int32_t>(w.flag, w.pos, n, w.scan_ws, w.scan_bytes, st);
    if (s != HLN_OK) return s;
    hipLaunchKernelGGL(k_cc1_compact, dim3(grid_for(n, 256, di->cus)), dim3(256), 0, st, n, w.flag, w.pos, ids, count);
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

}  // extern "C"
