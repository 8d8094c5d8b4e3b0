// CC-node selection and the composition step (Theta) of the decoupling
// method.
//
//   HLN_RANK_WF    one graph: score = closeness (Sec. 4, Eq. 1, Wasserman-
//                  Faust form); the CC nodes of a layer or of the ground-truth
//                  aggregate.
//   HLN_RANK_CC2   r layers: est(u) = max over layers of the penalised
//                  distance sum S + n(n - R) (Sec. 5.1: unreachable at
//                  distance n; Sec. 5.2, Algorithm 1), score = (n-1)/est
//                  (Eq. 1 on the estimate).
//   HLN_RANK_NAIVE r layers: the intersection of the layers' above-average
//                  CC-node sets (Sec. 4); only with k = -1.
//
// k >= 0: the k highest scores, ties by ascending vertex id, in rank order
// (a stable radix sort of the score keys over vertices in id order).
// k = -1: every vertex with score >= the mean (Sec. 4, "same or above
// average"), ids ascending; the mean is summed in a fixed shape --
// sequentially inside id-chunks of 1024, then sequentially over the chunk
// sums -- and divided by n, so the threshold is reproducible.
#include "hln_internal.hpp"
#include "hln_prim.hpp"

#include <algorithm>

namespace {

constexpr int kMaxLayers = 64;
constexpr int kChunk = 1024;

struct SR {
    int r;
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

__device__ __forceinline__ int64_t cc2_est(int n, const SR& L, int u) {
    int64_t best = 0;
    for (int l = 0; l < L.r; ++l) {
        const int64_t p = L.S[l][u] + static_cast<int64_t>(n) * static_cast<int64_t>(n - L.R[l][u]);
        if (l == 0 || p > best) best = p;
    }
    return best;
}

// score of every vertex and, for the top-k path, its ascending sort key
__global__ void k_scores(int mode, int n, SR L, double* score, unsigned long long* key, int32_t* val) {
    for (long long uu = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; uu < n;
         uu += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int u = static_cast<int>(uu);
        double sc;
        unsigned long long k;
        if (mode == HLN_RANK_CC2) {
            const int64_t est = cc2_est(n, L, u);
            sc = est > 0 ? static_cast<double>(n - 1) / static_cast<double>(est) : 0.0;
            k = static_cast<unsigned long long>(est);                     // smaller estimate ranks higher
        } else {
            sc = closeness_wf(n, L.S[0][u], L.R[0][u]);
            // scores are >= 0, so their bit patterns order like the values
            k = 0x7fffffffffffffffull - static_cast<unsigned long long>(__double_as_longlong(sc));
        }
        score[u] = sc;
        if (key) {
            key[u] = k;
            val[u] = u;
        }
    }
}

__global__ void k_layer_cc(int n, const int64_t* __restrict__ S, const int32_t* __restrict__ R, double* score) {
    for (long long uu = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; uu < n;
         uu += static_cast<long long>(gridDim.x) * blockDim.x)
        score[uu] = closeness_wf(n, S[uu], R[uu]);
}

// sequential sum of each id-chunk of 1024 values (one thread per chunk)
__global__ void k_chunk_sums(int n, const double* __restrict__ x, double* part) {
    const long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const long long lo = c * kChunk;
    if (lo >= n) return;
    const long long hi = lo + kChunk < n ? lo + kChunk : n;
    double s = 0.0;
    for (long long i = lo; i < hi; ++i) s += x[i];
    part[c] = s;
}

// sequential sum of the chunk sums, divided by n (one thread)
__global__ void k_mean(int n, const double* __restrict__ part, double* mean) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const long long chunks = (static_cast<long long>(n) + kChunk - 1) / kChunk;
    double t = 0.0;
    for (long long c = 0; c < chunks; ++c) t += part[c];
    *mean = n > 0 ? t / static_cast<double>(n) : 0.0;
}

// flag[u] = (score >= mean) (and, when `accumulate`, AND-ed into flag)
__global__ void k_flag_above(int n, const double* __restrict__ score, const double* __restrict__ mean, int accumulate,
                             int32_t* flag) {
    const double m = *mean;
    for (long long u = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; u < n;
         u += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int f = score[u] >= m ? 1 : 0;
        flag[u] = accumulate ? (flag[u] & f) : f;
    }
}

__global__ void k_compact(int n, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                          const double* __restrict__ score, int32_t* ids, double* out_score, int32_t* count) {
    for (long long u = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; u < n;
         u += static_cast<long long>(gridDim.x) * blockDim.x) {
        if (flag[u]) {
            ids[pos[u]] = static_cast<int32_t>(u);
            if (out_score) out_score[pos[u]] = score ? score[u] : 0.0;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = pos[n];
}

__global__ void k_take(int k, const int32_t* __restrict__ order, const double* __restrict__ score, int32_t* ids,
                       double* out_score, int32_t* count) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < k;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int u = order[i];
        ids[i] = u;
        if (out_score) out_score[i] = score[u];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = k;
}

unsigned grid_for(long long count, int block = 256) {
    return static_cast<unsigned>(std::max<long long>(1, std::min<long long>((count + block - 1) / block, 8192)));
}

int bits_of(unsigned long long x) {
    int b = 1;
    while (b < 64 && (x >> b) != 0) ++b;
    return b;
}

size_t select_ws(int n) {
    using hln::Arena;
    const size_t un = static_cast<size_t>(n) + 1;
    const long long chunks = (static_cast<long long>(n) + kChunk - 1) / kChunk + 1;
    return Arena::round(un * 8) /*score*/ + Arena::round(un * 8) /*key*/ + Arena::round(un * 4) /*val*/ +
           Arena::round(un * 4) /*flag*/ + Arena::round(un * 4) /*pos*/ + Arena::round(chunks * 8) /*part*/ +
           Arena::round(64) /*mean*/ +
           std::max(hln::prim::sort_workspace(n), hln::prim::scan_workspace(n + 1));
}

}  // namespace

extern "C" {

size_t hln_compose_cc_topk_workspace_size(int32_t n) { return n < 1 ? 0 : select_ws(n); }

hln_status hln_compose_cc_topk(int32_t mode, int32_t n, int32_t r, const int64_t* const* S, const int32_t* const* R,
                               int32_t k, int32_t* ids, double* score, int32_t* count, void* workspace,
                               size_t workspace_bytes, void* stream) {
    using hln::fail;
    hln::clear_error();
    if (mode != HLN_RANK_WF && mode != HLN_RANK_CC2 && mode != HLN_RANK_NAIVE) return fail(HLN_EINVAL, "bad mode %d", mode);
    if (n < 1) return fail(HLN_EINVAL, "n must be >= 1");
    if (r < 1 || r > kMaxLayers) return fail(HLN_EINVAL, "r must be in [1, %d]", kMaxLayers);
    if (mode == HLN_RANK_WF && r != 1) return fail(HLN_EINVAL, "HLN_RANK_WF ranks one graph (r = 1)");
    if (k < -1 || k > n) return fail(HLN_EINVAL, "k must be -1 or in [0, n] (got %d)", k);
    if (mode == HLN_RANK_NAIVE && k != -1) return fail(HLN_EINVAL, "HLN_RANK_NAIVE gives a set: k must be -1");
    if (!S || !R || !ids || !count) return fail(HLN_EINVAL, "NULL argument");
    SR L;
    L.r = r;
    for (int l = 0; l < r; ++l) {
        if (!S[l] || !R[l]) return fail(HLN_EINVAL, "layer %d arrays are NULL", l);
        L.S[l] = S[l];
        L.R[l] = R[l];
    }
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % hln::Arena::kAlign)
        return fail(HLN_EINVAL, "workspace NULL or not 256-byte aligned");
    const size_t need = select_ws(n);
    if (workspace_bytes < need) return fail(HLN_ENOMEM, "workspace too small: %zu < %zu", workspace_bytes, need);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hln::Arena ar{static_cast<char*>(workspace), workspace_bytes};
    double* sc = ar.take<double>(n + 1);
    unsigned long long* key = ar.take<unsigned long long>(n + 1);
    int32_t* val = ar.take<int32_t>(n + 1);
    int32_t* flag = ar.take<int32_t>(n + 1);
    int32_t* pos = ar.take<int32_t>(n + 1);
    const long long chunks = (static_cast<long long>(n) + kChunk - 1) / kChunk;
    double* part = ar.take<double>(chunks + 1);
    double* mean = ar.take<double>(8);
    void* sws = ar.base + ar.off;
    const size_t sws_bytes = workspace_bytes - ar.off;
    const unsigned g = grid_for(n);
    const unsigned gc = grid_for(chunks, 64);

    if (mode == HLN_RANK_NAIVE) {
        for (int l = 0; l < r; ++l) {
            hipLaunchKernelGGL(k_layer_cc, dim3(g), dim3(256), 0, st, n, L.S[l], L.R[l], sc);
            hipLaunchKernelGGL(k_chunk_sums, dim3(gc), dim3(64), 0, st, n, sc, part);
            hipLaunchKernelGGL(k_mean, dim3(1), dim3(64), 0, st, n, part, mean);
            hipLaunchKernelGGL(k_flag_above, dim3(g), dim3(256), 0, st, n, sc, mean, l > 0 ? 1 : 0, flag);
        }
        hln_status s = hln::prim::scan_exclusive<int32_t>(flag, pos, n, sws, sws_bytes, st);
        if (s != HLN_OK) return s;
        hipLaunchKernelGGL(k_compact, dim3(g), dim3(256), 0, st, n, flag, pos, static_cast<const double*>(nullptr),
                           ids, score, count);
        HLN_TRY_HIP(hipGetLastError());
        return HLN_OK;
    }

    hipLaunchKernelGGL(k_scores, dim3(g), dim3(256), 0, st, static_cast<int>(mode), n, L, sc, k >= 0 ? key : nullptr,
                       val);
    if (k >= 0) {
        // CC2 keys are estimates <= n*n; closeness keys use 63 bits
        const unsigned long long nn = static_cast<unsigned long long>(n) * static_cast<unsigned long long>(n);
        const int bits = mode == HLN_RANK_CC2 ? bits_of(nn) : 63;
        hln_status s = hln::prim::sort_pairs(key, val, n, bits, sws, sws_bytes, st);
        if (s != HLN_OK) return s;
        hipLaunchKernelGGL(k_take, dim3(grid_for(std::max(k, 1))), dim3(256), 0, st, k, val, sc, ids, score, count);
    } else {
        hipLaunchKernelGGL(k_chunk_sums, dim3(gc), dim3(64), 0, st, n, sc, part);
        hipLaunchKernelGGL(k_mean, dim3(1), dim3(64), 0, st, n, part, mean);
        hipLaunchKernelGGL(k_flag_above, dim3(g), dim3(256), 0, st, n, sc, mean, 0, flag);
        hln_status s = hln::prim::scan_exclusive<int32_t>(flag, pos, n, sws, sws_bytes, st);
        if (s != HLN_OK) return s;
        hipLaunchKernelGGL(k_compact, dim3(g), dim3(256), 0, st, n, flag, pos, sc, ids, score, count);
    }
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

}  // extern "C"
