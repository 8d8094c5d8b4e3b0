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
//   HLN_RANK_NAIVE r layers: the intersection of the layers' CC-node sets
//                  (Sec. 4): their above-average sets (k = -1) or their
//                  top-k sets (k >= 0; the intersection may hold fewer than
//                  k vertices).
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

__device__ __forceinline__ int64_t cc2_est(int n, int r, const int64_t* const* S, const int32_t* const* R, int u) {
    int64_t best = 0;
    for (int l = 0; l < r; ++l) {
        const int64_t p = S[l][u] + static_cast<int64_t>(n) * static_cast<int64_t>(n - R[l][u]);
        if (l == 0 || p > best) best = p;
    }
    return best;
}

// score of vertex u and its ascending sort key (HLN_RANK_WF or HLN_RANK_CC2)
__device__ __forceinline__ double score_key(int mode, int n, int r, const int64_t* const* S, const int32_t* const* R,
                                            int u, unsigned long long& k) {
    double sc;
    if (mode == HLN_RANK_CC2) {
        const int64_t est = cc2_est(n, r, S, R, u);
        sc = est > 0 ? static_cast<double>(n - 1) / static_cast<double>(est) : 0.0;
        k = static_cast<unsigned long long>(est);                     // smaller estimate ranks higher
    } else {
        sc = closeness_wf(n, S[0][u], R[0][u]);
        // scores are >= 0, so their bit patterns order like the values
        k = 0x7fffffffffffffffull - static_cast<unsigned long long>(__double_as_longlong(sc));
    }
    return sc;
}

// score of every vertex and, for the top-k path, its ascending sort key
__global__ void k_scores(int mode, int n, SR L, double* score, unsigned long long* key, int32_t* val) {
    for (long long uu = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; uu < n;
         uu += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int u = static_cast<int>(uu);
        unsigned long long k;
        score[u] = score_key(mode, n, L.r, L.S, L.R, u, k);
        if (key) {
            key[u] = k;
            val[u] = u;
        }
    }
}

// ------------------------------------------------------ batched top-k
// Problem p owns scores / keys [e_off[p], e_off[p+1]) (one per vertex, in id
// order), its layers' S and R pointers at sr_off in the pointer tables and
// output slots [k_off[p], k_off[p+1]) of the concatenated take.  The keys of
// all problems go through one segmented stable sort.
struct TopkDesc {
    int32_t* ids;
    double* score;
    int32_t* count;
    long long sr_off;
    int mode, n, r, k;
};

constexpr int kTopkChunk = 24;
constexpr int kPtrChunk = 96;
struct TopkChunk {
    TopkDesc d[kTopkChunk];
    long long e_off[kTopkChunk + 1], t_off[kTopkChunk + 1], k_off[kTopkChunk + 1];
    int first, count;
};
struct PtrChunk {
    const int64_t* S[kPtrChunk];
    const int32_t* R[kPtrChunk];
    long long first;
    int count;
};

__global__ void k_put_topk(TopkChunk c, TopkDesc* desc, long long* e_off, long long* t_off, long long* k_off) {
    const int i = threadIdx.x;
    if (i < c.count) desc[c.first + i] = c.d[i];
    if (i <= c.count) {
        e_off[c.first + i] = c.e_off[i];
        t_off[c.first + i] = c.t_off[i];
        k_off[c.first + i] = c.k_off[i];
    }
}

__global__ void k_put_ptrs(PtrChunk c, const int64_t** S, const int32_t** R) {
    const int i = threadIdx.x;
    if (i < c.count) {
        S[c.first + i] = c.S[i];
        R[c.first + i] = c.R[i];
    }
}

// largest p in [0, np) with off[p] <= x
__device__ __forceinline__ int problem_of(const long long* __restrict__ off, int np, long long x) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void k_bt_scores(const TopkDesc* __restrict__ desc, const long long* __restrict__ e_off, int np,
                            long long total, const int64_t* const* __restrict__ S, const int32_t* const* __restrict__ R,
                            double* score, unsigned long long* key, int32_t* val) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int p = problem_of(e_off, np, i);
        const TopkDesc D = desc[p];
        const int u = static_cast<int>(i - e_off[p]);
        unsigned long long k;
        score[i] = score_key(D.mode, D.n, D.r, S + D.sr_off, R + D.sr_off, u, k);
        key[i] = k;
        val[i] = u;
    }
}

// the first k of every problem's sorted order, and every problem's count
__global__ void k_bt_take(const TopkDesc* __restrict__ desc, const long long* __restrict__ e_off,
                          const long long* __restrict__ k_off, int np, long long total_k,
                          const int32_t* __restrict__ order, const double* __restrict__ score) {
    for (long long j = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; j < total_k;
         j += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int p = problem_of(k_off, np, j);
        const TopkDesc D = desc[p];
        const long long i = j - k_off[p];
        const int u = order[e_off[p] + i];
        D.ids[i] = u;
        if (D.score) D.score[i] = score[e_off[p] + u];
    }
    for (long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; p < np;
         p += static_cast<long long>(gridDim.x) * blockDim.x)
        *desc[p].count = desc[p].k;
}

__global__ void k_layer_cc(int n, const int64_t* __restrict__ S, const int32_t* __restrict__ R, double* score) {
    for (long long uu = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; uu < n;
         uu += static_cast<long long>(gridDim.x) * blockDim.x)
        score[uu] = closeness_wf(n, S[uu], R[uu]);
}

// sequential sum of each id-chunk of 1024 values: one wave per chunk loads
// the chunk into LDS (coalesced), then one lane adds it up in id order (the
// fixed summation shape, so the sum is the same bit for bit)
__global__ __launch_bounds__(64) void k_chunk_sums(int n, const double* __restrict__ x, double* part) {
    __shared__ double s_x[kChunk];
    const long long c = blockIdx.x;
    const long long lo = c * kChunk;
    if (lo >= n) return;
    const int len = static_cast<int>(lo + kChunk < n ? kChunk : n - lo);
    for (int i = threadIdx.x; i < len; i += blockDim.x) s_x[i] = x[lo + i];
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < len; ++i) s += s_x[i];
        part[c] = s;
    }
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

// key = value = the id, for sorting a list of ids ascending
__global__ void k_id_keys(int k, const int32_t* __restrict__ ids, unsigned long long* key, int32_t* val) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < k;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        key[i] = static_cast<unsigned long long>(static_cast<uint32_t>(ids[i]));
        val[i] = ids[i];
    }
}

__global__ void k_zero_flags(int n, int32_t* flag) {
    for (long long u = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; u < n;
         u += static_cast<long long>(gridDim.x) * blockDim.x)
        flag[u] = 0;
}

// one more layer's top-k set: flag[u] counts the layers whose top k hold u
// (`order` is the layer's ranking, a permutation, so no two threads share u)
__global__ void k_count_top(int k, const int32_t* __restrict__ order, int32_t* flag) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < k;
         i += static_cast<long long>(gridDim.x) * blockDim.x)
        flag[order[i]] += 1;
}

// flag[u] = (u is in every layer's top-k set)
__global__ void k_flag_all(int n, int r, int32_t* flag) {
    for (long long u = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; u < n;
         u += static_cast<long long>(gridDim.x) * blockDim.x)
        flag[u] = flag[u] == r ? 1 : 0;
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

struct TopkSizes {
    long long elems = 0, tiles = 0, ks = 0, ptrs = 0;
    int key_bits = 1;
};

hln_status topk_sizes(const hln_topk_problem* pr, int32_t count, TopkSizes& Z, bool check_ptrs) {
    using hln::fail;
    if (count < 0) return fail(HLN_EINVAL, "count must be >= 0");
    if (count > 0 && !pr) return fail(HLN_EINVAL, "problems is NULL");
    for (int p = 0; p < count; ++p) {
        const hln_topk_problem& q = pr[p];
        if (q.mode != HLN_RANK_WF && q.mode != HLN_RANK_CC2)
            return fail(HLN_EINVAL, "problem %d: mode must be HLN_RANK_WF or HLN_RANK_CC2", p);
        if (q.n < 1) return fail(HLN_EINVAL, "problem %d: n must be >= 1", p);
        if (q.r < 1 || q.r > kMaxLayers) return fail(HLN_EINVAL, "problem %d: r must be in [1, %d]", p, kMaxLayers);
        if (q.mode == HLN_RANK_WF && q.r != 1) return fail(HLN_EINVAL, "problem %d: HLN_RANK_WF ranks one graph", p);
        if (q.k < 0 || q.k > q.n) return fail(HLN_EINVAL, "problem %d: k must be in [0, n]", p);
        if (check_ptrs) {
            if (!q.S || !q.R || !q.ids || !q.count) return fail(HLN_EINVAL, "problem %d: NULL argument", p);
            for (int l = 0; l < q.r; ++l)
                if (!q.S[l] || !q.R[l]) return fail(HLN_EINVAL, "problem %d: layer %d arrays are NULL", p, l);
        }
        Z.elems += q.n;
        Z.tiles += hln::prim::seg_sort_tiles(q.n);
        Z.ks += q.k;
        Z.ptrs += q.r;
        const unsigned long long nn = static_cast<unsigned long long>(q.n) * static_cast<unsigned long long>(q.n);
        Z.key_bits = std::max(Z.key_bits, q.mode == HLN_RANK_CC2 ? bits_of(nn) : 63);
    }
    if (Z.elems >= (1ll << 31) - 1) return fail(HLN_EUNSUPPORTED, "batch too large (%lld vertices): split it", Z.elems);
    return HLN_OK;
}

size_t topk_ws(int32_t count, const TopkSizes& Z) {
    using hln::Arena;
    const size_t P1 = static_cast<size_t>(count) + 1;
    const size_t N = static_cast<size_t>(std::max<long long>(Z.elems, 1));
    const size_t Q = static_cast<size_t>(std::max<long long>(Z.ptrs, 1));
    return Arena::round(P1 * sizeof(TopkDesc)) + 3 * Arena::round(P1 * 8) + 2 * Arena::round(Q * 8) +
           Arena::round(N * 8) /*score*/ + 2 * Arena::round(N * 8) /*keys*/ + 2 * Arena::round(N * 4) /*vals*/ +
           hln::prim::seg_sort_workspace(Z.tiles);
}

}  // namespace

extern "C" {

size_t hln_compose_cc_topk_workspace_size(int32_t n) { return n < 1 ? 0 : select_ws(n); }

hln_status hln_compose_cc_topk(int32_t mode, int32_t n, int32_t r, const int64_t* const* S, const int32_t* const* R,
                               int32_t k, int32_t* ids, double* score, int32_t* count, void* workspace,
                               size_t workspace_bytes, void* stream) {
    using hln::fail;
    hln::clear_error();
    const bool as_set = (mode & HLN_TOPK_SET) != 0;
    mode &= ~HLN_TOPK_SET;
    if (mode != HLN_RANK_WF && mode != HLN_RANK_CC2 && mode != HLN_RANK_NAIVE) return fail(HLN_EINVAL, "bad mode %d", mode);
    if (as_set && (mode == HLN_RANK_NAIVE || k < 0))
        return fail(HLN_EINVAL, "HLN_TOPK_SET applies to the k >= 0 form of HLN_RANK_WF and HLN_RANK_CC2");
    if (n < 1) return fail(HLN_EINVAL, "n must be >= 1");
    if (r < 1 || r > kMaxLayers) return fail(HLN_EINVAL, "r must be in [1, %d]", kMaxLayers);
    if (mode == HLN_RANK_WF && r != 1) return fail(HLN_EINVAL, "HLN_RANK_WF ranks one graph (r = 1)");
    if (k < -1 || k > n) return fail(HLN_EINVAL, "k must be -1 or in [0, n] (got %d)", k);
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

    if (mode == HLN_RANK_NAIVE && k >= 0) {
        // each layer's top k by its own closeness (ties by id), counted per
        // vertex; the vertices every layer holds, ids ascending
        hipLaunchKernelGGL(k_zero_flags, dim3(g), dim3(256), 0, st, n, flag);
        for (int l = 0; l < r; ++l) {
            SR one;
            one.r = 1;
            one.S[0] = L.S[l];
            one.R[0] = L.R[l];
            hipLaunchKernelGGL(k_scores, dim3(g), dim3(256), 0, st, static_cast<int>(HLN_RANK_WF), n, one, sc, key,
                               val);
            hln_status s = hln::prim::sort_pairs(key, val, n, 63, sws, sws_bytes, st);
            if (s != HLN_OK) return s;
            if (k > 0) hipLaunchKernelGGL(k_count_top, dim3(grid_for(k)), dim3(256), 0, st, k, val, flag);
        }
        hipLaunchKernelGGL(k_flag_all, dim3(g), dim3(256), 0, st, n, r, flag);
        hln_status s = hln::prim::scan_exclusive<int32_t>(flag, pos, n, sws, sws_bytes, st);
        if (s != HLN_OK) return s;
        hipLaunchKernelGGL(k_compact, dim3(g), dim3(256), 0, st, n, flag, pos, static_cast<const double*>(nullptr),
                           ids, score, count);
        HLN_TRY_HIP(hipGetLastError());
        return HLN_OK;
    }
    if (mode == HLN_RANK_NAIVE) {
        for (int l = 0; l < r; ++l) {
            hipLaunchKernelGGL(k_layer_cc, dim3(g), dim3(256), 0, st, n, L.S[l], L.R[l], sc);
            hipLaunchKernelGGL(k_chunk_sums, dim3(static_cast<unsigned>(chunks)), dim3(64), 0, st, n, sc, part);
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
        if (as_set && k > 1) {
            // the same k vertices in ascending id order, with their scores
            hipLaunchKernelGGL(k_id_keys, dim3(grid_for(k)), dim3(256), 0, st, k, ids, key, val);
            s = hln::prim::sort_pairs(key, val, k, bits_of(static_cast<unsigned long long>(n - 1)), sws, sws_bytes, st);
            if (s != HLN_OK) return s;
            hipLaunchKernelGGL(k_take, dim3(grid_for(k)), dim3(256), 0, st, k, val, sc, ids, score, count);
        }
    } else {
        hipLaunchKernelGGL(k_chunk_sums, dim3(static_cast<unsigned>(chunks)), dim3(64), 0, st, n, sc, part);
        hipLaunchKernelGGL(k_mean, dim3(1), dim3(64), 0, st, n, part, mean);
        hipLaunchKernelGGL(k_flag_above, dim3(g), dim3(256), 0, st, n, sc, mean, 0, flag);
        hln_status s = hln::prim::scan_exclusive<int32_t>(flag, pos, n, sws, sws_bytes, st);
        if (s != HLN_OK) return s;
        hipLaunchKernelGGL(k_compact, dim3(g), dim3(256), 0, st, n, flag, pos, sc, ids, score, count);
    }
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

size_t hln_compose_cc_topk_batch_workspace_size(const hln_topk_problem* problems, int32_t count) {
    TopkSizes Z;
    if (topk_sizes(problems, count, Z, false) != HLN_OK) return 0;
    return topk_ws(count, Z);
}

hln_status hln_compose_cc_topk_batch(const hln_topk_problem* problems, int32_t count, void* workspace,
                                     size_t workspace_bytes, void* stream) {
    using hln::fail;
    hln::clear_error();
    TopkSizes Z;
    hln_status s = topk_sizes(problems, count, Z, true);
    if (s != HLN_OK) return s;
    if (count == 0) return HLN_OK;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % hln::Arena::kAlign)
        return fail(HLN_EINVAL, "workspace NULL or not 256-byte aligned");
    const size_t need = topk_ws(count, Z);
    if (workspace_bytes < need) return fail(HLN_ENOMEM, "workspace too small: %zu < %zu", workspace_bytes, need);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long N = std::max<long long>(Z.elems, 1);
    hln::Arena ar{static_cast<char*>(workspace), workspace_bytes};
    TopkDesc* desc = ar.take<TopkDesc>(count + 1);
    long long* e_off = ar.take<long long>(count + 1);
    long long* t_off = ar.take<long long>(count + 1);
    long long* k_off = ar.take<long long>(count + 1);
    const int64_t** Sp = ar.take<const int64_t*>(std::max<long long>(Z.ptrs, 1));
    const int32_t** Rp = ar.take<const int32_t*>(std::max<long long>(Z.ptrs, 1));
    double* sc = ar.take<double>(N);
    unsigned long long* key = ar.take<unsigned long long>(N);
    unsigned long long* kalt = ar.take<unsigned long long>(N);
    int32_t* val = ar.take<int32_t>(N);
    int32_t* valt = ar.take<int32_t>(N);
    void* sws = ar.base + ar.off;
    const size_t sws_bytes = workspace_bytes - ar.off;

    long long eo = 0, to = 0, ko = 0, so = 0;
    for (int first = 0; first < count; first += kTopkChunk) {
        TopkChunk c{};
        c.first = first;
        c.count = std::min(kTopkChunk, count - first);
        for (int i = 0; i <= c.count; ++i) {
            c.e_off[i] = eo;
            c.t_off[i] = to;
            c.k_off[i] = ko;
            if (i == c.count) break;
            const hln_topk_problem& q = problems[first + i];
            c.d[i] = TopkDesc{q.ids, q.score, q.count, so, q.mode, q.n, q.r, q.k};
            eo += q.n;
            to += hln::prim::seg_sort_tiles(q.n);
            ko += q.k;
            so += q.r;
        }
        hipLaunchKernelGGL(k_put_topk, dim3(1), dim3(64), 0, st, c, desc, e_off, t_off, k_off);
    }
    {
        PtrChunk c{};
        c.first = 0;
        c.count = 0;
        for (int p = 0; p < count; ++p)
            for (int l = 0; l < problems[p].r; ++l) {
                c.S[c.count] = problems[p].S[l];
                c.R[c.count] = problems[p].R[l];
                if (++c.count == kPtrChunk) {
                    hipLaunchKernelGGL(k_put_ptrs, dim3(1), dim3(128), 0, st, c, Sp, Rp);
                    c.first += c.count;
                    c.count = 0;
                }
            }
        if (c.count) hipLaunchKernelGGL(k_put_ptrs, dim3(1), dim3(128), 0, st, c, Sp, Rp);
    }
    HLN_TRY_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_bt_scores, dim3(grid_for(Z.elems)), dim3(256), 0, st, desc, e_off, count, Z.elems, Sp, Rp,
                       sc, key, val);
    bool in_alt = false;
    s = hln::prim::sort_segmented(key, kalt, val, valt, e_off, t_off, count, Z.tiles, Z.key_bits, sws, sws_bytes, st,
                                  &in_alt);
    if (s != HLN_OK) return s;
    hipLaunchKernelGGL(k_bt_take, dim3(grid_for(std::max<long long>(Z.ks, count))), dim3(256), 0, st, desc, e_off,
                       k_off, count, Z.ks, in_alt ? valt : val, sc);
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

}  // extern "C"
