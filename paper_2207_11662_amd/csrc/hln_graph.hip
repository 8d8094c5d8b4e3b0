// Layer ingest, CSR validation and Boolean AND / OR aggregation.
//
// Ingest (Sec. 1: simple undirected layers over one vertex set): every edge
// becomes the two arcs u->v and v->u keyed u*n+v, the keys are radix sorted,
// self-loops and repeated keys are dropped, and the surviving keys are the
// CSR (rows sorted by construction).
//
// Aggregation (Sec. 3.1): AND keeps an edge present in every selected
// layer, OR one present in at least one.  Both work arc-parallel with
// binary searches in the other layers' sorted rows, then compact with an
// exclusive scan, so output rows come out sorted and the result does not
// depend on scheduling.
#include "hln_internal.hpp"
#include "hln_prim.hpp"

#include <algorithm>

namespace {

constexpr int kMaxLayers = 64;

struct LayerSet {
    int r;
    int n;
    const int32_t* rp[kMaxLayers];
    const int32_t* ci[kMaxLayers];
    long long base[kMaxLayers + 1];     // prefix of nnz over layers
};

__device__ __forceinline__ int row_of(const int32_t* __restrict__ rp, int n, long long e) {
    // last u with rp[u] <= e
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rp[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// first position p in [lo, hi) with ci[p] >= x
__device__ __forceinline__ int lower_bound(const int32_t* __restrict__ ci, int lo, int hi, int x) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ci[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool in_row(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci, int u, int x) {
    const int lo = rp[u], hi = rp[u + 1];
    const int p = lower_bound(ci, lo, hi, x);
    return p < hi && ci[p] == x;
}

// ------------------------------------------------------------------ ingest

__global__ void k_ingest_keys(int n, long long m, const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                              unsigned long long* keys, int32_t* vals, unsigned long long drop, int* fault) {
    const unsigned long long N = static_cast<unsigned long long>(n);
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < m;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int u = eu[i], v = ev[i];
        unsigned long long k0 = drop, k1 = drop;
        if (static_cast<unsigned>(u) >= static_cast<unsigned>(n) || static_cast<unsigned>(v) >= static_cast<unsigned>(n)) {
            hln::dev::store_agent_i32(fault, 2);
        } else if (u != v) {
            k0 = static_cast<unsigned long long>(u) * N + static_cast<unsigned long long>(v);
            k1 = static_cast<unsigned long long>(v) * N + static_cast<unsigned long long>(u);
        }
        keys[2 * i] = k0;
        keys[2 * i + 1] = k1;
        vals[2 * i] = 0;
        vals[2 * i + 1] = 0;
    }
}

__global__ void k_ingest_mark(const unsigned long long* __restrict__ keys, long long count, unsigned long long drop,
                              int32_t* flag) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        const unsigned long long k = keys[i];
        flag[i] = (k < drop && (i == 0 || keys[i - 1] != k)) ? 1 : 0;
    }
}

__global__ void k_zero_i32(int32_t* p, long long count) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += static_cast<long long>(gridDim.x) * blockDim.x)
        p[i] = 0;
}

__global__ void k_ingest_fill(int n, const unsigned long long* __restrict__ keys, long long count,
                              const int32_t* __restrict__ flag, const int32_t* __restrict__ pos, int32_t* col_idx,
                              int32_t* deg) {
    const unsigned long long N = static_cast<unsigned long long>(n);
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        if (!flag[i]) continue;
        const unsigned long long k = keys[i];
        col_idx[pos[i]] = static_cast<int32_t>(k % N);
        atomicAdd(&deg[k / N], 1);
    }
}

// ---------------------------------------------------------- batched ingest
// Many edge lists in one set of launches: list s owns edges [k_off[s]/2,
// k_off[s+1]/2) of the concatenation, keys [k_off[s], k_off[s+1]) and
// degree counters [d_off[s], d_off[s+1]) (n + 1 of them).  Keys of every
// list are sorted at once as segments; flags and degrees are scanned over
// the concatenation and each list subtracts the value at its own start.

struct IngestList {
    const int32_t* eu;
    const int32_t* ev;
    int32_t* row_ptr;
    int32_t* col_idx;
    int n;
};

// The list table and its offset arrays are written from kernel arguments
// (no host staging, so the call can be captured), kPutChunk lists a launch.
constexpr int kPutChunk = 24;
struct PutChunk {
    IngestList l[kPutChunk];
    long long k_off[kPutChunk + 1], d_off[kPutChunk + 1], t_off[kPutChunk + 1];
    int first, count;
};

__global__ void k_put_lists(PutChunk c, IngestList* lists, long long* k_off, long long* d_off, long long* t_off) {
    const int i = threadIdx.x;
    if (i < c.count) lists[c.first + i] = c.l[i];
    if (i <= c.count) {
        k_off[c.first + i] = c.k_off[i];
        d_off[c.first + i] = c.d_off[i];
        t_off[c.first + i] = c.t_off[i];
    }
}

// largest s in [0, nseg) with off[s] <= x
__device__ __forceinline__ int list_of(const long long* __restrict__ off, int nseg, long long x) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void k_bi_keys(const IngestList* __restrict__ lists, const long long* __restrict__ k_off, int nl,
                          long long edges, unsigned long long* keys, int* fault) {
    for (long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; e < edges;
         e += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int s = list_of(k_off, nl, 2 * e);
        const IngestList L = lists[s];
        const long long i = e - k_off[s] / 2;
        const unsigned long long N = static_cast<unsigned long long>(L.n);
        const int u = L.eu[i], v = L.ev[i];
        unsigned long long k0 = N * N, k1 = N * N;
        if (static_cast<unsigned>(u) >= static_cast<unsigned>(L.n) || static_cast<unsigned>(v) >= static_cast<unsigned>(L.n)) {
            hln::dev::store_agent_i32(fault, 2);
        } else if (u != v) {
            k0 = static_cast<unsigned long long>(u) * N + static_cast<unsigned long long>(v);
            k1 = static_cast<unsigned long long>(v) * N + static_cast<unsigned long long>(u);
        }
        keys[2 * e] = k0;
        keys[2 * e + 1] = k1;
    }
}

__global__ void k_bi_mark(const IngestList* __restrict__ lists, const long long* __restrict__ k_off, int nl,
                          const unsigned long long* __restrict__ keys, long long count, int32_t* flag) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int s = list_of(k_off, nl, i);
        const unsigned long long N = static_cast<unsigned long long>(lists[s].n);
        const unsigned long long k = keys[i];
        flag[i] = (k < N * N && (i == k_off[s] || keys[i - 1] != k)) ? 1 : 0;
    }
}

__global__ void k_bi_fill(const IngestList* __restrict__ lists, const long long* __restrict__ k_off,
                          const long long* __restrict__ d_off, int nl, const unsigned long long* __restrict__ keys,
                          long long count, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                          int32_t* deg) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        if (!flag[i]) continue;
        const int s = list_of(k_off, nl, i);
        const IngestList L = lists[s];
        const unsigned long long N = static_cast<unsigned long long>(L.n);
        const unsigned long long k = keys[i];
        L.col_idx[pos[i] - pos[k_off[s]]] = static_cast<int32_t>(k % N);
        atomicAdd(&deg[d_off[s] + static_cast<long long>(k / N)], 1);
    }
}

__global__ void k_bi_rowptr(const IngestList* __restrict__ lists, const long long* __restrict__ d_off, int nl,
                            long long count, const int32_t* __restrict__ dscan) {
    for (long long j = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; j < count;
         j += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int s = list_of(d_off, nl, j);
        lists[s].row_ptr[j - d_off[s]] = dscan[j] - dscan[d_off[s]];
    }
}

// ---------------------------------------------------------------- validate

__global__ void k_validate(int n, long long nnz, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           int32_t* result) {
    int bits = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && (rp[0] != 0 || rp[n] != nnz)) bits |= 1;
    for (long long uu = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; uu < n;
         uu += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int u = static_cast<int>(uu);
        const int lo = rp[u], hi = rp[u + 1];
        if (lo < 0 || hi < lo || hi > nnz) {
            bits |= 1;
            continue;
        }
        int prev = -1;
        for (int e = lo; e < hi; ++e) {
            const int v = ci[e];
            if (static_cast<unsigned>(v) >= static_cast<unsigned>(n)) {
                bits |= 2;
                continue;
            }
            if (v <= prev) bits |= 4;
            if (v == u) bits |= 8;
            prev = v;
            const int vlo = rp[v], vhi = rp[v + 1];
            if (vlo < 0 || vhi < vlo || vhi > nnz) {
                bits |= 1;
                continue;
            }
            const int p = lower_bound(ci, vlo, vhi, u);
            if (!(p < vhi && ci[p] == u)) bits |= 16;
        }
    }
    if (bits) atomicOr(result, bits);
}

// --------------------------------------------------------------- aggregate

__global__ void k_and_mark(LayerSet L, int p, int32_t* flag) {
    const long long nnz = L.base[p + 1] - L.base[p];
    for (long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; e < nnz;
         e += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int u = row_of(L.rp[p], L.n, e);
        const int x = L.ci[p][e];
        int keep = 1;
        for (int l = 0; l < L.r && keep; ++l)
            if (l != p && !in_row(L.rp[l], L.ci[l], u, x)) keep = 0;
        flag[e] = keep;
    }
}

__global__ void k_and_fill(LayerSet L, int p, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                           int32_t* out_rp, int32_t* out_ci) {
    const long long nnz = L.base[p + 1] - L.base[p];
    const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
    const long long t0 = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (long long e = t0; e < nnz; e += stride)
        if (flag[e]) out_ci[pos[e]] = L.ci[p][e];
    for (long long u = t0; u <= L.n; u += stride) out_rp[u] = pos[L.rp[p][u]];
}

// ------------------------------------------------------- batched AND
// Problem q keeps the arcs of its pivot layer (the one with the fewest arcs)
// that every other layer of q holds.  Its pivot arcs are [e_off[q],
// e_off[q+1]) of the concatenation and its row pointers [r_off[q],
// r_off[q+1]) (n + 1 of them); its layers are lay[l_off .. l_off + r).
struct AndProblem {
    int32_t* out_rp;
    int32_t* out_ci;
    long long l_off;
    int n, r, p;
};
struct LayerPtrs {
    const int32_t* rp;
    const int32_t* ci;
};

constexpr int kAndChunk = 24;
constexpr int kLayChunk = 96;
struct AndChunk {
    AndProblem q[kAndChunk];
    long long e_off[kAndChunk + 1], r_off[kAndChunk + 1];
    int first, count;
};
struct LayChunk {
    LayerPtrs l[kLayChunk];
    long long first;
    int count;
};

__global__ void k_put_and(AndChunk c, AndProblem* probs, long long* e_off, long long* r_off) {
    const int i = threadIdx.x;
    if (i < c.count) probs[c.first + i] = c.q[i];
    if (i <= c.count) {
        e_off[c.first + i] = c.e_off[i];
        r_off[c.first + i] = c.r_off[i];
    }
}

__global__ void k_put_lay(LayChunk c, LayerPtrs* lay) {
    const int i = threadIdx.x;
    if (i < c.count) lay[c.first + i] = c.l[i];
}

__global__ void k_ba_mark(const AndProblem* __restrict__ probs, const LayerPtrs* __restrict__ lay,
                          const long long* __restrict__ e_off, int np, long long total, int32_t* flag) {
    for (long long g = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int q = list_of(e_off, np, g);
        const AndProblem Q = probs[q];
        const long long e = g - e_off[q];
        const LayerPtrs P = lay[Q.l_off + Q.p];
        const int u = row_of(P.rp, Q.n, e);
        const int x = P.ci[e];
        int keep = 1;
        for (int l = 0; l < Q.r && keep; ++l) {
            const LayerPtrs O = lay[Q.l_off + l];
            if (l != Q.p && !in_row(O.rp, O.ci, u, x)) keep = 0;
        }
        flag[g] = keep;
    }
}

__global__ void k_ba_fill(const AndProblem* __restrict__ probs, const LayerPtrs* __restrict__ lay,
                          const long long* __restrict__ e_off, const long long* __restrict__ r_off, int np,
                          long long total, long long total_rows, const int32_t* __restrict__ flag,
                          const int32_t* __restrict__ pos) {
    const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
    const long long t0 = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (long long g = t0; g < total; g += stride)
        if (flag[g]) {
            const int q = list_of(e_off, np, g);
            const AndProblem Q = probs[q];
            Q.out_ci[pos[g] - pos[e_off[q]]] = lay[Q.l_off + Q.p].ci[g - e_off[q]];
        }
    for (long long j = t0; j < total_rows; j += stride) {
        const int q = list_of(r_off, np, j);
        const AndProblem Q = probs[q];
        const long long u = j - r_off[q];
        Q.out_rp[u] = pos[e_off[q] + lay[Q.l_off + Q.p].rp[u]] - pos[e_off[q]];
    }
}

__global__ void k_or_mark(LayerSet L, int32_t* keep) {
    const long long total = L.base[L.r];
    for (long long g = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<long long>(gridDim.x) * blockDim.x) {
        int l = 0;
        while (L.base[l + 1] <= g) ++l;
        const long long e = g - L.base[l];
        const int u = row_of(L.rp[l], L.n, e);
        const int x = L.ci[l][e];
        int k = 1;
        for (int q = 0; q < l && k; ++q)
            if (in_row(L.rp[q], L.ci[q], u, x)) k = 0;      // first layer holding the edge keeps it
        keep[g] = k;
    }
}

__global__ void k_or_count(LayerSet L, const int32_t* __restrict__ kpos, int32_t* cnt) {
    for (long long uu = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; uu < L.n;
         uu += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int u = static_cast<int>(uu);
        int c = 0;
        for (int l = 0; l < L.r; ++l) c += kpos[L.base[l] + L.rp[l][u + 1]] - kpos[L.base[l] + L.rp[l][u]];
        cnt[u] = c;
    }
}

__global__ void k_or_fill(LayerSet L, const int32_t* __restrict__ keep, const int32_t* __restrict__ kpos,
                          const int32_t* __restrict__ out_rp, int32_t* out_ci) {
    const long long total = L.base[L.r];
    for (long long g = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<long long>(gridDim.x) * blockDim.x) {
        if (!keep[g]) continue;
        int l = 0;
        while (L.base[l + 1] <= g) ++l;
        const long long e = g - L.base[l];
        const int u = row_of(L.rp[l], L.n, e);
        const int x = L.ci[l][e];
        // rank of x among the union's elements of row u: kept elements < x
        int rank = 0;
        for (int q = 0; q < L.r; ++q) {
            const int lo = L.rp[q][u], hi = L.rp[q][u + 1];
            const int at = (q == l) ? static_cast<int>(e) : lower_bound(L.ci[q], lo, hi, x);
            rank += kpos[L.base[q] + at] - kpos[L.base[q] + lo];
        }
        out_ci[out_rp[u] + rank] = x;
    }
}

unsigned grid_for(long long count, int block = 256) {
    return static_cast<unsigned>(std::max<long long>(1, std::min<long long>((count + block - 1) / block, 8192)));
}

int key_bits_for(int n) {
    // keys u*n+v < n*n, plus the drop sentinel n*n
    const unsigned long long top = static_cast<unsigned long long>(n) * static_cast<unsigned long long>(n);
    int b = 1;
    while (b < 64 && (top >> b) != 0) ++b;
    return b;
}

hln_status check_layers(const hln_csr* layers, int32_t r, LayerSet& L) {
    using hln::fail;
    if (!layers) return fail(HLN_EINVAL, "layers is NULL");
    if (r < 1 || r > kMaxLayers) return fail(HLN_EINVAL, "r must be in [1, %d] (got %d)", kMaxLayers, r);
    L.r = r;
    L.n = layers[0].n;
    L.base[0] = 0;
    if (L.n < 1) return fail(HLN_EINVAL, "n must be >= 1");
    for (int l = 0; l < r; ++l) {
        if (layers[l].n != L.n) return fail(HLN_EINVAL, "layer %d has n=%d, layer 0 has n=%d", l, layers[l].n, L.n);
        if (!layers[l].row_ptr || (layers[l].nnz > 0 && !layers[l].col_idx))
            return fail(HLN_EINVAL, "layer %d arrays are NULL", l);
        if (layers[l].nnz < 0) return fail(HLN_EINVAL, "layer %d nnz < 0", l);
        L.rp[l] = layers[l].row_ptr;
        L.ci[l] = layers[l].col_idx;
        L.base[l + 1] = L.base[l] + layers[l].nnz;
    }
    if (L.base[r] >= (1ll << 31)) return fail(HLN_EUNSUPPORTED, "total arcs exceed 2^31");
    return HLN_OK;
}

// Sizes of a batched ingest; HLN_OK with the totals, else the argument error.
struct BatchSizes {
    long long edges = 0, keys = 0, degs = 0, tiles = 0;
    int key_bits = 1;
};

hln_status batch_sizes(const hln_edge_list* lists, int32_t count, BatchSizes& B, bool check_ptrs) {
    using hln::fail;
    if (count < 0) return fail(HLN_EINVAL, "count must be >= 0");
    if (count > 0 && !lists) return fail(HLN_EINVAL, "lists is NULL");
    for (int s = 0; s < count; ++s) {
        const hln_edge_list& l = lists[s];
        if (l.n < 1) return fail(HLN_EINVAL, "list %d: n must be >= 1", s);
        if (l.m < 0 || l.m > (1ll << 30)) return fail(HLN_EINVAL, "list %d: m out of range", s);
        if (check_ptrs && (!l.row_ptr || (l.m > 0 && (!l.eu || !l.ev || !l.col_idx))))
            return fail(HLN_EINVAL, "list %d: NULL array", s);
        B.edges += l.m;
        B.degs += static_cast<long long>(l.n) + 1;
        B.tiles += hln::prim::seg_sort_tiles(2 * l.m);
        if (l.m > 0) B.key_bits = std::max(B.key_bits, key_bits_for(l.n));
    }
    B.keys = 2 * B.edges;
    if (B.keys >= (1ll << 31) - 1 || B.degs >= (1ll << 31) - 1)
        return fail(HLN_EUNSUPPORTED, "batch too large (arcs %lld, vertices %lld): split it", B.keys, B.degs);
    return HLN_OK;
}

size_t batch_workspace(int32_t count, const BatchSizes& B) {
    using hln::Arena;
    const long long a = std::max<long long>(B.keys, 1);
    const size_t L1 = static_cast<size_t>(count) + 1;
    return Arena::round(L1 * sizeof(IngestList)) + 3 * Arena::round(L1 * 8) + 2 * Arena::round(static_cast<size_t>(a) * 8) +
           2 * Arena::round(static_cast<size_t>(a + 1) * 4) + 2 * Arena::round(static_cast<size_t>(B.degs + 1) * 4) +
           std::max(hln::prim::seg_sort_workspace(B.tiles),
                    hln::prim::scan_workspace(std::max(a, B.degs) + 1));
}

}  // namespace

extern "C" {

size_t hln_csr_from_edges_workspace_size(int32_t n, int64_t m) {
    (void)n;
    if (m < 0) return 0;
    const long long a = 2 * m;
    using hln::Arena;
    return Arena::round(static_cast<size_t>(a + 1) * 8) + Arena::round(static_cast<size_t>(a + 1) * 4) +
           Arena::round(static_cast<size_t>(a + 1) * 4) + Arena::round(static_cast<size_t>(a + 1) * 4) +
           Arena::round(static_cast<size_t>(n + 1) * 4) +
           std::max(hln::prim::sort_workspace(a), hln::prim::scan_workspace(std::max<long long>(a, n) + 1));
}

hln_status hln_csr_from_edges(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev, int32_t* row_ptr,
                              int32_t* col_idx, void* workspace, size_t workspace_bytes, void* stream) {
    using hln::fail;
    hln::clear_error();
    if (n < 1) return fail(HLN_EINVAL, "n must be >= 1");
    if (m < 0 || m > (1ll << 30)) return fail(HLN_EINVAL, "m out of range");
    if (!row_ptr || (m > 0 && (!eu || !ev || !col_idx))) return fail(HLN_EINVAL, "NULL array");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % hln::Arena::kAlign)
        return fail(HLN_EINVAL, "workspace NULL or not 256-byte aligned");
    const size_t need = hln_csr_from_edges_workspace_size(n, m);
    if (workspace_bytes < need) return fail(HLN_ENOMEM, "workspace too small: %zu < %zu", workspace_bytes, need);
    int* fault = hln::fault_word();
    if (!fault) return HLN_EDEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long a = 2 * m;
    hln::Arena ar{static_cast<char*>(workspace), workspace_bytes};
    unsigned long long* keys = ar.take<unsigned long long>(a + 1);
    int32_t* vals = ar.take<int32_t>(a + 1);
    int32_t* flag = ar.take<int32_t>(a + 1);
    int32_t* pos = ar.take<int32_t>(a + 1);
    int32_t* deg = ar.take<int32_t>(n + 1);
    void* sws = ar.base + ar.off;
    const size_t sws_bytes = workspace_bytes - ar.off;
    const unsigned long long drop = static_cast<unsigned long long>(n) * static_cast<unsigned long long>(n);
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(n + 1)), dim3(256), 0, st, deg, static_cast<long long>(n + 1));
    if (m > 0) {
        hipLaunchKernelGGL(k_ingest_keys, dim3(grid_for(m)), dim3(256), 0, st, n, static_cast<long long>(m), eu, ev,
                           keys, vals, drop, fault);
        hln_status s = hln::prim::sort_pairs(keys, vals, a, key_bits_for(n), sws, sws_bytes, st);
        if (s != HLN_OK) return s;
        hipLaunchKernelGGL(k_ingest_mark, dim3(grid_for(a)), dim3(256), 0, st, keys, a, drop, flag);
        s = hln::prim::scan_exclusive<int32_t>(flag, pos, a, sws, sws_bytes, st);
        if (s != HLN_OK) return s;
        hipLaunchKernelGGL(k_ingest_fill, dim3(grid_for(a)), dim3(256), 0, st, n, keys, a, flag, pos, col_idx, deg);
    }
    hln_status s = hln::prim::scan_exclusive<int32_t>(deg, row_ptr, n, sws, sws_bytes, st);
    if (s != HLN_OK) return s;
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

size_t hln_csr_from_edges_batch_workspace_size(const hln_edge_list* lists, int32_t count) {
    BatchSizes B;
    if (batch_sizes(lists, count, B, false) != HLN_OK) return 0;
    return batch_workspace(count, B);
}

hln_status hln_csr_from_edges_batch(const hln_edge_list* lists, int32_t count, void* workspace,
                                    size_t workspace_bytes, void* stream) {
    using hln::fail;
    hln::clear_error();
    BatchSizes B;
    hln_status s = batch_sizes(lists, count, B, true);
    if (s != HLN_OK) return s;
    if (count == 0) return HLN_OK;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % hln::Arena::kAlign)
        return fail(HLN_EINVAL, "workspace NULL or not 256-byte aligned");
    const size_t need = batch_workspace(count, B);
    if (workspace_bytes < need) return fail(HLN_ENOMEM, "workspace too small: %zu < %zu", workspace_bytes, need);
    int* fault = hln::fault_word();
    if (!fault) return HLN_EDEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long a = std::max<long long>(B.keys, 1);
    hln::Arena ar{static_cast<char*>(workspace), workspace_bytes};
    IngestList* tab = ar.take<IngestList>(count + 1);
    long long* k_off = ar.take<long long>(count + 1);
    long long* d_off = ar.take<long long>(count + 1);
    long long* t_off = ar.take<long long>(count + 1);
    unsigned long long* keys = ar.take<unsigned long long>(a);
    unsigned long long* alt = ar.take<unsigned long long>(a);
    int32_t* flag = ar.take<int32_t>(a + 1);
    int32_t* pos = ar.take<int32_t>(a + 1);
    int32_t* deg = ar.take<int32_t>(B.degs + 1);
    int32_t* dscan = ar.take<int32_t>(B.degs + 1);
    void* sws = ar.base + ar.off;
    const size_t sws_bytes = workspace_bytes - ar.off;

    long long ko = 0, dof = 0, to = 0;
    for (int first = 0; first < count; first += kPutChunk) {
        PutChunk c{};
        c.first = first;
        c.count = std::min(kPutChunk, count - first);
        for (int i = 0; i <= c.count; ++i) {
            c.k_off[i] = ko;
            c.d_off[i] = dof;
            c.t_off[i] = to;
            if (i == c.count) break;
            const hln_edge_list& l = lists[first + i];
            c.l[i] = IngestList{l.eu, l.ev, l.row_ptr, l.col_idx, l.n};
            ko += 2 * l.m;
            dof += static_cast<long long>(l.n) + 1;
            to += hln::prim::seg_sort_tiles(2 * l.m);
        }
        hipLaunchKernelGGL(k_put_lists, dim3(1), dim3(64), 0, st, c, tab, k_off, d_off, t_off);
    }
    HLN_TRY_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(B.degs)), dim3(256), 0, st, deg, B.degs);
    const unsigned long long* sorted = keys;
    if (B.edges > 0) {
        hipLaunchKernelGGL(k_bi_keys, dim3(grid_for(B.edges)), dim3(256), 0, st, tab, k_off, count, B.edges, keys,
                           fault);
        bool in_alt = false;
        s = hln::prim::sort_segmented(keys, alt, nullptr, nullptr, k_off, t_off, count, B.tiles, B.key_bits, sws,
                                      sws_bytes, st, &in_alt);
        if (s != HLN_OK) return s;
        sorted = in_alt ? alt : keys;
        hipLaunchKernelGGL(k_bi_mark, dim3(grid_for(B.keys)), dim3(256), 0, st, tab, k_off, count, sorted, B.keys,
                           flag);
        s = hln::prim::scan_exclusive<int32_t>(flag, pos, B.keys, sws, sws_bytes, st);
        if (s != HLN_OK) return s;
        hipLaunchKernelGGL(k_bi_fill, dim3(grid_for(B.keys)), dim3(256), 0, st, tab, k_off, d_off, count, sorted,
                           B.keys, flag, pos, deg);
    }
    s = hln::prim::scan_exclusive<int32_t>(deg, dscan, B.degs, sws, sws_bytes, st);
    if (s != HLN_OK) return s;
    hipLaunchKernelGGL(k_bi_rowptr, dim3(grid_for(B.degs)), dim3(256), 0, st, tab, d_off, count, B.degs, dscan);
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

hln_status hln_csr_validate(const hln_csr* g, int32_t* result, void* stream) {
    using hln::fail;
    hln::clear_error();
    if (!g || !result) return fail(HLN_EINVAL, "NULL argument");
    if (g->n < 1 || g->nnz < 0 || !g->row_ptr || (g->nnz > 0 && !g->col_idx))
        return fail(HLN_EINVAL, "bad graph descriptor");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, result, 1ll);
    hipLaunchKernelGGL(k_validate, dim3(grid_for(g->n)), dim3(256), 0, st, g->n, static_cast<long long>(g->nnz),
                       g->row_ptr, g->col_idx, result);
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

}  // extern "C"

namespace {

struct AndSizes {
    long long arcs = 0, rows = 0, layers = 0;
};

hln_status and_sizes(const hln_and_problem* pr, int32_t count, AndSizes& Z, bool check_ptrs) {
    using hln::fail;
    if (count < 0) return fail(HLN_EINVAL, "count must be >= 0");
    if (count > 0 && !pr) return fail(HLN_EINVAL, "problems is NULL");
    for (int q = 0; q < count; ++q) {
        const hln_and_problem& P = pr[q];
        if (!P.layers) return fail(HLN_EINVAL, "problem %d: layers is NULL", q);
        LayerSet L;
        const hln_status s = check_layers(P.layers, P.r, L);
        if (s != HLN_OK) {
            char why[200];
            snprintf(why, sizeof why, "%s", hln_last_error());
            return fail(s, "problem %d: %s", q, why);
        }
        int p = 0;
        for (int l = 0; l < P.r; ++l)
            if (P.layers[l].nnz < P.layers[p].nnz) p = l;
        if (check_ptrs) {
            if (!P.out_row_ptr || (P.capacity > 0 && !P.out_col_idx)) return fail(HLN_EINVAL, "problem %d: NULL output", q);
            if (P.capacity < P.layers[p].nnz)
                return fail(HLN_ENOMEM, "problem %d: output capacity %lld < bound %lld", q,
                            static_cast<long long>(P.capacity), static_cast<long long>(P.layers[p].nnz));
        }
        Z.arcs += P.layers[p].nnz;
        Z.rows += static_cast<long long>(L.n) + 1;
        Z.layers += P.r;
    }
    if (Z.arcs >= (1ll << 31) - 1 || Z.rows >= (1ll << 31) - 1)
        return fail(HLN_EUNSUPPORTED, "batch too large (pivot arcs %lld, rows %lld): split it", Z.arcs, Z.rows);
    return HLN_OK;
}

size_t and_ws(int32_t count, const AndSizes& Z) {
    using hln::Arena;
    const size_t P1 = static_cast<size_t>(count) + 1;
    return Arena::round(P1 * sizeof(AndProblem)) + 2 * Arena::round(P1 * 8) +
           Arena::round(static_cast<size_t>(std::max<long long>(Z.layers, 1)) * sizeof(LayerPtrs)) +
           2 * Arena::round(static_cast<size_t>(Z.arcs + 1) * 4) + hln::prim::scan_workspace(Z.arcs + 1);
}

size_t compose_ws(const LayerSet& L) {
    using hln::Arena;
    const long long total = L.base[L.r];
    return Arena::round(static_cast<size_t>(total + 1) * 4) * 2 + Arena::round(static_cast<size_t>(L.n + 1) * 4) +
           hln::prim::scan_workspace(std::max<long long>(total, L.n) + 1);
}

hln_status compose(int mode, const hln_csr* layers, int32_t r, int32_t* out_rp, int32_t* out_ci, int64_t capacity,
                   void* workspace, size_t workspace_bytes, void* stream) {
    using hln::fail;
    hln::clear_error();
    LayerSet L;
    hln_status s = check_layers(layers, r, L);
    if (s != HLN_OK) return s;
    if (!out_rp || (capacity > 0 && !out_ci)) return fail(HLN_EINVAL, "NULL output");
    long long bound = 0;
    int p = 0;
    if (mode == 0) {
        for (int l = 0; l < r; ++l)
            if (layers[l].nnz < layers[p].nnz) p = l;
        bound = layers[p].nnz;
    } else {
        bound = L.base[r];
    }
    if (capacity < bound)
        return fail(HLN_ENOMEM, "output capacity %lld < bound %lld", static_cast<long long>(capacity), bound);
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % hln::Arena::kAlign)
        return fail(HLN_EINVAL, "workspace NULL or not 256-byte aligned");
    const size_t need = compose_ws(L);
    if (workspace_bytes < need) return fail(HLN_ENOMEM, "workspace too small: %zu < %zu", workspace_bytes, need);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hln::Arena ar{static_cast<char*>(workspace), workspace_bytes};
    const long long total = L.base[r];
    int32_t* flag = ar.take<int32_t>(total + 1);
    int32_t* pos = ar.take<int32_t>(total + 1);
    int32_t* cnt = ar.take<int32_t>(L.n + 1);
    void* sws = ar.base + ar.off;
    const size_t sws_bytes = workspace_bytes - ar.off;
    if (mode == 0) {
        const long long nnz = layers[p].nnz;
        hipLaunchKernelGGL(k_and_mark, dim3(grid_for(nnz)), dim3(256), 0, st, L, p, flag);
        s = hln::prim::scan_exclusive<int32_t>(flag, pos, nnz, sws, sws_bytes, st);
        if (s != HLN_OK) return s;
        hipLaunchKernelGGL(k_and_fill, dim3(grid_for(std::max<long long>(nnz, L.n + 1))), dim3(256), 0, st, L, p,
                           flag, pos, out_rp, out_ci);
    } else {
        hipLaunchKernelGGL(k_or_mark, dim3(grid_for(total)), dim3(256), 0, st, L, flag);
        s = hln::prim::scan_exclusive<int32_t>(flag, pos, total, sws, sws_bytes, st);
        if (s != HLN_OK) return s;
        hipLaunchKernelGGL(k_or_count, dim3(grid_for(L.n)), dim3(256), 0, st, L, pos, cnt);
        s = hln::prim::scan_exclusive<int32_t>(cnt, out_rp, L.n, sws, sws_bytes, st);
        if (s != HLN_OK) return s;
        hipLaunchKernelGGL(k_or_fill, dim3(grid_for(total)), dim3(256), 0, st, L, flag, pos, out_rp, out_ci);
    }
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

}  // namespace

extern "C" {

size_t hln_compose_workspace_size(const hln_csr* layers, int32_t r) {
    LayerSet L;
    if (check_layers(layers, r, L) != HLN_OK) return 0;
    return compose_ws(L);
}

hln_status hln_compose_and(const hln_csr* layers, int32_t r, int32_t* out_row_ptr, int32_t* out_col_idx,
                           int64_t capacity, void* workspace, size_t workspace_bytes, void* stream) {
    return compose(0, layers, r, out_row_ptr, out_col_idx, capacity, workspace, workspace_bytes, stream);
}

hln_status hln_compose_or(const hln_csr* layers, int32_t r, int32_t* out_row_ptr, int32_t* out_col_idx,
                          int64_t capacity, void* workspace, size_t workspace_bytes, void* stream) {
    return compose(1, layers, r, out_row_ptr, out_col_idx, capacity, workspace, workspace_bytes, stream);
}

size_t hln_compose_and_batch_workspace_size(const hln_and_problem* problems, int32_t count) {
    AndSizes Z;
    if (and_sizes(problems, count, Z, false) != HLN_OK) return 0;
    return and_ws(count, Z);
}

hln_status hln_compose_and_batch(const hln_and_problem* problems, int32_t count, void* workspace,
                                 size_t workspace_bytes, void* stream) {
    using hln::fail;
    hln::clear_error();
    AndSizes Z;
    hln_status s = and_sizes(problems, count, Z, true);
    if (s != HLN_OK) return s;
    if (count == 0) return HLN_OK;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % hln::Arena::kAlign)
        return fail(HLN_EINVAL, "workspace NULL or not 256-byte aligned");
    const size_t need = and_ws(count, Z);
    if (workspace_bytes < need) return fail(HLN_ENOMEM, "workspace too small: %zu < %zu", workspace_bytes, need);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hln::Arena ar{static_cast<char*>(workspace), workspace_bytes};
    AndProblem* probs = ar.take<AndProblem>(count + 1);
    long long* e_off = ar.take<long long>(count + 1);
    long long* r_off = ar.take<long long>(count + 1);
    LayerPtrs* lay = ar.take<LayerPtrs>(std::max<long long>(Z.layers, 1));
    int32_t* flag = ar.take<int32_t>(Z.arcs + 1);
    int32_t* pos = ar.take<int32_t>(Z.arcs + 1);
    void* sws = ar.base + ar.off;
    const size_t sws_bytes = workspace_bytes - ar.off;

    long long eo = 0, ro = 0, lo = 0;
    for (int first = 0; first < count; first += kAndChunk) {
        AndChunk c{};
        c.first = first;
        c.count = std::min(kAndChunk, count - first);
        for (int i = 0; i <= c.count; ++i) {
            c.e_off[i] = eo;
            c.r_off[i] = ro;
            if (i == c.count) break;
            const hln_and_problem& P = problems[first + i];
            int p = 0;
            for (int l = 0; l < P.r; ++l)
                if (P.layers[l].nnz < P.layers[p].nnz) p = l;
            c.q[i] = AndProblem{P.out_row_ptr, P.out_col_idx, lo, P.layers[0].n, P.r, p};
            eo += P.layers[p].nnz;
            ro += static_cast<long long>(P.layers[0].n) + 1;
            lo += P.r;
        }
        hipLaunchKernelGGL(k_put_and, dim3(1), dim3(64), 0, st, c, probs, e_off, r_off);
    }
    {
        LayChunk c{};
        c.first = 0;
        c.count = 0;
        for (int q = 0; q < count; ++q)
            for (int l = 0; l < problems[q].r; ++l) {
                c.l[c.count] = LayerPtrs{problems[q].layers[l].row_ptr, problems[q].layers[l].col_idx};
                if (++c.count == kLayChunk) {
                    hipLaunchKernelGGL(k_put_lay, dim3(1), dim3(128), 0, st, c, lay);
                    c.first += c.count;
                    c.count = 0;
                }
            }
        if (c.count) hipLaunchKernelGGL(k_put_lay, dim3(1), dim3(128), 0, st, c, lay);
    }
    HLN_TRY_HIP(hipGetLastError());
    if (Z.arcs > 0)
        hipLaunchKernelGGL(k_ba_mark, dim3(grid_for(Z.arcs)), dim3(256), 0, st, probs, lay, e_off, count, Z.arcs, flag);
    s = hln::prim::scan_exclusive<int32_t>(flag, pos, Z.arcs, sws, sws_bytes, st);
    if (s != HLN_OK) return s;
    hipLaunchKernelGGL(k_ba_fill, dim3(grid_for(std::max(Z.arcs, Z.rows))), dim3(256), 0, st, probs, lay, e_off, r_off,
                       count, Z.arcs, Z.rows, flag, pos);
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

}  // extern "C"
