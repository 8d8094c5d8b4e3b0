// Batched exact closeness of many graphs (layers and aggregates of many
// HoMLNs): the paper analyses every layer independently (Sec. 3, the Psi
// step, "in parallel"); here all of them go through one persistent launch
// per source-width class.
//
// Work unit: a tile = (graph g, batch b of W consecutive source ids).  One
// workgroup runs a tile's whole BFS: the frontier and next bitsets of the
// graph (n words of W bits) live in LDS, so a level is a block-local sweep
// separated by __syncthreads; no grid barrier is involved.  Persistent
// workgroups pull tiles from a device counter; tiles are ordered graph by
// graph, most expensive graph first, so concurrent workgroups share the
// graph's CSR in L2.
//
// Per level, two passes over the tile's graph:
//   arcs     every arc (u, w) is read from a packed (u << 16 | w) array
//            (coalesced, 4 bytes per arc; tile graphs have n < 65,536) and
//            the neighbour's frontier word fr[w] is ORed into acc[u] with an
//            LDS atomic -- no per-row work, so degree skew costs nothing;
//   vertices new = acc[u] & ~vis[u] becomes the next frontier fr[u], acc[u]
//            is cleared, and the partial sums are updated.
// The visited word and the per-tile partial sums of a vertex live in
// workgroup-private global scratch.  At the end of a tile the partials are
// added to the graph's S, R and h2 with atomics (R counts the batch sources
// that reached the vertex, itself included), so after every tile of a graph
// S[v], R[v] are v's own sums (undirected graph: d(s,v) = d(v,s)).  A final
// pass computes closeness in the fixed FP64 order.
#include "hln_internal.hpp"
#include "hln_prim.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

struct hln_plan {
    int device = -1;
    // tuned source width per log2(n) class: 8..64 = LDS tiles, 512..4096 =
    // the persistent cooperative kernel (hln_closeness_layer); 0 = untuned
    int width_for_class[32];
    void* pinned = nullptr;         // staging for per-call descriptors
    size_t pinned_bytes = 0;
    hipEvent_t staged = nullptr;    // completion of the last staging copy
    bool staged_pending = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // Staging of captured calls: a capture's copy node reads its buffer at
    // every replay, so each capture gets a buffer of its own.  `armed` is
    // reserved for the next capture (hln_plan_reserve, or hln_plan_capture
    // itself); a capture moves it to `own` (the plan's own graph, freed when
    // that graph is replaced) or to `frozen` (a graph the caller captured,
    // freed only when the plan is destroyed).
    void* armed = nullptr;
    size_t armed_bytes = 0;
    void* own = nullptr;
    std::vector<void*> frozen;
    // persistent launches of the last enqueue (call, capture or tuning run):
    // [1] cooperative, [2] ordinary kernel node inside a stream capture
    int paths[3] = {0, 0, 0};
};

namespace {

constexpr int kTileBlock = 1024;
constexpr int kMaxTileN = 65535;   // packed arcs hold 16-bit vertex ids

struct TileGraph {
    const int32_t* row_ptr;
    const int32_t* col_idx;
    int64_t* S;
    int32_t* R;
    int32_t* H2;
    double* cc;
    uint32_t* arcs;                 // packed (row << 16 | col), nnz entries (workspace)
    int64_t nnz;                    // declared arc count (row_ptr[n] must not exceed it)
    int32_t n;
    int32_t width;                  // source width of this graph's tiles
};

struct TileArgs {
    const TileGraph* graphs;
    const int2* tiles;              // (graph, batch), processing order
    int n_tiles;
    int* counter;                   // work queue head
    void* vis;                      // per workgroup: max_n words
    int32_t* s_part;                // per workgroup: max_n
    int32_t* h_part;                // per workgroup: max_n
    int max_n;
    int* fault;
};

template <typename T>
__device__ __forceinline__ int popc_t(T x) {
    if constexpr (sizeof(T) == 8) return __popcll(static_cast<unsigned long long>(x));
    else return __popc(static_cast<unsigned>(x));
}

template <typename T>
__device__ __forceinline__ T shfl_xor_t(T x, int m) {
    if constexpr (sizeof(T) == 8) return hln::dev::shfl_xor_u64(x, m);
    else return static_cast<T>(__shfl_xor(static_cast<int>(x), m, 64));
}

// OR x into the T-sized LDS slot u (sub-word slots go through the 32-bit
// word that contains them)
template <typename T>
__device__ __forceinline__ void lds_or(T* acc, int u, T x) {
    if constexpr (sizeof(T) == 8) {
        atomicOr(reinterpret_cast<unsigned long long*>(acc) + u, static_cast<unsigned long long>(x));
    } else if constexpr (sizeof(T) == 4) {
        atomicOr(reinterpret_cast<unsigned*>(acc) + u, static_cast<unsigned>(x));
    } else {
        constexpr int per = 4 / sizeof(T);
        const unsigned sh = 8u * sizeof(T) * static_cast<unsigned>(u % per);
        atomicOr(reinterpret_cast<unsigned*>(acc) + u / per, static_cast<unsigned>(x) << sh);
    }
}

template <typename T>
__global__ __launch_bounds__(kTileBlock) void k_tiles(TileArgs a) {
    constexpr int W = 8 * sizeof(T);
    extern __shared__ __align__(16) unsigned char s_raw[];
    __shared__ int s_tile;
    T* vis = static_cast<T*>(a.vis) + static_cast<size_t>(blockIdx.x) * a.max_n;
    int32_t* sp = a.s_part + static_cast<size_t>(blockIdx.x) * a.max_n;
    int32_t* hp = a.h_part + static_cast<size_t>(blockIdx.x) * a.max_n;
    // acc is padded to whole 32-bit words
    const int acc_words = (a.max_n * static_cast<int>(sizeof(T)) + 3) / 4;
    T* acc = reinterpret_cast<T*>(s_raw);
    T* fr = reinterpret_cast<T*>(s_raw + 4 * acc_words);
    if (hln::dev::load_agent_i32(a.fault) != 0) return;       // the preparation found bad input

    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(a.counter, 1);
        __syncthreads();
        const int tile = s_tile;
        __syncthreads();
        if (tile >= a.n_tiles) break;
        const int2 tb = a.tiles[tile];
        const TileGraph G = a.graphs[tb.x];
        const int n = G.n;
        const int nnz = G.row_ptr[n];
        const int src0 = tb.y * W;
        const int cnt = min(W, n - src0);
        const uint32_t* __restrict__ arcs = G.arcs;

        for (int i = threadIdx.x; i < (n * static_cast<int>(sizeof(T)) + 3) / 4; i += kTileBlock)
            reinterpret_cast<unsigned*>(acc)[i] = 0u;
        for (int v = threadIdx.x; v < n; v += kTileBlock) {
            const int bit = v - src0;
            const T w0 = (bit >= 0 && bit < cnt) ? static_cast<T>(T(1) << bit) : T(0);
            fr[v] = w0;
            vis[v] = w0;
            sp[v] = 0;
            hp[v] = 0;
        }
        __syncthreads();

        for (int d = 1;; ++d) {
            // arcs: acc[u] |= fr[w]
            for (int e = threadIdx.x; e < nnz; e += kTileBlock) {
                const uint32_t p = arcs[e];
                const T x = fr[p & 0xffffu];
                if (x) lds_or<T>(acc, static_cast<int>(p >> 16), x);
            }
            __syncthreads();
            // vertices: new bits become the next frontier
            int any = 0;
            for (int v = threadIdx.x; v < n; v += kTileBlock) {
                const T av = acc[v];
                acc[v] = T(0);                  // cleared by the thread that read it
                const T vv = vis[v];
                const T nw = static_cast<T>(av & ~vv);
                fr[v] = nw;
                if (nw) {
                    vis[v] = static_cast<T>(vv | nw);
                    const int c = popc_t(nw);
                    sp[v] += d * c;
                    if (d == 2) hp[v] += c;
                    any = 1;
                }
            }
            if (!__syncthreads_or(any)) break;
        }

        // flush the tile's partial sums into the graph's accumulators
        for (int v = threadIdx.x; v < n; v += kTileBlock) {
            const int r = popc_t(vis[v]);
            if (r) atomicAdd(&G.R[v], r);
            if (sp[v]) atomicAdd(reinterpret_cast<unsigned long long*>(&G.S[v]), static_cast<unsigned long long>(sp[v]));
            if (G.H2 && hp[v]) atomicAdd(&G.H2[v], hp[v]);
        }
        __syncthreads();
    }
}

// zero the accumulators of every graph and reset the work queues
__global__ void k_batch_prep(const TileGraph* graphs, int n_graphs, int* counters, int n_counters) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_counters; i += gridDim.x * blockDim.x) counters[i] = 0;
    for (int g = blockIdx.y; g < n_graphs; g += gridDim.y) {
        const TileGraph G = graphs[g];
        if (G.width >= 512) continue;                 // on the cooperative kernel
        for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < G.n; v += gridDim.x * blockDim.x) {
            G.S[v] = 0;
            G.R[v] = 0;
            if (G.H2) G.H2[v] = 0;
        }
    }
}

// packed arcs of every graph; the CSR is checked first (row pointers
// monotone within the declared arc count, ids in range: fault code 2) so no
// later access leaves a buffer
__global__ void k_batch_pack(const TileGraph* graphs, int n_graphs, int* fault) {
    for (int g = blockIdx.y; g < n_graphs; g += gridDim.y) {
        const TileGraph G = graphs[g];
        if (G.width >= 512) continue;
        for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < G.n; v += gridDim.x * blockDim.x) {
            const int e0 = G.row_ptr[v], e1 = G.row_ptr[v + 1];
            if (e0 < 0 || e1 < e0 || e1 > G.nnz) {
                hln::dev::store_agent_i32(fault, 2);
                continue;
            }
            for (int e = e0; e < e1; ++e) {
                const int w = G.col_idx[e];
                if (static_cast<unsigned>(w) >= static_cast<unsigned>(G.n)) {
                    hln::dev::store_agent_i32(fault, 2);
                    G.arcs[e] = 0u;
                } else {
                    G.arcs[e] = (static_cast<uint32_t>(v) << 16) | static_cast<uint32_t>(w);
                }
            }
        }
    }
}

__global__ void k_batch_cc(const TileGraph* graphs, int n_graphs) {
    for (int g = blockIdx.y; g < n_graphs; g += gridDim.y) {
        const TileGraph G = graphs[g];
        if (!G.cc || G.width >= 512) continue;
        const int n = G.n;
        for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
            const int64_t s = G.S[v];
            const int32_t r = G.R[v];
            double c = 0.0;
            if (r > 1 && s > 0 && n > 1) {
                const double reach = static_cast<double>(r - 1);
                const double q1 = reach / static_cast<double>(s);
                const double q2 = reach / static_cast<double>(n - 1);
                c = q1 * q2;
            }
            G.cc[v] = c;
        }
    }
}

int log2_class(int n) {
    int c = 0;
    while ((1 << (c + 1)) <= n && c < 31) ++c;
    return c;
}

size_t lds_budget() {
    const hln::DeviceInfo* di = hln::device_info();
    size_t b = di ? di->lds_per_block : 65536;
    if (b > 160 * 1024) b = 160 * 1024;
    return b > 1024 ? b - 1024 : b;      // room for the static shared words
}

// widest word (64/32/16/8 bits) whose two n-word arrays fit in LDS; 0 if none
int widest_fit(int n, size_t budget) {
    if (n > kMaxTileN) return 0;
    for (int w = 64; w >= 8; w >>= 1)
        if (2ull * static_cast<unsigned long long>(n) * (w / 8) + 8 <= budget) return w;
    return 0;
}

struct Layout {
    int n_graphs = 0;
    int max_n = 0;
    long long total_n = 0;
    long long total_nnz = 0;
    int n_tiles[4] = {0, 0, 0, 0};   // per width class: 64, 32, 16, 8
    int max_n_class[4] = {0, 0, 0, 0};
    int grid = 0;
    size_t coop_bytes = 0;             // cooperative graphs: coop_slices slices of coop_slice_bytes
    size_t coop_slice_bytes = 0;       // workspace of the largest graph on the cooperative kernel
    int coop_slices = 1;               // partitions of a multi-graph cooperative launch at most
    size_t desc_bytes = 0, tiles_bytes = 0, margs_bytes = 0, mlist_bytes = 0, counters_bytes = 0, heavy_bytes = 0;
    size_t stage_bytes = 0;            // host-staged tables: descriptors, tiles, launch arguments, lists
    size_t vis_bytes = 0, part_bytes = 0, total = 0;
};

int cls_of(int w) { return w == 64 ? 0 : w == 32 ? 1 : w == 16 ? 2 : 3; }

// Source width of a graph of n vertices: the tuned choice of its size class,
// else the widest LDS tile that fits, else the cooperative kernel at 4096.
int chosen_width(const hln_plan* plan, int n, size_t budget) {
    const int fit = widest_fit(n, budget);
    int w = plan ? plan->width_for_class[log2_class(n)] : 0;
    if (w >= 512) return w;
    if (!fit) return 4096;
    if (w <= 0 || w > fit) w = fit;
    return w;
}

bool is_coop(int w) { return w >= 512; }

constexpr int kPartsCap = 64;                // partitions of a multi-graph cooperative launch: at most

// Partitions a multi-graph launch may use (HLN_MAX_PARTS, default 4).
// Measured on config 3 (graphs of 10^4-5*10^4 vertices): 2, 4, 6, 8, 16
// and 32 partitions gave 1,425, 1,623, 1,296, 1,478, 1,148 and 936 GTEPS --
// a partition needs enough compute units for a graph's light levels, and a
// count that is not a power of two spreads partitions across the XCDs.
int max_parts() {
    int p = 4;
    if (const char* e = getenv("HLN_MAX_PARTS")) p = atoi(e);
    return std::max(1, std::min(p, kPartsCap));
}

// The largest power of two <= x (x >= 1): partition counts that divide the
// XCD count keep each partition on whole XCDs.
int pow2_floor(int x) {
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}
constexpr int kCoopWidths = 4;               // widths it runs: 512, 1024, 2048, 4096
constexpr int kCoopWidthList[kCoopWidths] = {512, 1024, 2048, 4096};
// Graphs larger than this run on the whole grid (one partition): config 2's
// five graphs of 10^5 vertices took 92.5 ms through one partition, 101.7 ms
// through two and 128 ms through four (a quarter of the chip runs such a
// graph 3.5x longer), while config 3's graphs of 10^4-5*10^4 vertices gain
// from four.
constexpr int kPartitionMaxN = 65536;

// Width of a graph with listed sources (always the persistent kernel): its
// size class's tuned persistent width, else the narrowest persistent width
// holding all its sources in one batch (4096 at most).
int listed_width(const hln_plan* plan, int n, int n_src) {
    const int w = plan ? plan->width_for_class[log2_class(n)] : 0;
    if (w >= 512) return w;
    int x = 512;
    while (x < 4096 && x < n_src) x *= 2;
    return x;
}

// Graph g of a call takes a list of sources when the call has a source
// table and n_src[g] >= 0 (-1: all of its vertices).  The count, not the
// pointer, decides: an empty list may come with a NULL pointer.
bool is_listed(const int32_t* const* sources, const int32_t* n_src, int g) {
    return sources != nullptr && n_src != nullptr && n_src[g] >= 0;
}

int graph_width(const hln_plan* plan, const hln_csr* graphs, const int32_t* const* sources, const int32_t* n_src,
                int g, size_t budget) {
    if (is_listed(sources, n_src, g)) return listed_width(plan, graphs[g].n, n_src[g]);
    return chosen_width(plan, graphs[g].n, budget);
}

// Workspace layout.  Sizes are worst cases over every width a graph could be
// tuned to (tiles of 8 sources, the cooperative kernel at 4096), so the
// workspace size does not change when the plan is tuned.
hln_status plan_layout(const hln_plan* plan, const hln_csr* graphs, int32_t n_graphs, Layout& L) {
    using hln::fail;
    if (!graphs || n_graphs < 1) return fail(HLN_EINVAL, "need at least one graph");
    const hln::DeviceInfo* di = hln::device_info();
    if (!di) return HLN_EDEVICE;
    const size_t budget = lds_budget();
    L.n_graphs = n_graphs;
    long long max_tiles = 0;
    double total_work = 0.0, max_work = 0.0;
    for (int g = 0; g < n_graphs; ++g) {
        const hln_csr& c = graphs[g];
        if (c.n < 1 || c.nnz < 0 || !c.row_ptr || (c.nnz > 0 && !c.col_idx))
            return fail(HLN_EINVAL, "graph %d: bad descriptor", g);
        L.coop_slice_bytes = std::max(L.coop_slice_bytes, hln::multi_slice_bytes(c.n, c.nnz, 4096));
        const double work = static_cast<double>(c.n) * static_cast<double>(c.nnz + c.n);
        total_work += work;
        max_work = std::max(max_work, work);
        if (widest_fit(c.n, budget)) {
            max_tiles += (c.n + 7) / 8;
            L.max_n = std::max(L.max_n, c.n);
            L.total_n += c.n;
            L.total_nnz += c.nnz;
        }
        const int w = chosen_width(plan, c.n, budget);
        if (is_coop(w)) continue;
        const int k = cls_of(w);
        L.n_tiles[k] += (c.n + w - 1) / w;
        L.max_n_class[k] = std::max(L.max_n_class[k], c.n);
    }
    using hln::Arena;
    L.grid = di->cus;
    L.desc_bytes = Arena::round(sizeof(TileGraph) * n_graphs);
    L.tiles_bytes = Arena::round(sizeof(int2) * static_cast<size_t>(std::max<long long>(max_tiles, 1)));
    L.counters_bytes = Arena::round(sizeof(int) * 4);
    L.heavy_bytes = Arena::round(sizeof(uint32_t) * static_cast<size_t>(L.total_nnz + 1));
    L.vis_bytes = Arena::round(static_cast<size_t>(L.grid) * std::max(L.max_n, 1) * 8);
    L.part_bytes = Arena::round(static_cast<size_t>(L.grid) * std::max(L.max_n, 1) * 4);
    // as many workspace slices as partitions a multi-graph launch can use:
    // up to 8, no more than the graphs, and one when a single graph holds
    // most of the work
    L.coop_slices = pow2_floor(
        std::max(1, std::min({max_parts(), n_graphs, static_cast<int>(total_work / std::max(max_work, 1.0))})));
    L.coop_bytes = static_cast<size_t>(L.coop_slices) * L.coop_slice_bytes;
    L.margs_bytes = Arena::round(hln::multi_args_bytes(n_graphs));
    L.mlist_bytes = Arena::round(sizeof(int) * (static_cast<size_t>(n_graphs) + 2 * kCoopWidths * (kPartsCap + 1)));
    L.stage_bytes = L.desc_bytes + L.tiles_bytes + L.margs_bytes + L.mlist_bytes;
    L.total = L.stage_bytes + L.counters_bytes + L.heavy_bytes + L.vis_bytes + 2 * L.part_bytes + L.coop_bytes;
    return HLN_OK;
}

// Host-side tables: descriptors and the tile order (per width class, graphs
// by decreasing n * nnz, batches in order).
void build_tables(const hln_plan* plan, const hln_csr* graphs, int32_t n_graphs, const int32_t* const* sources,
                  const int32_t* n_src, int64_t* const* S, int32_t* const* R, double* const* cc, int32_t* const* h2,
                  const Layout& L, char* dev_base, TileGraph* desc, int2* tiles, int* first_tile) {
    const size_t budget = lds_budget();
    uint32_t* arcs = reinterpret_cast<uint32_t*>(dev_base + L.stage_bytes + L.counters_bytes);
    long long off = 0;
    std::vector<int> order(n_graphs);
    for (int g = 0; g < n_graphs; ++g) {
        const hln_csr& c = graphs[g];
        desc[g].row_ptr = c.row_ptr;
        desc[g].col_idx = c.col_idx;
        desc[g].S = S[g];
        desc[g].R = R[g];
        desc[g].H2 = h2 ? h2[g] : nullptr;
        desc[g].cc = cc ? cc[g] : nullptr;
        desc[g].nnz = c.nnz;
        desc[g].n = c.n;
        desc[g].width = graph_width(plan, graphs, sources, n_src, g, budget);
        desc[g].arcs = arcs + off;
        if (!is_coop(desc[g].width)) off += c.nnz;
        order[g] = g;
    }
    std::sort(order.begin(), order.end(), [&](int x, int y) {
        const double cx = static_cast<double>(graphs[x].n) * static_cast<double>(graphs[x].nnz + graphs[x].n);
        const double cy = static_cast<double>(graphs[y].n) * static_cast<double>(graphs[y].nnz + graphs[y].n);
        return cx > cy || (cx == cy && x < y);
    });
    int t = 0;
    for (int k = 0; k < 4; ++k) {
        first_tile[k] = t;
        const int w = 64 >> k;
        for (int g : order) {
            if (desc[g].width != w) continue;
            const int nb = (graphs[g].n + w - 1) / w;
            for (int b = 0; b < nb; ++b) tiles[t++] = make_int2(g, b);
        }
    }
    first_tile[4] = t;
}

template <typename T>
hln_status launch_tiles(const TileArgs& ta, int grid, size_t lds, hipStream_t st) {
    const void* f = reinterpret_cast<const void*>(&k_tiles<T>);
    HLN_TRY_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    hipLaunchKernelGGL(k_tiles<T>, dim3(grid), dim3(kTileBlock), lds, st, ta);
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

hln_status enqueue_batch(hln_plan* plan, const hln_csr* graphs, int32_t n_graphs, const int32_t* const* sources,
                         const int32_t* n_src, int64_t* const* S, int32_t* const* R, double* const* cc,
                         int32_t* const* h2, void* workspace, size_t workspace_bytes, hipStream_t st,
                         bool own_capture) {
    using hln::fail;
    Layout L;
    hln_status s = plan_layout(plan, graphs, n_graphs, L);
    if (s != HLN_OK) return s;
    if (!S || !R) return fail(HLN_EINVAL, "S and R arrays are required");
    for (int g = 0; g < n_graphs; ++g)
        if (!S[g] || !R[g]) return fail(HLN_EINVAL, "graph %d: NULL output", g);
    if (sources) {
        if (!n_src) return fail(HLN_EINVAL, "a source table needs n_src");
        for (int g = 0; g < n_graphs; ++g) {
            if (n_src[g] == -1) continue;                   // all of graph g's vertices
            if (n_src[g] < -1 || n_src[g] > graphs[g].n)
                return fail(HLN_EINVAL, "graph %d: n_src %d outside [-1, n = %d]", g, n_src[g], graphs[g].n);
            if (n_src[g] > 0 && !sources[g]) return fail(HLN_EINVAL, "graph %d: %d listed sources at NULL", g, n_src[g]);
            if (h2 && h2[g]) return fail(HLN_EUNSUPPORTED, "graph %d: h2 is produced in all-source mode only", g);
            if (graphs[g].nnz >= (1LL << 29) || static_cast<long long>(graphs[g].n) * 512 >= (1LL << 31))
                return fail(HLN_EUNSUPPORTED, "graph %d too large for the persistent kernel", g);
        }
    }
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % hln::Arena::kAlign)
        return fail(HLN_EINVAL, "workspace NULL or not 256-byte aligned");
    if (workspace_bytes < L.total) return fail(HLN_ENOMEM, "workspace too small: %zu < %zu", workspace_bytes, L.total);
    const size_t stage = L.stage_bytes;
    // inside a stream capture (ours or the caller's) the staging is the
    // buffer armed beforehand, which the capture then keeps: no allocation,
    // no host wait
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HLN_TRY_HIP(hipStreamIsCapturing(st, &cap));
    const bool capturing = cap == hipStreamCaptureStatusActive || own_capture;
    void** pin = capturing ? &plan->armed : &plan->pinned;
    size_t* pin_bytes = capturing ? &plan->armed_bytes : &plan->pinned_bytes;
    if (capturing) {
        if (!plan->armed || *pin_bytes < stage)
            return fail(HLN_EINVAL, "capturing: reserve staging for this capture first (hln_plan_reserve)");
    } else {
        if (plan->staged_pending) {
            HLN_TRY_HIP(hipEventSynchronize(plan->staged));   // the previous copy has read the staging
            plan->staged_pending = false;
        }
        if (*pin_bytes < stage) {
            if (*pin) HLN_TRY_HIP(hipHostFree(*pin));
            *pin = nullptr;
            HLN_TRY_HIP(hipHostMalloc(pin, stage, hipHostMallocDefault));
            *pin_bytes = stage;
        }
    }
    char* dev = static_cast<char*>(workspace);
    TileGraph* desc_h = static_cast<TileGraph*>(*pin);
    int2* tiles_h = reinterpret_cast<int2*>(static_cast<char*>(*pin) + L.desc_bytes);
    int first[5];
    build_tables(plan, graphs, n_graphs, sources, n_src, S, R, cc, h2, L, dev, desc_h, tiles_h, first);

    // Graphs on the cooperative kernel, grouped by width: each group is one
    // multi-graph launch whose partitions take its graphs longest work first
    // (each to the least loaded partition).  Launch arguments and lists go
    // into the staging with the tables.
    char* const coop_ws = dev + L.stage_bytes + L.counters_bytes + L.heavy_bytes + L.vis_bytes + 2 * L.part_bytes;
    void* const args_h = static_cast<char*>(*pin) + L.desc_bytes + L.tiles_bytes;
    int* const lists_h = reinterpret_cast<int*>(static_cast<char*>(*pin) + L.desc_bytes + L.tiles_bytes + L.margs_bytes);
    struct CoopGroup {
        int width;
        bool per_source;
        int parts, pfirst_off;
    };
    std::vector<CoopGroup> groups;
    {
        auto listed = [&](int g) { return is_listed(sources, n_src, g); };
        auto work = [&](int g) {
            const double src = listed(g) ? static_cast<double>(n_src[g]) : static_cast<double>(graphs[g].n);
            return src * static_cast<double>(graphs[g].nnz + graphs[g].n);
        };
        int plist_n = 0, pfirst_n = n_graphs;
        for (int wi = 0; wi < kCoopWidths; ++wi)
            for (int ps = 0; ps < 2; ++ps) {
                const int width = kCoopWidthList[wi];
                std::vector<int> members;
                double total = 0.0, mx = 0.0;
                int max_n = 0;
                for (int g = 0; g < n_graphs; ++g) {
                    if (desc_h[g].width != width || listed(g) != (ps == 1)) continue;
                    if (listed(g) && n_src[g] == 0) continue;          // nothing to compute
                    members.push_back(g);
                    total += work(g);
                    mx = std::max(mx, work(g));
                    max_n = std::max(max_n, graphs[g].n);
                }
                if (members.empty()) continue;
                int parts = pow2_floor(std::max(1, std::min({L.coop_slices, static_cast<int>(members.size()),
                                                             static_cast<int>(total / std::max(mx, 1.0))})));
                if (max_n > kPartitionMaxN) parts = 1;
                std::sort(members.begin(), members.end(), [&](int x, int y) {
                    return work(x) > work(y) || (work(x) == work(y) && x < y);
                });
                std::vector<std::vector<int>> bins(parts);
                std::vector<double> load(parts, 0.0);
                for (int g : members) {
                    const int q = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
                    bins[q].push_back(g);
                    load[q] += work(g);
                }
                int* pf = lists_h + pfirst_n;
                for (int q = 0; q < parts; ++q) {
                    pf[q] = plist_n;
                    for (int g : bins[q]) {
                        lists_h[plist_n++] = g;
                        const hln_status r = hln::multi_fill(
                            graphs[g], listed(g) ? sources[g] : nullptr, listed(g) ? n_src[g] : graphs[g].n, S[g],
                            R[g], cc ? cc[g] : nullptr, h2 ? h2[g] : nullptr, width,
                            coop_ws + static_cast<size_t>(q) * L.coop_slice_bytes, L.coop_slice_bytes, args_h, g);
                        if (r != HLN_OK) return r;
                    }
                }
                pf[parts] = plist_n;
                groups.push_back(CoopGroup{width, ps == 1, parts, pfirst_n});
                pfirst_n += parts + 1;
            }
    }
    HLN_TRY_HIP(hipMemcpyAsync(dev, *pin, stage, hipMemcpyHostToDevice, st));
    if (capturing) {
        // the captured copy reads this buffer at every replay: it leaves the
        // armed slot and stays allocated while the graph can run
        if (own_capture) plan->own = plan->armed;
        else plan->frozen.push_back(plan->armed);
        plan->armed = nullptr;
        plan->armed_bytes = 0;
    } else {
        if (!plan->staged) HLN_TRY_HIP(hipEventCreateWithFlags(&plan->staged, hipEventDisableTiming));
        HLN_TRY_HIP(hipEventRecord(plan->staged, st));
        plan->staged_pending = true;
    }
    const TileGraph* desc_d = reinterpret_cast<const TileGraph*>(dev);
    const int2* tiles_d = reinterpret_cast<const int2*>(dev + L.desc_bytes);
    int* counters = reinterpret_cast<int*>(dev + L.stage_bytes);
    char* p = dev + L.stage_bytes + L.counters_bytes + L.heavy_bytes;
    void* vis = p;
    int32_t* s_part = reinterpret_cast<int32_t*>(p + L.vis_bytes);
    int32_t* h_part = reinterpret_cast<int32_t*>(p + L.vis_bytes + L.part_bytes);

    const unsigned gy = static_cast<unsigned>(std::min(n_graphs, 1024));
    const unsigned gx = static_cast<unsigned>(std::max(1, std::min((L.max_n + 255) / 256, 64)));
    int* fault = hln::fault_word();
    if (!fault) return HLN_EDEVICE;
    hipLaunchKernelGGL(k_batch_prep, dim3(gx, gy), dim3(256), 0, st, desc_d, n_graphs, counters, 4);
    hipLaunchKernelGGL(k_batch_pack, dim3(gx, gy), dim3(256), 0, st, desc_d, n_graphs, fault);
    HLN_TRY_HIP(hipGetLastError());
    for (int k = 0; k < 4; ++k) {
        const int nt = first[k + 1] - first[k];
        if (nt == 0) continue;
        TileArgs ta;
        ta.graphs = desc_d;
        ta.tiles = tiles_d + first[k];
        ta.n_tiles = nt;
        ta.counter = counters + k;
        ta.vis = vis;
        ta.s_part = s_part;
        ta.h_part = h_part;
        ta.max_n = L.max_n_class[k];
        ta.fault = fault;
        const int w = 64 >> k;
        const size_t lds = 4ull * ((static_cast<size_t>(ta.max_n) * (w / 8) + 3) / 4) + static_cast<size_t>(ta.max_n) * (w / 8);
        const int grid = std::min(L.grid, nt);
        hln_status r = HLN_OK;
        switch (w) {
            case 64: r = launch_tiles<uint64_t>(ta, grid, lds, st); break;
            case 32: r = launch_tiles<uint32_t>(ta, grid, lds, st); break;
            case 16: r = launch_tiles<uint16_t>(ta, grid, lds, st); break;
            default: r = launch_tiles<uint8_t>(ta, grid, lds, st); break;
        }
        if (r != HLN_OK) return r;
    }
    hipLaunchKernelGGL(k_batch_cc, dim3(gx, gy), dim3(256), 0, st, desc_d, n_graphs);
    HLN_TRY_HIP(hipGetLastError());
    // graphs tuned (or too large) for the persistent cooperative kernel: one
    // multi-graph launch per width; any other width one launch per graph in
    // the first slice
    const void* args_d = dev + L.desc_bytes + L.tiles_bytes;
    const int* lists_d = reinterpret_cast<const int*>(dev + L.desc_bytes + L.tiles_bytes + L.margs_bytes);
    plan->paths[0] = plan->paths[1] = plan->paths[2] = 0;
    for (const CoopGroup& cg : groups) {
        const hln_status r =
            hln::multi_launch(cg.width, cg.per_source, args_d, lists_d, lists_d + cg.pfirst_off, cg.parts, st);
        if (r != HLN_OK) return r;
        ++plan->paths[hln_last_launch_path() == 2 ? 2 : 1];
    }
    return HLN_OK;
}

}  // namespace

extern "C" {

hln_status hln_plan_create(hln_plan** plan) {
    hln::clear_error();
    if (!plan) return hln::fail(HLN_EINVAL, "plan is NULL");
    hln_plan* p = new (std::nothrow) hln_plan();
    if (!p) return hln::fail(HLN_ENOMEM, "out of host memory");
    for (int i = 0; i < 32; ++i) p->width_for_class[i] = 0;
    if (hipGetDevice(&p->device) != hipSuccess) p->device = -1;
    *plan = p;
    return HLN_OK;
}

void hln_plan_destroy(hln_plan* plan) {
    if (!plan) return;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->staged) {
        (void)hipEventSynchronize(plan->staged);
        (void)hipEventDestroy(plan->staged);
    }
    if (plan->pinned) (void)hipHostFree(plan->pinned);
    if (plan->armed) (void)hipHostFree(plan->armed);
    if (plan->own) (void)hipHostFree(plan->own);
    for (void* b : plan->frozen) (void)hipHostFree(b);
    delete plan;
}

hln_status hln_plan_launch_paths(const hln_plan* plan, int32_t* cooperative, int32_t* ordinary) {
    hln::clear_error();
    if (!plan || !cooperative || !ordinary) return hln::fail(HLN_EINVAL, "NULL argument");
    *cooperative = plan->paths[1];
    *ordinary = plan->paths[2];
    return HLN_OK;
}

int32_t hln_plan_width(const hln_plan* plan, int32_t n) {
    if (n < 1) return 0;
    return chosen_width(plan, n, lds_budget());
}

hln_status hln_plan_set_width(hln_plan* plan, int32_t n, int32_t width) {
    hln::clear_error();
    if (!plan) return hln::fail(HLN_EINVAL, "plan is NULL");
    if (n < 1) return hln::fail(HLN_EINVAL, "n must be >= 1 (got %d)", n);
    switch (width) {
        case 0: case 8: case 16: case 32: case 64: case 512: case 1024: case 2048: case 4096: break;
        default: return hln::fail(HLN_EINVAL, "width %d is not 0, a tile width (8/16/32/64) or a persistent one "
                                              "(512/1024/2048/4096)", width);
    }
    plan->width_for_class[log2_class(n)] = width;
    return HLN_OK;
}

size_t hln_closeness_batch_workspace_size(const hln_plan* plan, const hln_csr* graphs, int32_t n_graphs) {
    Layout L;
    if (plan_layout(plan, graphs, n_graphs, L) != HLN_OK) return 0;
    return L.total;
}

hln_status hln_closeness_batch(hln_plan* plan, const hln_csr* graphs, int32_t n_graphs,
                               const int32_t* const* sources, const int32_t* n_src, int64_t* const* S,
                               int32_t* const* R, double* const* cc, int32_t* const* h2, void* workspace,
                               size_t workspace_bytes, void* stream) {
    hln::clear_error();
    if (!plan) return hln::fail(HLN_EINVAL, "plan is NULL");
    return enqueue_batch(plan, graphs, n_graphs, sources, n_src, S, R, cc, h2, workspace, workspace_bytes,
                         static_cast<hipStream_t>(stream), false);
}

hln_status hln_plan_capture(hln_plan* plan, const hln_csr* graphs, int32_t n_graphs, const int32_t* const* sources,
                            const int32_t* n_src, int64_t* const* S, int32_t* const* R, double* const* cc,
                            int32_t* const* h2, void* workspace, size_t workspace_bytes, void* stream) {
    using hln::fail;
    hln::clear_error();
    if (!plan) return fail(HLN_EINVAL, "plan is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!st) return fail(HLN_EINVAL, "capture needs a non-null stream");
    if (plan->exec) {
        HLN_TRY_HIP(hipGraphExecDestroy(plan->exec));
        plan->exec = nullptr;
    }
    if (plan->graph) {
        HLN_TRY_HIP(hipGraphDestroy(plan->graph));
        plan->graph = nullptr;
    }
    // only the replaced graph read the old staging
    if (plan->own) {
        HLN_TRY_HIP(hipHostFree(plan->own));
        plan->own = nullptr;
    }
    // the staging buffer is allocated before capture begins (no allocation
    // inside a capture)
    {
        const hln_status r = hln_plan_reserve(plan, graphs, n_graphs);
        if (r != HLN_OK) return r;
    }
    HLN_TRY_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hln_status s = enqueue_batch(plan, graphs, n_graphs, sources, n_src, S, R, cc, h2, workspace, workspace_bytes,
                                 st, true);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s != HLN_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return fail(HLN_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    plan->graph = g;
    HLN_TRY_HIP(hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0));
    return HLN_OK;
}

hln_status hln_plan_reserve(hln_plan* plan, const hln_csr* graphs, int32_t n_graphs) {
    hln::clear_error();
    if (!plan) return hln::fail(HLN_EINVAL, "plan is NULL");
    Layout L;
    hln_status s = plan_layout(plan, graphs, n_graphs, L);
    if (s != HLN_OK) return s;
    const size_t stage = L.stage_bytes;
    if (plan->armed && plan->armed_bytes >= stage) return HLN_OK;
    // an armed buffer has not been captured yet, so nothing reads it
    if (plan->armed) HLN_TRY_HIP(hipHostFree(plan->armed));
    plan->armed = nullptr;
    plan->armed_bytes = 0;
    HLN_TRY_HIP(hipHostMalloc(&plan->armed, stage, hipHostMallocDefault));
    plan->armed_bytes = stage;
    return HLN_OK;
}

hln_status hln_plan_replay(hln_plan* plan, void* stream) {
    hln::clear_error();
    if (!plan || !plan->exec) return hln::fail(HLN_EINVAL, "no captured graph in this plan");
    HLN_TRY_HIP(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
    return HLN_OK;
}

// Autotuner: for each log2(n) class present, run the class's most expensive
// graph with every source width that fits in LDS, time it with HIP events
// and keep the fastest.  Synchronous.
hln_status hln_plan_tune(hln_plan* plan, const hln_csr* graphs, int32_t n_graphs, int64_t* const* S,
                         int32_t* const* R, void* workspace, size_t workspace_bytes, void* stream) {
    using hln::fail;
    hln::clear_error();
    if (!plan) return fail(HLN_EINVAL, "plan is NULL");
    if (!graphs || n_graphs < 1 || !S || !R) return fail(HLN_EINVAL, "bad arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t budget = lds_budget();
    int rep[32];
    for (int c = 0; c < 32; ++c) rep[c] = -1;
    for (int g = 0; g < n_graphs; ++g) {
        const int c = log2_class(graphs[g].n);
        if (rep[c] < 0 || graphs[g].nnz > graphs[rep[c]].nnz) rep[c] = g;
    }
    hipEvent_t e0, e1;
    HLN_TRY_HIP(hipEventCreate(&e0));
    HLN_TRY_HIP(hipEventCreate(&e1));
    hln_status result = HLN_OK;
    for (int c = 0; c < 32 && result == HLN_OK; ++c) {
        if (rep[c] < 0) continue;
        const int g = rep[c];
        const int fit = widest_fit(graphs[g].n, budget);
        float best = 1e30f;
        int best_w = fit ? fit : 4096;
        int cands[10];
        int nc = 0;
        for (int w = fit; w >= 8 && fit; w >>= 1) cands[nc++] = w;
        cands[nc++] = 1024;
        cands[nc++] = 2048;
        cands[nc++] = 4096;
        for (int ci = 0; ci < nc && result == HLN_OK; ++ci) {
            const int w = cands[ci];
            plan->width_for_class[c] = w;
            float ms = 0.f;
            for (int rep_i = 0; rep_i < 2 && result == HLN_OK; ++rep_i) {   // first run warms up
                if (hipEventRecord(e0, st) != hipSuccess) result = fail(HLN_EDEVICE, "event record failed");
                if (result == HLN_OK)
                    result = enqueue_batch(plan, &graphs[g], 1, nullptr, nullptr, &S[g], &R[g], nullptr, nullptr,
                                           workspace, workspace_bytes, st, false);
                if (result == HLN_OK && hipEventRecord(e1, st) != hipSuccess) result = fail(HLN_EDEVICE, "event record failed");
                if (result == HLN_OK && hipEventSynchronize(e1) != hipSuccess) result = fail(HLN_EDEVICE, "event sync failed");
                if (result == HLN_OK) (void)hipEventElapsedTime(&ms, e0, e1);
            }
            if (result == HLN_OK && ms < best) {
                best = ms;
                best_w = w;
            }
        }
        plan->width_for_class[c] = best_w;
        if (getenv("HLN_VERBOSE"))
            fprintf(stderr, "[hln] tune class 2^%d (n=%d): width %d (%.3f ms)\n", c, graphs[g].n, best_w, best);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return result;
}

}  // extern "C"
