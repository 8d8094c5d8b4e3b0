/*
 * hln.h -- C ABI of the MI355X (gfx950) library for exact closeness
 * centrality on homogeneous multilayer networks (HoMLNs).
 *
 * Paper: "Closeness Centrality Detection in Homogeneous Multilayer
 * Networks" (arXiv 2207.11662).  Problem Statement (Sec. 1): given layers
 * G_1(V,E_1) ... G_l(V,E_l) over one vertex set, find the closeness
 * centrality (CC) nodes of the Boolean AND aggregate of any r <= l layers;
 * each layer is analysed once (the Psi step) and partial results are
 * composed (the Theta step).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers marked [dev] are device pointers on the current HIP device;
 *    [host] pointers are host memory.  The caller owns every buffer.  No
 *    entry point allocates device memory: scratch comes from a caller
 *    workspace whose size the matching *_workspace_size query returns
 *    (256-byte aligned base required).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous and stream-ordered; results are valid after the
 *    stream is synchronised.  Results are deterministic.
 *  - Graphs are CSR over int32 vertex ids: row_ptr[n+1], col_idx[nnz],
 *    nnz = 2 * (undirected edges).  Layers must be symmetric, rows sorted
 *    ascending, no self-loops, no duplicate arcs (Sec. 1: simple undirected
 *    graphs); hln_csr_from_edges produces this form, hln_csr_validate checks
 *    it.
 *  - Every call returns an hln_status.  On an error nothing has been
 *    enqueued and no output has been written; hln_last_error() returns a
 *    thread-local message.  Argument checks that need no device data run on
 *    the host before anything is enqueued.  Faults detected by a kernel
 *    (e.g. a bounded wait that ran out) are reported as HLN_EDEVICE by the
 *    next call that synchronises (hln_device_status).
 */
#ifndef HLN_H
#define HLN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HLN_OK = 0,
    HLN_EINVAL = 1,        /* bad argument (null pointer, size, id range, mode) */
    HLN_ENOMEM = 2,        /* workspace or output capacity too small */
    HLN_EDEVICE = 3,       /* HIP runtime error or device-side fault */
    HLN_EUNSUPPORTED = 4   /* valid request outside what this build supports */
} hln_status;

/* A graph in device memory (see conventions).  n and nnz are host values. */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int32_t* row_ptr;   /* [dev] n+1 */
    const int32_t* col_idx;   /* [dev] nnz */
} hln_csr;

/* hln_opts.flags: listed sources, sums accumulated per vertex (sampling
 * estimate of closeness, hln_closeness_estimate). */
#define HLN_FLAG_PER_VERTEX 1

/* Source-batch width and traversal direction of the bit-parallel BFS. */
typedef struct {
    int32_t width_bits;   /* sources per batch: 64, 128, 256, 512, 1024, 2048 or 4096; 0 = library default
                             (512); n * width_bits / 8 must be below 2^31 (HLN_EUNSUPPORTED otherwise) */
    int32_t direction;    /* 0 = automatic per level (all sources at width 4096: every level
                             bottom-up; listed sources or narrower widths: top-down when
                             32 * frontier arc-words < arcs), 1 = top-down only, 2 = bottom-up only */
    int32_t flags;        /* 0 or HLN_FLAG_PER_VERTEX (see hln_closeness_layer) */
    int32_t* levels;      /* [dev] nullable: per batch of width_bits sources, the BFS levels run
                             (1 + the largest eccentricity among the batch's sources).  All-source
                             mode batches only the vertices that have arcs (one without arcs
                             reaches only itself), by degree class (more than 64 arcs, 64, 32-63,
                             16-31, 8-15, 4-7, 2-3, 1) and ids ascending inside a class, so entries from
                             ceil(#vertices with arcs / width_bits) on are not written; with more
                             than one batch, the batches after the first take the remaining
                             vertices by BFS distance from the first batch's highest-degree
                             vertex (nearest first, distances above 30 together, unreached last;
                             the order above among equals).  Listed sources are batched by the
                             same classes (a source without arcs with the last), list positions
                             ascending inside a class, and the later batches by distance as above
                             (with per-source outputs only below width 4096); outputs stay
                             indexed by list position */
    int64_t* trace;       /* [dev] nullable, zero-filled by the caller: per level run (in order, over
                             all batches) 4 int64: s_memrealtime ticks (100 MHz) when the level's
                             barrier completed, vertices given new bits, new (vertex, source) pairs,
                             the level's direction (0 bottom-up, 1 top-down) */
    int32_t trace_cap;    /* levels `trace` can hold; later levels are not recorded */
} hln_opts;

/* Thread-local text of the last error of this thread ("" if none). */
const char* hln_last_error(void);

/* Library version, e.g. 0x000100 for 0.1.0. */
int32_t hln_version(void);

/* Number of compute units of the current device (0 on error). */
int32_t hln_device_cu_count(void);

/* Synchronises `stream` and reports a device-side fault recorded by the
 * library's kernels since the last call (HLN_EDEVICE), else HLN_OK. */
hln_status hln_device_status(void* stream);

/* Co-residency of the persistent closeness kernels.  Their level loop
 * separates levels with grid barriers, so every block of a launch must be
 * resident at once.  The grid is held to `bound` blocks per compute unit:
 * the smaller of the runtime's occupancy answer and what the kernel's own
 * resources allow on CDNA4 (4 SIMDs per compute unit with 512 VGPRs per lane
 * each, allocated in granules of 8, at most 8 waves per SIMD; 160 KB of LDS
 * per compute unit in granules of 512 bytes; a block of B threads takes
 * ceil(ceil(B/64)/4) wave slots on every SIMD).
 * hln_resident_blocks: that resource bound for a kernel using `vgprs` VGPRs
 *   per lane and `lds_bytes` of LDS per block of `block_threads` threads
 *   (pure arithmetic, no device needed; 0 for invalid arguments).
 * hln_closeness_kernel_residency: info [host] 5 int32 for the kernel that
 *   hln_closeness_layer (mode 0: all-source or per-vertex sums; 1: listed
 *   sources with per-source sums) or hln_closeness_batch (the multi-graph
 *   kernel, block 1024, widths 512-4096; mode 2: all sources, 3: listed
 *   sources) runs at `width_bits`
 *   with blocks of 256, 512 or 1024 threads: VGPRs per lane, static LDS
 *   bytes per block, scratch bytes per lane (hipFuncGetAttributes), the
 *   runtime's occupancy answer, and the bound used.
 * The environment variable HLN_BLOCKS_PER_CU may lower the blocks per
 * compute unit of these launches; a value above the bound makes the launch
 * fail with HLN_EUNSUPPORTED.
 * hln_last_launch_path: how this thread's last persistent launch went out:
 *   0 none yet, 1 a cooperative launch, 2 an ordinary kernel node inside a
 *   stream capture where the runtime refused the cooperative one (the same
 *   grid, within the bound; every wait in the kernel is bounded, so a grid
 *   that did not all start would report fault code 1 instead of hanging). */
int32_t hln_resident_blocks(int32_t vgprs, int32_t lds_bytes, int32_t block_threads);
hln_status hln_closeness_kernel_residency(int32_t width_bits, int32_t block_threads, int32_t mode, int32_t* info);
int32_t hln_last_launch_path(void);

/* ------------------------------------------------------------------------
 * Layer ingest (Sec. 1, Problem Statement; Sec. 4: undirected layers).
 * ------------------------------------------------------------------------
 * hln_csr_from_edges: normalised symmetric CSR from an arbitrary edge list
 * eu[i]--ev[i], i < m (either orientation, duplicates and self-loops
 * allowed: self-loops are dropped, duplicates merged, both arcs of every
 * edge emitted, rows sorted).  row_ptr [dev] n+1 and col_idx [dev] with room
 * for 2*m entries are outputs; the arc count is row_ptr[n].  Ids outside
 * [0, n) are a device-side fault (HLN_EDEVICE at hln_device_status) and
 * leave the outputs unspecified.  n >= 1, 0 <= m <= 2^30. */
size_t hln_csr_from_edges_workspace_size(int32_t n, int64_t m);
hln_status hln_csr_from_edges(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                              int32_t* row_ptr, int32_t* col_idx,
                              void* workspace, size_t workspace_bytes, void* stream);

/* hln_csr_from_edges_batch: hln_csr_from_edges of `count` edge lists in one
 * set of launches (many small layers, e.g. the layers of many HoMLNs, at
 * the cost of one large one).  lists [host] array of count descriptors; each
 * list's outputs are exactly those of hln_csr_from_edges on it, under the
 * same rules (n >= 1, 0 <= m <= 2^30, row_ptr always, eu / ev / col_idx when
 * m > 0; ids outside [0, n) a device-side fault).  The totals sum(2 m) and
 * sum(n + 1) must stay below 2^31 - 1 (HLN_EUNSUPPORTED: split the batch).
 * Nothing is staged on the host, so the call can be captured into a
 * hipGraph; the lists' outputs must not overlap.  count = 0 does nothing.
 * The workspace size reads only n and m (0 for invalid sizes). */
typedef struct {
    int32_t n;
    int64_t m;
    const int32_t* eu;     /* [dev] m */
    const int32_t* ev;     /* [dev] m */
    int32_t* row_ptr;      /* [dev] n + 1, output */
    int32_t* col_idx;      /* [dev] room for 2 m, output */
} hln_edge_list;
size_t hln_csr_from_edges_batch_workspace_size(const hln_edge_list* lists, int32_t count);
hln_status hln_csr_from_edges_batch(const hln_edge_list* lists, int32_t count, void* workspace,
                                    size_t workspace_bytes, void* stream);

/* hln_csr_validate: checks the CSR conventions on the device and writes a
 * bit mask to *result [dev] (0 = valid): 1 row_ptr not monotone or
 * row_ptr[0] != 0 or row_ptr[n] != nnz, 2 id out of range, 4 row not
 * strictly ascending (duplicate or unsorted), 8 self-loop, 16 asymmetric
 * (arc u->v without v->u). */
hln_status hln_csr_validate(const hln_csr* g, int32_t* result, void* stream);

/* ------------------------------------------------------------------------
 * Boolean aggregation of r layers (Sec. 3.1; ground truth, Sec. 4).
 * ------------------------------------------------------------------------
 * AND keeps an edge present in every layer, OR one present in at least one
 * layer.  layers [host] array of r graphs with equal n; out_row_ptr [dev]
 * n+1, out_col_idx [dev] with `capacity` entries; the arc count is
 * out_row_ptr[n].  capacity must be >= min nnz (AND) or >= sum nnz (OR),
 * else HLN_ENOMEM.  1 <= r <= 64. */
size_t hln_compose_workspace_size(const hln_csr* layers, int32_t r);   /* 0 on bad arguments */
hln_status hln_compose_and(const hln_csr* layers, int32_t r, int32_t* out_row_ptr, int32_t* out_col_idx,
                           int64_t capacity, void* workspace, size_t workspace_bytes, void* stream);
hln_status hln_compose_or(const hln_csr* layers, int32_t r, int32_t* out_row_ptr, int32_t* out_col_idx,
                          int64_t capacity, void* workspace, size_t workspace_bytes, void* stream);

/* hln_compose_and_batch: hln_compose_and of `count` problems in one set of
 * launches (e.g. the AND aggregates of many HoMLNs, or of every layer subset
 * of one); each problem's outputs are exactly those of the one-problem call,
 * under its rules (1 <= r <= 64 layers of equal n, capacity >= the smallest
 * layer's nnz, else HLN_ENOMEM naming the problem).  problems [host];
 * layers [host] per problem.  The problem and layer tables are written by
 * kernels from their launch arguments, so nothing is staged on the host and
 * the call can be captured.  The sums of the smallest layers' nnz and of
 * n + 1 must stay below 2^31 - 1 (HLN_EUNSUPPORTED).  count = 0 does
 * nothing; the workspace size checks the layers as the call does (0 when a
 * problem is invalid) but not the outputs or capacities. */
typedef struct {
    int32_t r;
    const hln_csr* layers;     /* [host] r graphs */
    int32_t* out_row_ptr;      /* [dev] n + 1, output */
    int32_t* out_col_idx;      /* [dev] capacity, output */
    int64_t capacity;
} hln_and_problem;
size_t hln_compose_and_batch_workspace_size(const hln_and_problem* problems, int32_t count);
hln_status hln_compose_and_batch(const hln_and_problem* problems, int32_t count, void* workspace,
                                 size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Exact closeness of one graph (Sec. 4, Eq. 1 with the Wasserman-Faust
 * normalisation used for disconnected graphs; one BFS per source).
 * ------------------------------------------------------------------------
 * sources [dev] NULL: every vertex is a source and the outputs are indexed
 *   by vertex (n_src must equal n), or, with n_src = 0, an empty list.
 *   Otherwise n_src distinct vertex ids and the outputs are indexed by
 *   position in `sources`.
 * S  [dev] int64: sum of hop distances to the reachable vertices.
 * R  [dev] int32: number of reachable vertices, the source included.
 * cc [dev] double, nullable: ((R-1)/S) * ((R-1)/(n-1)) rounded in that
 *   order (IEEE division), 0 when R <= 1 or n <= 1.
 * h2 [dev] int32, nullable: vertices at distance exactly 2 (all-source
 *   mode only; HLN_EUNSUPPORTED with listed sources).
 * opts [host] nullable (defaults).  0 <= n_src; n >= 1.
 * opts->flags = HLN_FLAG_PER_VERTEX (listed sources only; cc and h2 must be
 *   NULL): the outputs are indexed by vertex (n entries) and hold sums over
 *   the listed sources, S[v] = sum of d(s, v) over listed s reaching v and
 *   R[v] = how many listed s reach v (v itself when listed; a repeated id
 *   counts each time).  n_src = 0 writes zeros (sources may then be NULL).
 *   These are the sample sums
 *   hln_closeness_estimate takes. */
size_t hln_closeness_workspace_size(int32_t n, int64_t nnz, int32_t n_src, const hln_opts* opts);
hln_status hln_closeness_layer(const hln_csr* g, const int32_t* sources, int32_t n_src, const hln_opts* opts,
                               int64_t* S, int32_t* R, double* cc, int32_t* h2,
                               void* workspace, size_t workspace_bytes, void* stream);

/* hln_closeness_layer_static: hln_closeness_layer without a workspace, for
 * callers that cannot allocate device memory (code under hipGraph capture,
 * serving loops, harnesses that forbid allocation).  Arguments, outputs
 * and errors as hln_closeness_layer, same kernels and results.  Its scratch
 * is one library-owned array of HLN_STATIC_SCRATCH_BYTES per device, held
 * from the library's first use on that device until the process ends; a
 * graph whose hln_closeness_workspace_size exceeds it is HLN_ENOMEM (64 MiB
 * holds, e.g., n = 10^5 vertices with 10^6 arcs at 512 sources per batch;
 * 4096 sources never fit).  Every call on a device shares that device's
 * array and the kernels clear what they use, so calls in stream order are
 * independent, but calls that can overlap on one device (different
 * streams, different host threads) race and must not be issued.  Nothing is
 * allocated: the array's address is looked up once per device. */
#define HLN_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
hln_status hln_closeness_layer_static(const hln_csr* g, const int32_t* sources, int32_t n_src, const hln_opts* opts,
                                      int64_t* S, int32_t* R, double* cc, int32_t* h2, void* stream);

/* ------------------------------------------------------------------------
 * Sampling estimate of every vertex's closeness (Sec. 2: the sampling
 * approximations of closeness it cites, Eppstein-Wang and Cohen et al.).
 * ------------------------------------------------------------------------
 * S, R [dev] n entries: the per-vertex sums of a sample of k distinct
 *   sources (hln_closeness_layer with HLN_FLAG_PER_VERTEX over the same
 *   list); sources [dev] k ids, the sample, drawn uniformly from a
 *   population of n_pop vertices (vertices outside it are taken to reach
 *   none of it).
 * cc [dev] double, n entries, output.  With q = R[v] - [v sampled] and
 *   k' = k - [v sampled]:
 *     cc[v] = (q / S[v]) * (q / k') * ((n_pop - 1) / (n - 1)),
 *   rounded in that order (IEEE division), 0 when q = 0, S[v] = 0, k' = 0
 *   or n = 1.  A sample of every vertex (k = n_pop = n) gives the exact
 *   closeness of hln_closeness_layer bit for bit.
 * 1 <= n, 1 <= n_pop <= n, 0 <= k <= n_pop, else HLN_EINVAL.  A sample id
 * outside [0, n) is a device-side fault (HLN_EDEVICE at hln_device_status).
 * No workspace; cc may not alias S or R. */
hln_status hln_closeness_estimate(int32_t n, int32_t n_pop, const int32_t* sources, int32_t k,
                                  const int64_t* S, const int32_t* R, double* cc, void* stream);

/* ------------------------------------------------------------------------
 * CC-node selection and composition (Theta step).
 * ------------------------------------------------------------------------
 * HLN_RANK_WF    r = 1: score = the graph's closeness (Sec. 4, Eq. 1 in the
 *                Wasserman-Faust form) from its S and R.
 * HLN_RANK_CC2   r >= 1 layers: est(u) = max over layers of S + n*(n - R),
 *                the distance sum with unreachable vertices at distance n
 *                (Sec. 5.1); score = (n-1)/est (Sec. 5.2, Algorithm 1, then
 *                Eq. 1); ranking by est ascending is the same order.
 * HLN_RANK_NAIVE r >= 1 layers: the naive composition (Sec. 4), the
 *                intersection of the layers' CC-node sets: their above-
 *                average sets (k = -1) or their top-k sets by each layer's
 *                closeness, ties by ascending id (k >= 0).  Either way ids
 *                ascending, score 0.0, count = the intersection's size
 *                (at most k when k >= 0).
 * S, R [host] arrays of r device pointers to the layers' all-source outputs
 * of hln_closeness_layer (n entries each).
 * k >= 0 (HLN_RANK_WF, HLN_RANK_CC2): ids [dev] the k best vertices (score
 *   descending, ties by ascending id, Sec. 5.2 "top-k"), score [dev,
 *   nullable] their scores.  mode | HLN_TOPK_SET: the same k vertices and
 *   scores in ascending id order (the top-k as a set).  HLN_RANK_NAIVE with k >= 0: see above; ids and
 *   score need room for k entries.
 * k = -1: every vertex whose score is >= the mean score (Sec. 4: "same or
 *   above average"), ids ascending; the mean is the sum over ids taken
 *   sequentially in chunks of 1024, chunk sums added in order, divided by n.
 *   ids and score need room for n entries.
 * count [dev] int32: number of ids written.  0 <= k <= n or k = -1. */
typedef enum { HLN_RANK_WF = 0, HLN_RANK_CC2 = 1, HLN_RANK_NAIVE = 2 } hln_rank_mode;
/* Flag OR-ed into a top-k mode (hln_compose_cc_topk) or score dtype
 * (hln_topk): return the k best as ascending ids instead of rank order. */
#define HLN_TOPK_SET 0x100
size_t hln_compose_cc_topk_workspace_size(int32_t n);
hln_status hln_compose_cc_topk(int32_t mode, int32_t n, int32_t r, const int64_t* const* S, const int32_t* const* R,
                               int32_t k, int32_t* ids, double* score, int32_t* count,
                               void* workspace, size_t workspace_bytes, void* stream);

/* hln_compose_cc_topk_batch: the k >= 0 form of hln_compose_cc_topk for
 * `count` problems in one set of launches (e.g. the CC2 top-k of many
 * HoMLNs); each problem's ids, score and count are exactly those of the
 * one-problem call.  mode HLN_RANK_WF (r = 1) or HLN_RANK_CC2, 1 <= r <= 64,
 * 0 <= k <= n, S / R as there.  The keys of all problems go through one
 * segmented radix sort; the problem table is written by kernels from their
 * launch arguments, so nothing is staged on the host and the call can be
 * captured.  sum(n) must stay below 2^31 - 1 (HLN_EUNSUPPORTED: split the
 * batch).  count = 0 does nothing.  The workspace size reads only mode, n,
 * r and k (0 for invalid problems). */
typedef struct {
    int32_t mode, n, r, k;
    const int64_t* const* S;   /* [host] r device pointers (n entries each) */
    const int32_t* const* R;   /* [host] r device pointers */
    int32_t* ids;              /* [dev] k, output */
    double* score;             /* [dev] k, output, nullable */
    int32_t* count;            /* [dev] 1, output (= k) */
} hln_topk_problem;
size_t hln_compose_cc_topk_batch_workspace_size(const hln_topk_problem* problems, int32_t count);
hln_status hln_compose_cc_topk_batch(const hln_topk_problem* problems, int32_t count, void* workspace,
                                     size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Heuristic CC1 (Sec. 5.1, Eq. 2-3): CC nodes of the AND aggregate of r
 * layers from per-layer degrees, penalised distance sums and neighbour
 * lists.  The paper describes CC1 in words; readings:
 *   ratio_l(u) = (S_l + n(n - R_l))(u) / m(u), m(u) = smallest degree of u
 *     over the layers (Eq. 2); no ratio when m(u) = 0;
 *   avg_l = mean of ratio_l over the vertices with m > 0 (fixed summation
 *     shape: chunks of 1024 ids, chunk sums in order); avg = max_l avg_l
 *     (Eq. 3);
 *   v is central in layer l when m(v) > 0 and ratio_l(v) < avg;
 *   a vertex c in every layer's above-average closeness set (Sec. 4) is kept
 *     when, with C_l(c) = central neighbours of c in layer l, I = their
 *     intersection and s = min_l |C_l(c)|: s > 0 and
 *     |I| * tau_den >= tau_num * s ("significant overlap"; the paper gives
 *     no threshold, tau = 1/2 is this library's default in the bindings).
 * layers [host] r graphs with equal n (CSR conventions); S, R [host] arrays
 * of r device pointers to the layers' all-source outputs of
 * hln_closeness_layer.  ids [dev] room for n entries, written ascending;
 * count [dev] int32; avg [dev, nullable] double: Eq. 3's value.
 * 1 <= r <= 64, tau_num >= 0, tau_den >= 1, else HLN_EINVAL. */
size_t hln_compose_cc1_workspace_size(int32_t n, int32_t r);   /* 0 on bad arguments */
hln_status hln_compose_cc1(const hln_csr* layers, int32_t r, const int64_t* const* S, const int32_t* const* R,
                           int32_t tau_num, int32_t tau_den, int32_t* ids, int32_t* count, double* avg,
                           void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched closeness of many graphs (Sec. 3: every layer is analysed
 * independently and in parallel; the Problem Statement, Sec. 1: the layers
 * and any aggregates of many HoMLNs, each with all of its vertices or a
 * list of them as sources, through one persistent launch per source-width
 * class and accumulation mode).
 * ------------------------------------------------------------------------
 * A plan is an opaque host object: tuned source widths per graph-size class,
 * pinned staging for the per-call descriptors, and optionally one captured
 * hipGraph of a whole batch.  Plans are not thread-safe; destroy with
 * hln_plan_destroy (waits for its staging copies).
 * sources [host] NULL (every graph uses all its vertices as sources; n_src
 *   may be NULL) or an array of n_graphs device pointers read with n_src
 *   [host] n_graphs int32: n_src[g] = -1 for all of graph g's vertices
 *   (sources[g] is not read), else 0 <= n_src[g] <= n distinct vertex ids
 *   of graph g at sources[g] (NULL allowed when n_src[g] = 0; ids outside
 *   [0, n) are a device-side fault).  The count decides, not the pointer.
 * S[g], R[g], cc[g], h2[g]: host arrays of n_graphs device pointers.  All-
 *   source graphs: n_g entries indexed by vertex, as hln_closeness_layer's
 *   all-source mode.  Listed graphs: n_src[g] entries indexed by position
 *   in sources[g], as hln_closeness_layer with listed sources; h2[g] must be
 *   NULL (HLN_EUNSUPPORTED); n_src[g] = 0 writes nothing.  cc and h2 (arrays
 *   or entries) nullable.
 * All-source graphs with n <= 65535 can run as LDS tiles (one workgroup
 * keeps the frontier, next and visited bitsets of the whole graph in LDS);
 * larger graphs, graphs the tuner assigns to it and every listed graph run
 * through the persistent kernel inside the same call: one cooperative launch
 * per (width, mode), its grid cut into partitions (up to 4; one when a graph
 * of the launch has more than 65,536 vertices) that run different graphs at
 * once.  A listed graph takes its size class's tuned persistent width, else
 * the narrowest of 512, 1024, 2048, 4096 holding all its sources.
 * hln_plan_tune times, for each log2(n) class present, the class's largest
 * graph with every LDS tile width that fits (64/32/16/8 bits per vertex)
 * and with the persistent kernel at 1024, 2048 and 4096 sources, and keeps
 * the fastest; it synchronises `stream` and overwrites that graph's S and
 * R.  hln_plan_width reports the width an all-source graph of n vertices
 * gets (untuned: the widest fitting tile, else 4096).  hln_plan_set_width
 * sets the choice of n's log2 class by hand (a tuned plan saved and
 * restored, or two plans made to agree): 8, 16, 32 or 64 for LDS tiles
 * (narrowed to the widest that fits a graph, the persistent kernel at 4096
 * where none does), 512, 1024, 2048 or 4096 for the persistent kernel, 0
 * for the untuned default; any other width is HLN_EINVAL and changes
 * nothing.
 * hln_plan_capture records the whole batch (staging copy, preparation,
 * tile launches, closeness pass) into a hipGraph owned by the plan, which
 * hln_plan_replay launches on `stream`; the captured buffers must stay
 * valid while replays are possible.  Capture needs a non-null stream.
 * hln_closeness_batch may also be called while the caller captures
 * `stream` into a graph of its own: call hln_plan_reserve for the same
 * graphs before each such capture.  It sets aside the pinned staging that
 * the captured copy reads at every replay; the capture keeps that buffer
 * until the plan is destroyed, so graphs captured earlier stay valid.  A
 * capture without a reserved buffer is HLN_EINVAL. */
typedef struct hln_plan hln_plan;
hln_status hln_plan_create(hln_plan** plan);
void hln_plan_destroy(hln_plan* plan);
int32_t hln_plan_width(const hln_plan* plan, int32_t n);
hln_status hln_plan_set_width(hln_plan* plan, int32_t n, int32_t width);
size_t hln_closeness_batch_workspace_size(const hln_plan* plan, const hln_csr* graphs, int32_t n_graphs);
hln_status hln_closeness_batch(hln_plan* plan, const hln_csr* graphs, int32_t n_graphs,
                               const int32_t* const* sources, const int32_t* n_src, int64_t* const* S,
                               int32_t* const* R, double* const* cc, int32_t* const* h2,
                               void* workspace, size_t workspace_bytes, void* stream);
hln_status hln_plan_tune(hln_plan* plan, const hln_csr* graphs, int32_t n_graphs, int64_t* const* S,
                         int32_t* const* R, void* workspace, size_t workspace_bytes, void* stream);
hln_status hln_plan_capture(hln_plan* plan, const hln_csr* graphs, int32_t n_graphs,
                            const int32_t* const* sources, const int32_t* n_src, int64_t* const* S,
                            int32_t* const* R, double* const* cc, int32_t* const* h2,
                            void* workspace, size_t workspace_bytes, void* stream);
hln_status hln_plan_reserve(hln_plan* plan, const hln_csr* graphs, int32_t n_graphs);
hln_status hln_plan_replay(hln_plan* plan, void* stream);
/* Persistent launches of the plan's last enqueue (hln_closeness_batch,
 * hln_plan_capture or a tuning run): how many went out as cooperative
 * launches and how many as ordinary kernel nodes inside a stream capture
 * (see hln_last_launch_path).  cooperative, ordinary [host]. */
hln_status hln_plan_launch_paths(const hln_plan* plan, int32_t* cooperative, int32_t* ordinary);

/* ------------------------------------------------------------------------
 * Learned candidate proposer (not in the paper; its inputs are the Psi
 * step's per-layer outputs: degree, closeness and 2-hop count, echoing
 * CC1's degree bound, Sec. 5.1, and CC2's per-layer sums, Sec. 5.2).
 * ------------------------------------------------------------------------
 * hln_proposer_features: X [dev] float[n][12]; for each of three per-layer
 *   quantities -- log1p(deg / mean degree of the layer), the closeness
 *   ((R-1)/S)((R-1)/(n-1)) and log1p(h2 / mean degree^2) -- the min, max,
 *   mean and standard deviation over the r layers.  row_ptr, S, R, h2:
 *   [host] arrays of r device pointers (n+1, n, n, n entries; S, R, h2 as
 *   hln_closeness_layer's all-source outputs); nnz [host] r exact arc
 *   counts.  1 <= r <= 64.
 * The MLP is 12 -> 64 (ReLU) -> 64 (ReLU) -> 1 in FP32 with
 *   hln_mlp_param_count() parameters in the order W1[12][64], b1[64],
 *   W2[64][64], b2[64], w3[64], b3 (params [dev] float).
 * hln_mlp_init: Glorot-uniform weights from a counter-based generator
 *   (splitmix64 of seed and index), zero biases; zeroes adam_m / adam_v
 *   (nullable).
 * hln_mlp_forward: y [dev] float[n] scores for X.
 * hln_mlp_train_step: one Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8,
 *   bias-corrected with `step` >= 1) on the mean squared error of the n
 *   rows of X against target [dev] float[n]; *loss [dev, nullable] the loss
 *   before the step.  Deterministic (block partials summed in order).
 * hln_topk: ids [dev] of the k largest scores (float64 dtype 0, float32
 *   dtype 1), descending, ties by ascending index; -0.0 ties with +0.0;
 *   scores must not be NaN.  0 <= k <= n.  dtype | HLN_TOPK_SET: the same k
 *   ids written in ascending order (a candidate set whose later ranking
 *   breaks ties by position then breaks them by vertex id).
 * hln_rank_labels: label [dev] float[n] = log((n+1)/(g+1)) / log(n+1)
 *   with g the number of vertices with a strictly larger score (computed in
 *   double, rounded to float): the log-rank the proposer is trained to
 *   predict, 1 for the best vertex.  Both take hln_topk_workspace_size(n)
 *   bytes of workspace. */
int32_t hln_mlp_param_count(void);
hln_status hln_proposer_features(int32_t n, int32_t r, const int32_t* const* row_ptr, const int64_t* const* S,
                                 const int32_t* const* R, const int32_t* const* h2, const int64_t* nnz, float* X,
                                 void* stream);
hln_status hln_mlp_init(float* params, float* adam_m, float* adam_v, uint64_t seed, void* stream);
hln_status hln_mlp_forward(const float* params, const float* X, int32_t n, float* y, void* stream);
size_t hln_mlp_train_workspace_size(int32_t n);
hln_status hln_mlp_train_step(float* params, float* adam_m, float* adam_v, int32_t step, float lr, const float* X,
                              const float* target, int32_t n, float* loss, void* workspace, size_t workspace_bytes,
                              void* stream);
size_t hln_topk_workspace_size(int32_t n);
hln_status hln_topk(int32_t n, const void* score, int32_t dtype, int32_t k, int32_t* ids,
                    void* workspace, size_t workspace_bytes, void* stream);
hln_status hln_rank_labels(int32_t n, const void* score, int32_t dtype, float* label,
                           void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HLN_H */
