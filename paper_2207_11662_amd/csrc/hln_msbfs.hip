// Exact closeness of one graph by bit-parallel multi-source BFS (the Psi
// step of the decoupling method, Sec. 3; Sec. 4: one BFS from every vertex,
// Eq. 1 with the Wasserman-Faust normalisation for disconnected graphs).
//
// W = 64*NW sources run together; every vertex holds NW 64-bit words per
// bitset (vertex-major, so one vertex's W bits are contiguous):
//   vis  -- sources that have reached the vertex,
//   fr   -- sources that reached it at the previous level (the frontier),
//   nx   -- sources reaching it at this level.
// One level, bottom-up (pull):  nx[v] = (OR_{w in N(v)} fr[w]) & ~vis[v];
//   a lane stops gathering a word once vis | OR covers all 64 bits.
// One level, top-down (push): every segment of a frontier vertex u ORs
//   fr[u] into its neighbours' accumulators (agent-scope atomics) and marks
//   them touched; after a grid barrier the touched vertices are finalised
//   as in the pull case and the word masks of the older frontier cleared.
// A frontier word is read only where its vertex's word mask has the bit, so
// words outside the masks are never cleared.
// A level's new bits at v are the sources at distance d from v.
// Direction: every finalised vertex with new bits appends its segments to
// its block's frontier list in LDS and adds its arc-words (arcs times the
// frontier words holding new bits, which is what a push ORs) to a per-phase
// counter; a top-down level's blocks push their own lists.  A level runs
// top-down when alpha * (frontier arc-words) < arcs of the graph (after
// Beamer, Asanovic and Patterson, SC'12, with the bit-parallel frontier's
// word count in the cost) and no block's list overflowed; the barrier's
// releasing thread decides and every block receives the same bit.  With all
// sources at W = 4096 the automatic choice is bottom-up at every level
// (alpha = 0).
//
// Saturation: a vertex that holds every source bit it can ever receive in
// the batch gains nothing more, so later bottom-up levels skip its segments
// (no ids, flags or gathers).  What it can receive is judged against one
// component C: the component of the first batch's highest-degree source,
// marked exactly by that source's own bit after the first batch.  In later
// batches a vertex holding any of the batch's sources in C lies in C, and
// once it holds all of them no other source of the batch can reach it.
//
// Accumulation:
//   all sources (sources == NULL): the batches take the vertices that have
//     arcs (a vertex without arcs reaches only itself); the graph is
//     undirected, so d(s,v) = d(v,s) and the vertex v accumulates
//     S[v] += d*popc(new), R[v] += popc(new); after all n sources S[v], R[v]
//     are v's own sums.  H2[v] counts the new bits at d = 2.
// Batch order: the first batch takes the sources of the largest degree
// classes; the later ones by BFS distance from the first batch's hub, which
// that batch measures (a batch runs 1 + its sources' largest eccentricity
// levels, and vertices at one distance from a hub have close ones).
//   listed sources: per-source counts c_i(d) = #{v : bit i new at d} are
//     gathered per block in LDS and reduced over blocks at the batch end.
//   listed sources, per-vertex sums (HLN_FLAG_PER_VERTEX): as for all
//     sources, so S[v] and R[v] sum over the listed sources only (the sums
//     a sampling estimator of closeness needs); R[v] starts at 0 and every
//     listed occurrence of v adds 1.
//
// Execution: one cooperative persistent launch per call.  All batches and
// levels run inside it, separated by grid barriers with bounded waits; the
// direction of each level and the end of each BFS are decided on the device
// from counters of the previous level, so the host never synchronises.
//
// Load balance: rows are cut into segments of at most SEG arcs, ordered
// heavy-first and then by decreasing degree.  A group of LPV lanes
// processes one segment (NPAR = LPV/NW arcs at a time, one 64-bit word per
// lane).  A row with several segments merges its partial ORs with atomic OR
// into a per-vertex accumulator; the last segment to finish (atomic counter)
// finalises the vertex, so a hub never serialises a level.
#include "hln_internal.hpp"

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <cstdio>
#include <cstdlib>

namespace {

using hln::dev::load_agent_i32;
using hln::dev::shfl_xor_i32;
using hln::dev::shfl_xor_u64;
using hln::dev::store_agent_i32;

#ifndef HLN_GATHER_CHUNK
#define HLN_GATHER_CHUNK 8     // frontier gathers in flight per lane and chunk
#endif
#ifndef HLN_GATHER_CHUNK_W4096
#define HLN_GATHER_CHUNK_W4096 8    // the same at W = 4096 (one group per wave)
#endif

// Arcs per segment (the unit of work of a lane group; longer rows are split).
constexpr int kSegLen = 64;

// Frontier gathers use raw buffer loads: 32-bit byte offsets (one VALU
// operation per address) and an out-of-range offset for a lane that needs no
// word, which returns zero without a memory access.  The host guarantees
// that a bitset is smaller than 2^31 bytes.
typedef unsigned int hln_u32x2 __attribute__((ext_vector_type(2)));
constexpr uint32_t kNoWord = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t words_rsrc(const uint64_t* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint64_t*>(p), static_cast<short>(0), static_cast<int>(bytes),
                                             0x00020000);
}

__device__ __forceinline__ uint32_t buf_u32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

__device__ __forceinline__ int4 buf_i4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return make_int4(static_cast<int>(x.x), static_cast<int>(x.y), static_cast<int>(x.z), static_cast<int>(x.w));
}

__device__ __forceinline__ void buf_store_u64(uint64_t x, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    hln_u32x2 v;
    v.x = static_cast<uint32_t>(x);
    v.y = static_cast<uint32_t>(x >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
}

// The same store written through to the device coherence point (cache
// policy sc0 sc1), so the L2 write-back at the next grid barrier has less to
// flush.  Used for the finaliser's next-frontier and visited words (+1% on
// config 2); for the word masks it measured slower, and non-temporal stores
// slower still (-5%).
__device__ __forceinline__ void buf_store_u64_wt(uint64_t x, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    hln_u32x2 v;
    v.x = static_cast<uint32_t>(x);
    v.y = static_cast<uint32_t>(x >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 17);
}

__device__ __forceinline__ void buf_store_u32(uint32_t x, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(x, r, off, 0, 0);
}

__device__ __forceinline__ void buf_add_u32(uint32_t x, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    (void)__builtin_amdgcn_raw_ptr_buffer_atomic_add_i32(static_cast<int>(x), r, off, 0, 0);
}

// Per-lane select by a wave-wide lane mask (bit i of `lanes` picks lane i):
// one v_cndmask with the mask in an SGPR pair.
__device__ __forceinline__ uint32_t select_lanes(uint64_t lanes, uint32_t if_set, uint32_t if_clear) {
    uint32_t r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(if_clear), "v"(if_set), "s"(lanes));
    return r;
}

__device__ __forceinline__ uint64_t buf_word(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const hln_u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    return (static_cast<uint64_t>(v.y) << 32) | v.x;
}

// Value of lane gbase + j of the group for every lane of the group; j is
// uniform over the group.  A group of 64 lanes is the wave: one readlane.
template <int LPV>
__device__ __forceinline__ int group_bcast(int x, int gbase, int j) {
    if constexpr (LPV == 64) return __builtin_amdgcn_readlane(x, j);
    else return __shfl(x, gbase + j, 64);
}

// Sum of x over the 64 lanes of the wave, in every lane: DPP adds within
// each row of 16 lanes (quad swaps, then rotations by 4 and 8), then the four
// row totals read from lanes 0, 16, 32 and 48.  Every lane must be active.
__device__ __forceinline__ int wave_sum_i32(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
    x += __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
    x += __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false);   // row_ror:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);   // row_ror:8
    return __builtin_amdgcn_readlane(x, 0) + __builtin_amdgcn_readlane(x, 16) + __builtin_amdgcn_readlane(x, 32) +
           __builtin_amdgcn_readlane(x, 48);
}

// Sum of x over each aligned group of LPV lanes (8, 16 or 32), in every
// lane of the group: DPP quad swaps, then the half-row mirror (8 lanes), the
// row mirror (16) and one cross-row exchange (32).
template <int LPV>
__device__ __forceinline__ int group_sum_i32(int x) {
    static_assert(LPV == 8 || LPV == 16 || LPV == 32, "group of 8, 16 or 32 lanes");
    x += __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
    x += __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
    x += __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false);   // row_half_mirror
    if constexpr (LPV >= 16) x += __builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false);   // row_mirror
    if constexpr (LPV >= 32) x += __shfl_xor(x, 16, 64);
    return x;
}

// Word masks of a frontier buffer: bit k set when word k of a vertex may be
// nonzero (32-bit for up to 32 words, 64-bit for 64).
template <int NW>
using MaskT = typename std::conditional<(NW > 32), unsigned long long, uint32_t>::type;

template <class M>
__device__ __forceinline__ M shfl_mask(M x, int lane) {
    if constexpr (sizeof(M) == 8) {
        const int lo = __shfl(static_cast<int>(static_cast<uint32_t>(x)), lane, 64);
        const int hi = __shfl(static_cast<int>(static_cast<uint32_t>(x >> 32)), lane, 64);
        return (static_cast<M>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
    } else {
        return static_cast<M>(__shfl(static_cast<int>(x), lane, 64));
    }
}

template <class M>
__device__ __forceinline__ M buf_mask(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (sizeof(M) == 8) return buf_word(r, off);
    else return buf_u32(r, off);
}

template <class M>
__device__ __forceinline__ void buf_store_mask(M x, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (sizeof(M) == 8) buf_store_u64(x, r, off);
    else buf_store_u32(x, r, off);
}

// lanes per group (one segment at a time): 8, or NW when NW > 8
template <int NW>
constexpr int lpv() { return NW > 8 ? NW : 8; }
constexpr int kMinLpv = 8;
constexpr int kClasses = 40;

// Every word here is read and written with agent-scope atomics only; the
// barrier counter sits alone on its cache line.
struct Ctrl {
    int bins[kClasses];                    // segments per class
    int cursor[kClasses];                  // fill cursors (segment units)
    int n_seg;
    int fbad[3];                           // nonzero: a block's frontier list overflowed (slot = phase mod 3)
    unsigned long long farcs[3];           // frontier arc-words of the same phases
    unsigned long long probe_key;          // first batch's probe source: degree << 32 | ~position (max)
    unsigned long long gcm[64];            // this batch's sources in the largest component (bit per source)
    int n_act;                        // all sources: vertices with arcs
};

// LDS frontier-list entries per block and phase; a phase that lists more in
// one block makes the next level bottom-up (such a frontier is far past the
// top-down threshold anyway).
constexpr int kFlCap = 4096;
// Degree classes that order the all-source batches (segments of 64 arcs:
// class 0 holds rows longer than a segment, class 7 rows of one arc).
constexpr int kRankClasses = 8;

struct BfsArgs {
    int32_t n;
    int32_t n_src;                    // number of sources (n when sources == nullptr)
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const int32_t* sources;           // nullptr: all vertices, per-vertex accumulation
    int listed;                       // sources come from the list (it may be empty)
    uint64_t* bufA;                   // n*NW
    uint64_t* bufB;                   // n*NW
    void* flagA;                      // n word masks (MaskT<NW>): bufA word k of v is read only when bit k is set
    void* flagB;                      // n: the same for bufB
    uint64_t* vis;                    // n*NW
    uint64_t* hacc;                   // n*NW partial ORs of multi-segment rows (kept zero)
    int32_t* hcnt;                    // n finished-segment counters (kept zero)
    int4* seg;                        // segments: vertex, first arc, end arc, segments of the row
    long long seg_cap;                // capacity of seg
    long long nnz_cap;                // arcs the caller declared (col_idx holds at least row_ptr[n] <= nnz_cap)
    int32_t* seg_first;               // n: index of the vertex's first segment
    uint32_t* segsat;                 // seg_cap: the level at which the segment's vertex came to hold every bit it
                                      // can get in the batch (0: not yet)
    uint32_t* member;                 // n: 1 when the vertex lies in the probe source's component
    int64_t* part;                    // per-source mode: [grid][2][W] block partials
    int64_t* S;
    uint32_t* S32;                    // n: distance sums since the last fold (levels below kS32Levels), folded into S
    int32_t* R;
    int32_t* H2;
    double* cc;
    Ctrl* ctrl;
    unsigned long long* bar;          // grid barrier words (hln::dev::kBarrierWords)
    int* fault;
    uint64_t wait_ticks;              // bound of one barrier wait (s_memrealtime ticks)
    int32_t direction;                // 0 auto, 1 top-down only, 2 bottom-up only
    int32_t seg_len;                  // SEG
    int32_t* levels;                  // nullable: levels run per batch
    int64_t* trace;                   // nullable: per level {ticks, vertices with new bits, new pairs, direction}
    int32_t trace_cap;
    int32_t alpha;                    // top-down when alpha * frontier arc-words < arcs of the graph (0: never)
    int32_t* perm;                    // all sources: the vertices with arcs, in id order (the batches' sources)
    int32_t* iperm;                   // all sources: a vertex's position in perm, -1 without arcs
    int32_t* bcount;                  // all sources: vertices with arcs per block range and degree class
    int32_t s32_levels;               // depth from which distance sums go to S with 64-bit atomics
};

// Levels from this depth on add to S directly (64-bit atomics): below it a
// batch's sum per vertex is at most W * depth < 2^32.  (HLN_S32_LEVELS
// lowers it, so that tests reach the 64-bit path on small graphs.)
constexpr int kS32Levels = 1 << 18;

// Buffer resources of one level.  Loads and stores of the pull loop and the
// finaliser go through them with an out-of-range offset for lanes that need
// no access: such a load reads zero and such a store or atomic is dropped,
// so every instruction issues on every path and the loop's memory counter
// waits stay exact (stores count in the same in-order counter as loads).
struct LevelBufs {
    __amdgpu_buffer_rsrc_t nx, vis, flag_nx, flag_fr, s32, r, h2, col, seg, segsat;
};

// A block's frontier lists in LDS, double-buffered by phase parity: the
// vertices its groups finalised with new bits, as segment indices.
struct FrontierLds {
    int32_t fl[2][kFlCap];
    int cnt[2];
    unsigned long long arcs[2];
};

// Record that a vertex got new bits: its segments [first, first + nseg)
// join the list of parity `par`.  Called by one lane.
__device__ __forceinline__ void frontier_note(FrontierLds& f, int par, int first, int nseg, int arcs) {
    atomicAdd(&f.arcs[par], static_cast<unsigned long long>(arcs));
    const int p = atomicAdd(&f.cnt[par], nseg);
    if (p + nseg <= kFlCap)
        for (int j = 0; j < nseg; ++j) f.fl[par][p + j] = first + j;
}

// Barrier hooks at the end of a phase.  PhaseEnd (each block's thread 0,
// block synchronised): adds the block's frontier arcs to the phase's
// counter, flags an overflowed list and clears the other parity's list for
// the next phase (the previous phase's list was last read before this
// barrier).  Decide (the releasing thread): the direction of the next level.
struct PhaseEnd {
    FrontierLds* f;
    Ctrl* ctrl;
    int phase;
    bool on;                              // false: no level can run top-down, the lists are not kept
    __device__ void operator()() const {
        if (!on) return;
        const int par = phase & 1;
        const int slot = phase % 3;
        if (f->arcs[par]) hln::dev::atomic_add_agent(&ctrl->farcs[slot], f->arcs[par]);
        if (f->cnt[par] > kFlCap) store_agent_i32(&ctrl->fbad[slot], 1);
        f->cnt[par ^ 1] = 0;
        f->arcs[par ^ 1] = 0;
    }
};

struct Decide {
    Ctrl* ctrl;
    long long m_arcs;
    int direction;
    int alpha;
    int phase;
    __device__ bool operator()() const {
        const int slot = phase % 3;
        if (direction == 2 || alpha == 0 || load_agent_i32(&ctrl->fbad[slot]) != 0) return false;
        if (direction == 1) return true;
        const unsigned long long arcs = hln::dev::load_agent(&ctrl->farcs[slot]);
        return static_cast<long long>(arcs) * alpha < m_arcs;
    }
};

// Segments of vertex v, for the list: (first index, count, arcs).
__device__ __forceinline__ int3 vertex_segments(const BfsArgs& a, int v) {
    const int deg = a.row_ptr[v + 1] - a.row_ptr[v];
    return make_int3(a.seg_first[v], (deg + a.seg_len - 1) / a.seg_len, deg);
}

__device__ __forceinline__ int seg_class(int deg, int seg_len) {
    if (deg > seg_len) return 0;
    int lg = 31 - __clz(deg);                 // floor(log2 deg), deg >= 1
    int top = 31 - __clz(seg_len);
    return 1 + (top - lg);                    // larger degree first
}

__device__ __forceinline__ int trace_add(int64_t* row, int verts, long long pairs) {
    atomicAdd(reinterpret_cast<unsigned long long*>(row + 1), static_cast<unsigned long long>(verts));
    atomicAdd(reinterpret_cast<unsigned long long*>(row + 2), static_cast<unsigned long long>(pairs));
    return 0;
}

// Finalise vertex v at level d: new bits, bitset updates, accumulation.
// Called by the lanes of a group with the group's full OR in `acc` (lane
// (sub, k) holds word k; only sub == 0 lanes write).  Returns the number of
// new bits, the number of words holding them, and whether the vertex is now
// saturated: `gcm_k` is word k of the batch's sources that lie in one
// component C (that of the first batch's probe source); a vertex holding one
// of them lies in C, and once it holds all of them no other source of the
// batch can ever reach it, so it can gain nothing more in this batch.
// vis_all: every visited word is stored, not only those with new bits (the
// first level of a batch whose start did not clear the visited bitset).
template <int NW, bool PER_SOURCE>
__device__ __forceinline__ int3 finalize_vertex(const BfsArgs& a, const LevelBufs& B, int v, int d, int k, int sub,
                                                int gl, int gbase, uint64_t acc, uint64_t vis_v, int32_t* s_cnt,
                                                MaskT<NW> flag_old, uint64_t gcm_k, bool vis_all = false) {
    using Mask = MaskT<NW>;
    constexpr int LPV = lpv<NW>();
    constexpr Mask kWordMask = static_cast<Mask>(NW >= 64 ? ~0ull : ((1ull << (NW & 63)) - 1ull));
    const uint32_t woff = (static_cast<uint32_t>(v) * NW + static_cast<uint32_t>(k)) * 8u;
    const uint64_t nw = acc & ~vis_v;
    // lanes with sub == 0 hold word k at group lane k
    const Mask nmask = static_cast<Mask>((__ballot(sub == 0 && nw != 0) >> gbase) & kWordMask);
    int c = sub == 0 ? __popcll(nw) : 0;
    if constexpr (LPV == 64) c = wave_sum_i32(c);
    else c = group_sum_i32<LPV>(c);
    // new bits go to the next frontier; words without new bits keep whatever
    // they held, as the word mask (exact, stored below when it changes) keeps
    // every reader off them
    buf_store_u64_wt(nw, B.nx, (sub == 0 && nw != 0) ? woff : kNoWord);
    buf_store_u64_wt(vis_v | nw, B.vis, (sub == 0 && (nw != 0 || vis_all)) ? woff : kNoWord);
    if (PER_SOURCE && sub == 0 && nw) {
        uint64_t b = nw;
        while (b) {
            const int bit = __ffsll(static_cast<long long>(b)) - 1;
            b &= b - 1;
            atomicAdd(&s_cnt[k * 64 + bit], 1);
        }
    }
    const uint32_t voff = static_cast<uint32_t>(v);
    buf_store_mask<Mask>(nmask, B.flag_nx, (gl == 0 && nmask != flag_old) ? voff * static_cast<uint32_t>(sizeof(Mask))
                                                                          : kNoWord);
    if (!PER_SOURCE) {
        // one finaliser per vertex and level: non-returning adds need no old
        // values in flight
        const uint32_t aoff = (gl == 0 && c != 0) ? voff * 4u : kNoWord;
        if (d < a.s32_levels) {
            buf_add_u32(static_cast<uint32_t>(d) * static_cast<uint32_t>(c), B.s32, aoff);
        } else if (gl == 0 && c != 0) {
            __hip_atomic_fetch_add(reinterpret_cast<unsigned long long*>(&a.S[v]),
                                   static_cast<unsigned long long>(static_cast<int64_t>(d) * c), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        buf_add_u32(static_cast<uint32_t>(c), B.r, aoff);
        if (d == 2 && a.H2) buf_add_u32(static_cast<uint32_t>(c), B.h2, aoff);
    }
    // saturation (lanes with sub != 0 hold copies and do not vote)
    const uint64_t have = (vis_v | nw) & gcm_k;
    const bool full_k = sub != 0 || have == gcm_k;
    constexpr unsigned long long kGroupMask = LPV >= 64 ? ~0ull : ((1ull << LPV) - 1ull);
    const bool in_gc = ((__ballot(sub == 0 && have != 0) >> gbase) & kGroupMask) != 0;
    const int sat = (c != 0 && in_gc && ((__ballot(full_k) >> gbase) & kGroupMask) == kGroupMask) ? 1 : 0;
    return make_int3(c, __popcll(static_cast<unsigned long long>(nmask)), sat);
}

// A vertex saturated at level d: its segments record d, and later pull
// levels of the batch read no ids, masks or frontier words for them (they
// only clear the vertex's stale next-frontier word masks; at W = 4096 they
// are left out altogether from level d + 3 on).  Called by the lanes of its
// group.
template <int LPV>
__device__ __forceinline__ void mark_saturated(const BfsArgs& a, int first, int nseg, int gl, int d) {
    for (int j = gl; j < nseg; j += LPV) a.segsat[first + j] = static_cast<uint32_t>(d);
}

// Gathering the frontier over a segment [lo, hi) for the word k of this
// lane.  The group's LPV lanes load LPV column ids per instruction (CH such
// chunks per round) and then every lane issues NW independent 8-byte
// gathers per chunk: lane (sub, k) takes the chunk's arcs sub, sub + NPAR,
// ... (NPAR = LPV / NW).
template <int NW>
struct Gather {
    static constexpr int LPV = lpv<NW>();
    static constexpr int NPAR = LPV / NW;
    static constexpr int CH = NW >= 16 ? 1 : 2;     // chunks of LPV arcs per round
    static constexpr int ROUND = CH * LPV;

    __device__ __forceinline__ static void load_ids(__amdgpu_buffer_rsrc_t col, int c, int hi, int gl,
                                                    int (&cid)[CH]) {
#pragma unroll
        for (int h = 0; h < CH; ++h) {
            const int e = c + h * LPV + gl;
            const uint32_t x = buf_u32(col, e < hi ? static_cast<uint32_t>(e) * 4u : kNoWord);
            cid[h] = e < hi ? static_cast<int>(x) : -1;
        }
    }

    // word masks of the neighbours' frontier slots (0 for no neighbour)
    using Mask = MaskT<NW>;
    __device__ __forceinline__ static void load_masks(__amdgpu_buffer_rsrc_t flag_fr, const int (&cid)[CH],
                                                      Mask (&msk)[CH]) {
#pragma unroll
        for (int h = 0; h < CH; ++h)
            msk[h] = buf_mask<Mask>(flag_fr, cid[h] >= 0 ? static_cast<uint32_t>(cid[h]) * static_cast<uint32_t>(sizeof(Mask))
                                                         : kNoWord);
    }

    // Gathers go out in wave-uniform chunks of K with no branch inside a
    // chunk, so a chunk's loads are all in flight before the first OR waits
    // for one: a lane whose arc is absent, whose neighbour's word is zero or
    // whose word is saturated (skip: vis | OR so far is all ones, so nothing
    // outside vis can be added) loads from an out-of-range offset, which
    // reads zero.  A chunk that no lane of the wave needs is skipped.  `cnt`
    // is the number of arcs of this round that belong to the group's
    // segment.
    static constexpr int T = NW * CH;                    // (chunk, t) steps per round
    static constexpr int KMAX = NW == 64 ? HLN_GATHER_CHUNK_W4096 : HLN_GATHER_CHUNK;
    static constexpr int K = T < KMAX ? T : KMAX;

    __device__ __forceinline__ static int steps_needed(int cnt) {
        if (cnt <= 0) return 0;
        return ((cnt - 1) / LPV) * NW + ((cnt - 1) % LPV) / NPAR + 1;
    }


    // one chunk of KK gathers, starting at step q0, into v[] (no wait)
    template <int KK>
    __device__ __forceinline__ static void issue_chunk(__amdgpu_buffer_rsrc_t fr, const int (&cid)[CH],
                                                       const Mask (&msk)[CH], int k, int sub, int gbase, bool skip,
                                                       int need, int q0, uint64_t (&v)[KK]) {
        if constexpr (NW == 64) {
            // one group is the whole wave, so step t's neighbour id and mask are
            // wave-uniform: read them into scalar registers (no LDS round trip)
            // and select each lane's word by the mask directly.  Steps past the
            // segment's end need no test: their id is -1, so their mask was
            // loaded from an out-of-range offset and is zero (no lane loads).
            (void)need;
            const uint64_t allowed = __ballot(!skip);
            const uint32_t koff = static_cast<uint32_t>(k) * 8u;
#pragma unroll
            for (int q = 0; q < KK; ++q) {
                const int t = q0 + q;
                const int w = __builtin_amdgcn_readlane(cid[0], t);
                const uint32_t mlo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(msk[0])), t));
                const uint32_t mhi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(msk[0] >> 32)), t));
                const uint64_t lanes = ((static_cast<uint64_t>(mhi) << 32) | mlo) & allowed;
                const uint32_t rowoff = static_cast<uint32_t>(w) * (NW * 8u);
                v[q] = buf_word(fr, select_lanes(lanes, rowoff + koff, kNoWord));
            }
            return;
        }
#pragma unroll
        for (int q = 0; q < KK; ++q) {
            const int h = (q0 + q) / NW;
            const int t = (q0 + q) % NW;
            const int j = t * NPAR + sub;
            const int w = __shfl(cid[h], gbase + j, 64);
            const Mask m = shfl_mask(msk[h], gbase + j);
            const bool ok = ((m >> k) & 1u) && !skip && (q0 + q) < need;
            const uint32_t off = ok ? static_cast<uint32_t>(w) * (NW * 8u) + static_cast<uint32_t>(k) * 8u : kNoWord;
            v[q] = buf_word(fr, off);
        }
    }

    template <int KK>
    __device__ __forceinline__ static uint64_t or_all(const uint64_t (&v)[KK]) {
        uint64_t x = 0;
#pragma unroll
        for (int q = 0; q < KK; ++q) x |= v[q];
        return x;
    }

    // skip: no gather at all in this round; later chunks also stop once
    // prior | OR so far is all ones.  At W = 4096 (one group per wave) a
    // round's last chunk is issued at a quarter or half of its size when the
    // segment needs no more further steps than that (a row of 1-2 arcs
    // issues K / 4 gather instructions, one of 3-4 arcs K / 2, not K).
    __device__ __forceinline__ static uint64_t round_or(__amdgpu_buffer_rsrc_t fr, const int (&cid)[CH],
                                                        const Mask (&msk)[CH], int k, int sub, int gbase,
                                                        bool skip, int cnt, uint64_t prior) {
        const int need = steps_needed(cnt);
        uint64_t x = 0;
#pragma unroll
        for (int q0 = 0; q0 < T; q0 += K) {
            if (!__any(q0 < need)) break;
            const bool sk = skip || (q0 > 0 && (prior | x) == ~0ull);
            if constexpr (NW == 64 && K >= 4) {
                if (!__any(q0 + K / 4 < need)) {
                    uint64_t v[K / 4];
                    issue_chunk<K / 4>(fr, cid, msk, k, sub, gbase, sk, need, q0, v);
                    x |= or_all<K / 4>(v);
                    break;
                }
                if (!__any(q0 + K / 2 < need)) {
                    uint64_t v[K / 2];
                    issue_chunk<K / 2>(fr, cid, msk, k, sub, gbase, sk, need, q0, v);
                    x |= or_all<K / 2>(v);
                    break;
                }
            }
            uint64_t v[K];
            issue_chunk<K>(fr, cid, msk, k, sub, gbase, sk, need, q0, v);
            x |= or_all<K>(v);
        }
        return x;
    }
};

// What a group reads for a segment before gathering: the record, the first
// round of column ids, the activity flags of those neighbours, the flag of
// the vertex's next-frontier slot and (single-segment rows, all-source mode)
// its accumulators.  The segment loop runs a three-stage pipeline -- records
// three segments ahead, ids and accumulators two ahead, neighbour flags one
// ahead -- so that a segment waits only for its own frontier gathers.
template <int NW>
struct SegPre {
    int4 sg;
    int cid[Gather<NW>::CH];
    MaskT<NW> fl[Gather<NW>::CH]; // frontier word masks of the neighbours in cid
    MaskT<NW> flag_old;          // word mask of the vertex's next-frontier slot
    bool sat;                    // the vertex holds every bit of the batch: no gathers
    int ipv;                     // level 1 of an all-source batch: the vertex's place in the batches
};

template <int NW, bool PER_SOURCE>
__device__ __forceinline__ void seg_prefetch(const LevelBufs& B, const int4 sg, bool valid, bool sat, int gl,
                                             SegPre<NW>& p) {
    using Mask = MaskT<NW>;
    p.sg = sg;
    p.sat = sat;
    // a saturated segment reads no ids (so no neighbour flags either); its
    // next-frontier word mask is still read, as the finaliser clears a stale one
    Gather<NW>::load_ids(B.col, sg.y, (valid && !sat) ? sg.z : sg.y, gl, p.cid);
    p.flag_old = buf_mask<Mask>(B.flag_nx, (valid && sg.w == 1) ? static_cast<uint32_t>(sg.x) * static_cast<uint32_t>(sizeof(Mask))
                                                              : kNoWord);
#pragma unroll
    for (int h = 0; h < Gather<NW>::CH; ++h) p.fl[h] = 0;
}

template <int NW>
__device__ __forceinline__ void seg_flags(const LevelBufs& B, SegPre<NW>& p) {
    Gather<NW>::load_masks(B.flag_fr, p.cid, p.fl);
}

template <int NW>
__device__ __forceinline__ LevelBufs level_bufs(const BfsArgs& a, const uint64_t* nx, const MaskT<NW>* flag_nx,
                                                const MaskT<NW>* flag_fr) {
    const uint32_t n = static_cast<uint32_t>(a.n);
    LevelBufs B;
    B.nx = words_rsrc(nx, n * (NW * 8u));
    B.vis = words_rsrc(a.vis, n * (NW * 8u));
    B.flag_nx = __builtin_amdgcn_make_buffer_rsrc(const_cast<MaskT<NW>*>(flag_nx), 0, static_cast<int>(n * sizeof(MaskT<NW>)), 0x00020000);
    B.flag_fr = __builtin_amdgcn_make_buffer_rsrc(const_cast<MaskT<NW>*>(flag_fr), 0, static_cast<int>(n * sizeof(MaskT<NW>)), 0x00020000);
    B.s32 = __builtin_amdgcn_make_buffer_rsrc(a.S32, 0, a.S32 ? static_cast<int>(n * 4u) : 0, 0x00020000);
    B.r = __builtin_amdgcn_make_buffer_rsrc(a.R, 0, static_cast<int>(n * 4u), 0x00020000);
    B.h2 = __builtin_amdgcn_make_buffer_rsrc(a.H2, 0, a.H2 ? static_cast<int>(n * 4u) : 0, 0x00020000);
    B.col = __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t*>(a.col_idx), 0, static_cast<int>(a.nnz_cap * 4), 0x00020000);
    B.seg = __builtin_amdgcn_make_buffer_rsrc(a.seg, 0, static_cast<int>(a.seg_cap * 16), 0x00020000);
    B.segsat = __builtin_amdgcn_make_buffer_rsrc(a.segsat, 0, static_cast<int>(a.seg_cap * 4), 0x00020000);
    return B;
}

// Distance classes of the ranking after the first batch.
constexpr int kDistClasses = 32;

__device__ __forceinline__ int dist_class(uint32_t member) {
    return member == 0u ? kDistClasses - 1 : min(static_cast<int>(member) - 1, kDistClasses - 2);
}

// Re-ranks the batch positions [W, n_act) -- the items after the first
// batch: vertices, or list positions of listed sources -- by the distance
// class of their vertex (member = 1 + distance from the first batch's probe,
// 0 outside its component), stable: each block counts the classes of its
// range of positions, then places them after every lower class and every
// earlier block's equal ones (ballots rank them inside a block), writing the
// new positions to iperm; perm is then rebuilt from iperm.  Called by every
// block of the graph's grid.
template <int BLOCK, class Barrier>
__device__ bool rank_by_distance(const BfsArgs& a, Barrier& gb, const unsigned blk, const unsigned nblk, const int W,
                                 const int n_act) {
    __shared__ int s_cnt[kDistClasses], s_tot[kDistClasses], s_before[kDistClasses], s_off[kDistClasses];
    __shared__ int s_wv[BLOCK / 64][kDistClasses];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const long long tail = static_cast<long long>(n_act) - W;
    const long long chunk = (tail + nblk - 1) / nblk;
    const long long q_lo = W + min(static_cast<long long>(blk) * chunk, tail);
    const long long q_hi = W + min(static_cast<long long>(blk) * chunk + chunk, tail);
    if (threadIdx.x < kDistClasses) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    // an item is a vertex (all sources) or a list position (listed sources)
    auto vertex_of = [&](int item) { return a.listed ? a.sources[item] : item; };
    for (long long q = q_lo + threadIdx.x; q < q_hi; q += BLOCK)
        atomicAdd(&s_cnt[dist_class(a.member[vertex_of(a.perm[q])])], 1);
    __syncthreads();
    if (threadIdx.x < kDistClasses) a.bcount[blk * kDistClasses + threadIdx.x] = s_cnt[threadIdx.x];
    if (!gb.wait()) return false;
    if (threadIdx.x < kDistClasses) s_tot[threadIdx.x] = s_before[threadIdx.x] = 0;
    __syncthreads();
    for (unsigned t = threadIdx.x; t < nblk * kDistClasses; t += BLOCK) {
        const unsigned b2 = t / kDistClasses, c = t % kDistClasses;
        const int x = a.bcount[t];
        if (x) {
            atomicAdd(&s_tot[c], x);
            if (b2 < blk) atomicAdd(&s_before[c], x);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = W;
#pragma unroll 1
        for (int c = 0; c < kDistClasses; ++c) {
            s_off[c] = acc + s_before[c];
            acc += s_tot[c];
        }
    }
    __syncthreads();
    for (long long base = q_lo; base < q_hi; base += BLOCK) {
        const long long q = base + threadIdx.x;
        const int v = q < q_hi ? a.perm[q] : -1;
        const int cls = v >= 0 ? dist_class(a.member[vertex_of(v)]) : -1;
        int before = 0;
#pragma unroll 1
        for (int c = 0; c < kDistClasses; ++c) {
            const unsigned long long bal = __ballot(cls == c);
            if (cls == c) before = __popcll(bal & ((1ull << lane) - 1ull));
            if (lane == 0) s_wv[wave][c] = __popcll(bal);
        }
        __syncthreads();
        if (cls >= 0) {
            int woff = 0;
#pragma unroll 1
            for (int w2 = 0; w2 < wave; ++w2) woff += s_wv[w2][cls];
            a.iperm[v] = s_off[cls] + woff + before;
        }
        __syncthreads();
        if (threadIdx.x < kDistClasses) {
            int tot = 0;
#pragma unroll 1
            for (int w2 = 0; w2 < BLOCK / 64; ++w2) tot += s_wv[w2][threadIdx.x];
            s_off[threadIdx.x] += tot;
        }
        __syncthreads();
    }
    if (!gb.wait()) return false;
    const long long tid = static_cast<long long>(blk) * BLOCK + threadIdx.x;
    const long long nthreads = static_cast<long long>(nblk) * BLOCK;
    const long long n_items = a.listed ? static_cast<long long>(a.n_src) : static_cast<long long>(a.n);
    for (long long v = tid; v < n_items; v += nthreads) {
        const int q = a.iperm[v];
        if (q >= W) a.perm[q] = static_cast<int32_t>(v);
    }
    return gb.wait();
}

// The whole computation for one graph, run by `nblk` blocks (this one is
// `blk`) that synchronise through `gb`: the grid of k_closeness, or one
// partition of the grid of k_closeness_multi.  Returns false when a barrier
// wait failed (every block then leaves).
template <int NW, int BLOCK, bool PER_SOURCE, class Barrier>
__device__ __forceinline__ bool closeness_run(const BfsArgs& a, Barrier& gb, const unsigned blk, const unsigned nblk) {
    constexpr int kLpv = lpv<NW>();
    constexpr int W = 64 * NW;
    using Mask = MaskT<NW>;
    const int n = a.n;
    const int lane = threadIdx.x & 63;
    const int gl = lane & (kLpv - 1);
    const int gbase = lane - gl;
    const int k = gl & (NW - 1);
    const int sub = gl / NW;
    const long long tid = static_cast<long long>(blk) * BLOCK + threadIdx.x;
    const long long nthreads = static_cast<long long>(nblk) * BLOCK;
    const long long gid = tid / kLpv;
    const long long ngroups = nthreads / kLpv;
    // block-interleaved thread and group numbers: consecutive indices fall in
    // different blocks, which spreads the block-local frontier lists
    const long long tid_x = static_cast<long long>(threadIdx.x) * nblk + blk;
    const long long gid_x = static_cast<long long>(threadIdx.x / kLpv) * nblk + blk;
    Ctrl* ctrl = a.ctrl;
    const int seg_len = a.seg_len;

    __shared__ int32_t s_cnt[PER_SOURCE ? W : 1];
    __shared__ int64_t s_S[PER_SOURCE ? W : 1];
    __shared__ int32_t s_R[PER_SOURCE ? W : 1];
    __shared__ int s_bins[kClasses];
    __shared__ int s_base[kClasses];
    __shared__ long long s_trace[2];
    __shared__ FrontierLds s_fr;

    // ---- phase 0: zero accumulators and scratch, check the input, count
    // segments per class.  The input is checked here so that no later access
    // can leave its buffer: row pointers monotone within the declared arc
    // count, column ids and listed sources in [0, n).  A violation is fault
    // code 2.
    if (threadIdx.x < kClasses) s_bins[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        s_fr.cnt[0] = s_fr.cnt[1] = 0;
        s_fr.arcs[0] = s_fr.arcs[1] = 0;
    }
    __syncthreads();
    int bad = 0;
    for (long long v = tid; v < n; v += nthreads) {
        if (!PER_SOURCE) {
            a.S[v] = 0;
            a.S32[v] = 0;
            // the vertex itself (d = 0); with listed sources each listed
            // occurrence adds its own 1 at batch init
            a.R[v] = a.listed ? 0 : 1;
            if (a.H2) a.H2[v] = 0;
        }
        a.hcnt[v] = 0;
        a.member[v] = 0u;
        const int e0 = a.row_ptr[v];
        const int e1 = a.row_ptr[v + 1];
        if (e0 < 0 || e1 < e0 || e1 > a.nnz_cap) {
            bad = 1;
            continue;
        }
        for (int e = e0; e < e1; ++e) bad |= static_cast<unsigned>(a.col_idx[e]) >= static_cast<unsigned>(n);
        const int deg = e1 - e0;
        if (deg > 0) atomicAdd(&s_bins[seg_class(deg, seg_len)], (deg + seg_len - 1) / seg_len);
    }
    if (a.listed)
        for (long long i = tid; i < a.n_src; i += nthreads)
            bad |= static_cast<unsigned>(a.sources[i]) >= static_cast<unsigned>(n);
    if (bad) store_agent_i32(a.fault, 2);
    for (long long i = tid; i < static_cast<long long>(n) * NW; i += nthreads) {
        a.hacc[i] = 0;
        a.bufB[i] = 0;
    }
    for (long long v = tid; v < n; v += nthreads) {
        static_cast<Mask*>(a.flagA)[v] = 0;
        static_cast<Mask*>(a.flagB)[v] = 0;
    }
    // All sources: the batches take only the vertices that have arcs (one
    // without any reaches just itself: R = 1 and S = 0 as set above), largest
    // degree class first and in id order inside a class (batches of hubs end
    // in fewer levels).  Block blk counts those of its range of ids per class
    // here and ranks them in phase 1.
    // Listed sources are ranked the same way by their vertex's class, over
    // list positions (positions ascending inside a class; a source without
    // arcs goes with the last class): batches of hub sources end early
    // there too, and the per-source outputs still go to the caller's
    // positions.
    __shared__ int s_act[BLOCK / 64][kRankClasses];
    __shared__ int s_cls[kRankClasses];
    const long long n_items = a.listed ? static_cast<long long>(a.n_src) : static_cast<long long>(n);
    const long long id_chunk = (n_items + nblk - 1) / nblk;
    const long long id_lo = min(static_cast<long long>(blk) * id_chunk, n_items);
    const long long id_hi = min(id_lo + id_chunk, n_items);
    auto rank_class = [&](long long item) {
        if (a.listed) {
            const int v = a.sources[item];
            if (static_cast<unsigned>(v) >= static_cast<unsigned>(n)) return -1;   // fault code 2, set above
            const int deg = a.row_ptr[v + 1] - a.row_ptr[v];
            return deg > 0 ? min(seg_class(deg, seg_len), kRankClasses - 1) : kRankClasses - 1;
        }
        const int deg = a.row_ptr[item + 1] - a.row_ptr[item];
        return deg > 0 ? min(seg_class(deg, seg_len), kRankClasses - 1) : -1;
    };
    if (threadIdx.x < kRankClasses) s_cls[threadIdx.x] = 0;
    __syncthreads();
    for (long long v = id_lo + threadIdx.x; v < id_hi; v += BLOCK) {
        const int c = rank_class(v);
        if (c >= 0) atomicAdd(&s_cls[c], 1);
    }
    __syncthreads();
    if (threadIdx.x < kRankClasses) a.bcount[blk * kRankClasses + threadIdx.x] = s_cls[threadIdx.x];
    if (threadIdx.x < kClasses && s_bins[threadIdx.x]) atomicAdd(&ctrl->bins[threadIdx.x], s_bins[threadIdx.x]);
    if (!gb.wait()) return false;
    if (load_agent_i32(a.fault) != 0) return false;              // uniform: read after the barrier

    // ---- phase 1: class offsets
    if (blk == 0 && threadIdx.x == 0) {
        int acc = 0;
        for (int c = 0; c < kClasses; ++c) {
            int b = load_agent_i32(&ctrl->bins[c]);
            store_agent_i32(&ctrl->cursor[c], acc);
            acc += b;
        }
        store_agent_i32(&ctrl->n_seg, acc);
    }
    {
        // this block's first position in each class: all items of the
        // classes before it, then those of the blocks before it
        __shared__ int s_tot[kRankClasses], s_before[kRankClasses], s_off[kRankClasses];
        if (threadIdx.x < kRankClasses) s_tot[threadIdx.x] = s_before[threadIdx.x] = 0;
        __syncthreads();
        for (unsigned t = threadIdx.x; t < nblk * kRankClasses; t += BLOCK) {
            const unsigned b2 = t / kRankClasses, c = t % kRankClasses;
            const int x = a.bcount[t];
            if (x) {
                atomicAdd(&s_tot[c], x);
                if (b2 < blk) atomicAdd(&s_before[c], x);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int c = 0; c < kRankClasses; ++c) {
                s_off[c] = acc + s_before[c];
                acc += s_tot[c];
            }
            if (blk == 0) store_agent_i32(&ctrl->n_act, acc);
        }
        __syncthreads();
        const int wave = threadIdx.x >> 6;
        for (long long base = id_lo; base < id_hi; base += BLOCK) {
            const long long v = base + threadIdx.x;
            const int cls = v < id_hi ? rank_class(v) : -1;
            int before = 0;
#pragma unroll
            for (int c = 0; c < kRankClasses; ++c) {
                const unsigned long long bal = __ballot(cls == c);
                if (cls == c) before = __popcll(bal & ((1ull << lane) - 1ull));
                if (lane == 0) s_act[wave][c] = __popcll(bal);
            }
            __syncthreads();
            if (v < id_hi) {
                int pos = -1;
                if (cls >= 0) {
                    int woff = 0;
                    for (int w2 = 0; w2 < wave; ++w2) woff += s_act[w2][cls];
                    pos = s_off[cls] + woff + before;
                    a.perm[pos] = static_cast<int32_t>(v);
                }
                a.iperm[v] = pos;
            }
            __syncthreads();
            if (threadIdx.x < kRankClasses) {
                int tot = 0;
                for (int w2 = 0; w2 < BLOCK / 64; ++w2) tot += s_act[w2][threadIdx.x];
                s_off[threadIdx.x] += tot;
            }
            __syncthreads();
        }
    }
    if (!gb.wait()) return false;

    // ---- phase 2: fill the segment list (heavy rows first, then by
    // decreasing degree; order inside a class is arbitrary and does not
    // affect any result)
    // Each block reserves one range per class for its vertices (LDS counts,
    // then one global add per class), so the class cursors see a few
    // thousand atomics rather than one per vertex.
    for (long long base = static_cast<long long>(blk) * BLOCK; base < n; base += nthreads) {
        const long long v = base + threadIdx.x;
        if (threadIdx.x < kClasses) s_bins[threadIdx.x] = 0;
        __syncthreads();
        int e0 = 0, deg = 0, segs = 0, cls = 0, local = 0;
        if (v < n) {
            e0 = a.row_ptr[v];
            deg = a.row_ptr[v + 1] - e0;
            if (deg > 0) {
                segs = (deg + seg_len - 1) / seg_len;
                cls = seg_class(deg, seg_len);
                local = atomicAdd(&s_bins[cls], segs);
            }
        }
        __syncthreads();
        if (threadIdx.x < kClasses && s_bins[threadIdx.x])
            s_base[threadIdx.x] = atomicAdd(&ctrl->cursor[threadIdx.x], s_bins[threadIdx.x]);
        __syncthreads();
        if (deg > 0) {
            const int pos = s_base[cls] + local;
            a.seg_first[v] = pos;
            for (int j = 0; j < segs && pos + j < a.seg_cap; ++j)
                a.seg[pos + j] = make_int4(static_cast<int>(v), e0 + j * seg_len, min(e0 + (j + 1) * seg_len, e0 + deg), segs);
        }
        __syncthreads();
    }
    if (!gb.wait()) return false;
    const long long n_seg = min(static_cast<long long>(load_agent_i32(&ctrl->n_seg)), a.seg_cap);

    // all sources: the batches run over the vertices with arcs (perm)
    const int n_src_eff = a.listed ? a.n_src : load_agent_i32(&ctrl->n_act);
    const int n_batches = (n_src_eff + W - 1) / W;
    // frontier lists and their arc counts feed only the push decision: not
    // kept when no level can run top-down
    const bool lists = a.direction == 1 || (a.direction == 0 && a.alpha != 0);
    const long long m_arcs = a.row_ptr[n];               // checked against nnz_cap in phase 0
    const unsigned long long gmask = (kLpv >= 64 ? ~0ull : ((1ull << kLpv) - 1ull)) << gbase;
    int trace_row = 0;
    int phase = 0;                                       // list slot of a phase: phase % 3
    // All sources at W = 4096 with level 1 always bottom-up: level 1 visits
    // every segment and knows each vertex's visited words without reading
    // them (the vertex's own source bit), so it stores them all and the batch
    // start does not clear the visited bitset.  Vertices without arcs are
    // never read.
    const bool l1_vis = NW == 64 && !a.listed && (a.alpha == 0 || a.direction == 2);
    // Per-vertex sums: a batch adds less than W * min(n, s32_levels) to a
    // vertex's 32-bit sum (at most W new bits, at depths below both), so
    // the 32-bit sums are folded into S only before a batch that could carry
    // them past 2^32 - 1, and at the end.
    const unsigned long long s32_cap = static_cast<unsigned long long>(W) * static_cast<unsigned long long>(min(n, a.s32_levels));
    unsigned long long s32_pend = 0;                     // bound on every S32 entry
    for (int b = 0; b < n_batches; ++b) {
        const int src0 = b * W;
        const int cnt = min(W, n_src_eff - src0);

        // ---- batch init: vis = fr = the batch's source bits (vis is left to
        // level 1 when l1_vis holds); the sources' segments form the first
        // frontier list; no segment is saturated
        bool push;
        {
            const int par = phase & 1;
            const bool fold = s32_pend + s32_cap > 0xFFFFFFFFull;
            s32_pend = fold ? s32_cap : s32_pend + s32_cap;
            for (long long i = tid; i < n_seg; i += nthreads) a.segsat[i] = 0u;
            // Saturation is judged against the component C of a probe: the
            // first batch's source of highest degree (ties: the first), whose
            // own BFS in that batch marks C exactly.  From the second batch
            // on, the batch's sources in C, one ballot per word (a wave's
            // lanes hold consecutive source positions); the first batch has
            // none, so nothing saturates in it.
            for (long long i = tid; i < W; i += nthreads) {
                bool in = false;
                if (i < cnt) {
                    const int src = a.listed ? a.sources[a.perm[src0 + i]] : a.perm[src0 + i];
                    // all sources: the source's own frontier bit (frontier
                    // words are read only where the word mask has the bit, so
                    // only the sources' own words are written)
                    if (!PER_SOURCE && !a.listed) a.bufA[static_cast<size_t>(src) * NW + (i >> 6)] = 1ull << (i & 63);
                    if (b == 0) {
                        const unsigned long long deg = static_cast<unsigned long long>(a.row_ptr[src + 1] - a.row_ptr[src]);
                        __hip_atomic_fetch_max(&ctrl->probe_key, (deg << 32) | (0xffffffffull - static_cast<unsigned long long>(i)),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        in = a.member[src] != 0u;
                    }
                }
                const unsigned long long word = __ballot(in);
                if ((threadIdx.x & 63) == 0)
                    __hip_atomic_store(&ctrl->gcm[i >> 6], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (blk == 0 && threadIdx.x == 0) {
                const int nx_slot = (phase + 1) % 3;
                store_agent_i32(&ctrl->fbad[nx_slot], 0);
                __hip_atomic_store(&ctrl->farcs[nx_slot], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (!PER_SOURCE && !a.listed) {
                for (long long i = l1_vis ? static_cast<long long>(n) * NW : tid; i < static_cast<long long>(n) * NW;
                     i += nthreads) {
                    const long long v = i / NW;
                    const int kk = static_cast<int>(i % NW);
                    const long long bit = static_cast<long long>(a.iperm[v]) - src0;
                    uint64_t w0 = 0;
                    if (bit >= 0 && bit < cnt && (bit >> 6) == kk) w0 = 1ull << (bit & 63);
                    a.vis[i] = w0;
                }
                for (long long v = tid; v < n; v += nthreads) {
                    const int j = a.iperm[v] - src0;
                    static_cast<Mask*>(a.flagA)[v] =
                        (j >= 0 && j < cnt) ? static_cast<Mask>(static_cast<Mask>(1) << (j >> 6)) : Mask(0);
                    // the earlier batches' 32-bit sums into S
                    if (fold) {
                        const uint32_t x = a.S32[v];
                        if (x) {
                            a.S[v] += x;
                            a.S32[v] = 0;
                        }
                    }
                }
                if (lists)
                    for (long long i = tid_x; i < cnt; i += nthreads) {
                        const int3 sg = vertex_segments(a, a.perm[src0 + i]);
                        if (sg.y > 0) frontier_note(s_fr, par, sg.x, sg.y, sg.z);
                    }
            } else {
                for (long long i = tid; i < static_cast<long long>(n) * NW; i += nthreads) a.vis[i] = 0;
                // only the words the sources' bits go to are cleared
                for (long long i = tid; i < cnt; i += nthreads)
                    a.bufA[static_cast<size_t>(a.sources[a.perm[src0 + i]]) * NW + (i >> 6)] = 0;
                for (long long v = tid; v < n; v += nthreads) {
                    static_cast<Mask*>(a.flagA)[v] = 0;
                    if (!PER_SOURCE && fold) {
                        // per-vertex sums: the earlier batches' 32-bit sums into S
                        const uint32_t x = a.S32[v];
                        if (x) {
                            a.S[v] += x;
                            a.S32[v] = 0;
                        }
                    }
                }
                if (PER_SOURCE)
                    for (int i = threadIdx.x; i < W; i += BLOCK) {
                        s_cnt[i] = 0;
                        s_S[i] = 0;
                        s_R[i] = 0;
                    }
                if (!gb.wait()) return false;
                for (long long i = tid_x; i < cnt; i += nthreads) {
                    const int s = a.sources[a.perm[src0 + i]];
                    const size_t w = static_cast<size_t>(s) * NW + (i >> 6);
                    atomicOr(reinterpret_cast<unsigned long long*>(&a.vis[w]), 1ull << (i & 63));
                    atomicOr(reinterpret_cast<unsigned long long*>(&a.bufA[w]), 1ull << (i & 63));
                    if (!PER_SOURCE) atomicAdd(&a.R[s], 1);      // per-vertex sums: the source reaches itself
                    atomicOr(&static_cast<Mask*>(a.flagA)[s], static_cast<Mask>(static_cast<Mask>(1) << (i >> 6)));
                }
                // The sources' segments form the first frontier lists, spread
                // over the blocks: segment j of a source goes to the list of
                // block (first + j) mod nblk, so a hub among the sources is
                // pushed by many blocks instead of by one.  A vertex listed
                // twice is noted twice (its words are ORed in twice: no change).
                for (int i = threadIdx.x; lists && i < cnt; i += BLOCK) {
                    const int3 sg = vertex_segments(a, a.sources[a.perm[src0 + i]]);
                    long long j = (static_cast<long long>(blk) - sg.x) % static_cast<long long>(nblk);
                    if (j < 0) j += nblk;
                    for (; j < sg.y; j += nblk)
                        frontier_note(s_fr, par, sg.x + static_cast<int>(j), 1,
                                      min(seg_len, sg.z - static_cast<int>(j) * seg_len));
                }
            }
            const hln::dev::BarrierResult br =
                gb.sync(0, PhaseEnd{&s_fr, ctrl, phase, lists}, Decide{ctrl, m_arcs, a.direction, a.alpha, phase});
            if (!br.ok) return false;
            push = br.decision;
            ++phase;
        }
        const uint64_t gcm_k = hln::dev::load_agent(&ctrl->gcm[k]);
        // the first batch records in member, for every vertex its probe
        // source (highest degree, first position on ties) reaches, 1 + the
        // distance: at the start of level d, from the frontier of level d - 1
        const int probe_pos = (b == 0 && n_batches > 1)
            ? static_cast<int>(0xffffffffu - static_cast<unsigned>(hln::dev::load_agent(&ctrl->probe_key) & 0xffffffffull))
            : -1;

        // ---- level loop; the barrier's OR tells every block whether any
        // vertex got a new bit, which ends this batch's BFS
        uint64_t* fr = a.bufA;
        uint64_t* nx = a.bufB;
        Mask* flag_fr = static_cast<Mask*>(a.flagA);
        Mask* flag_nx = static_cast<Mask*>(a.flagB);
        for (int d = 1;; ++d) {
            const int par = phase & 1;                   // this phase's list; the previous one is par ^ 1
            const bool vis1 = l1_vis && d == 1;
            if (blk == 0 && threadIdx.x == 0) {
                const int nx_slot = (phase + 1) % 3;
                store_agent_i32(&ctrl->fbad[nx_slot], 0);
                __hip_atomic_store(&ctrl->farcs[nx_slot], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            int any = 0;
            long long t_pairs = 0;
            int t_verts = 0;
            if (probe_pos >= 0) {
                const int kp = probe_pos >> 6;
                for (long long v = tid; v < n; v += nthreads)
                    if (((flag_fr[v] >> kp) & 1u) != 0 && ((fr[static_cast<size_t>(v) * NW + kp] >> (probe_pos & 63)) & 1ull) != 0)
                        a.member[v] = static_cast<uint32_t>(d);
            }
            const LevelBufs B = level_bufs<NW>(a, nx, flag_nx, flag_fr);
            if (push) {
                // ---- top-down, part 1: each block ORs the frontier words of
                // the segments on its own list into their neighbours'
                // accumulators (no block's list overflowed, or the level
                // would be bottom-up)
                const int flen = min(s_fr.cnt[par ^ 1], kFlCap);
                for (int i = static_cast<int>(threadIdx.x) / kLpv; i < flen; i += BLOCK / kLpv) {
                    const int4 sg = a.seg[s_fr.fl[par ^ 1][i]];
                    const int u = sg.x;
                    const Mask fm = flag_fr[u];
                    const uint64_t x = ((fm >> k) & 1u) ? fr[static_cast<size_t>(u) * NW + k] : 0ull;
                    for (int c = sg.y; c < sg.z; c += kLpv) {
                        const int wl = (c + gl < sg.z) ? a.col_idx[c + gl] : -1;
#pragma unroll
                        for (int t = 0; t < NW; ++t) {
                            const int w = group_bcast<kLpv>(wl, gbase, t * Gather<NW>::NPAR + sub);
                            if (w >= 0 && x)
                                __hip_atomic_fetch_or(reinterpret_cast<unsigned long long*>(&a.hacc[static_cast<size_t>(w) * NW + k]),
                                                      static_cast<unsigned long long>(x), __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                        }
                        if (wl >= 0) store_agent_i32(&a.hcnt[wl], 1);
                    }
                }
                if (!gb.wait()) return false;
                // ---- part 2: finalise touched vertices; vertices whose nx
                // word mask still holds the older frontier get it cleared
                for (long long v0 = gid_x * kLpv; v0 < n; v0 += ngroups * kLpv) {
                    const long long vl = v0 + gl;
                    int touched = 0;
                    Mask fo = 0;
                    if (vl < n) {
                        touched = load_agent_i32(&a.hcnt[vl]);
                        fo = flag_nx[vl];
                    }
                    unsigned long long ball = (__ballot(touched != 0 || fo != 0u) & gmask) >> gbase;
                    while (ball) {
                        const int j = __ffsll(static_cast<long long>(ball)) - 1;
                        ball &= ball - 1;
                        const int v = static_cast<int>(v0 + j);
                        const int tj = group_bcast<kLpv>(touched, gbase, j);
                        Mask foj;
                        if constexpr (kLpv == 64) {
                            const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(fo)), j));
                            const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(static_cast<uint64_t>(fo) >> 32)), j));
                            foj = static_cast<Mask>((static_cast<uint64_t>(hi) << 32) | lo);
                        } else {
                            foj = shfl_mask(fo, gbase + j);
                        }
                        const size_t base = static_cast<size_t>(v) * NW + k;
                        uint64_t acc = 0, vis_v = 0;
                        if (tj) {
                            if (sub == 0) {
                                acc = __hip_atomic_exchange(reinterpret_cast<unsigned long long*>(&a.hacc[base]), 0ull,
                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                vis_v = a.vis[base];
                            }
                            if (gl == 0) store_agent_i32(&a.hcnt[v], 0);
                        }
                        const int3 cw = finalize_vertex<NW, PER_SOURCE>(a, B, v, d, k, sub, gl, gbase, acc, vis_v,
                                                                        s_cnt, foj, gcm_k);
                        if (cw.x) {
                            any = 1;
                            t_pairs += cw.x;
                            t_verts += 1;
                            const int3 sgv = vertex_segments(a, v);
                            if (lists && gl == 0 && sgv.y > 0) frontier_note(s_fr, par, sgv.x, sgv.y, sgv.z * cw.y);
                            if (cw.z) mark_saturated<kLpv>(a, sgv.x, sgv.y, gl, d);
                        }
                    }
                }
            } else {
                // ---- bottom-up over all segments
                const __amdgpu_buffer_rsrc_t fr_rsrc = words_rsrc(fr, static_cast<uint32_t>(n) * (NW * 8u));
                auto rec_at = [&](long long i) {
                    return buf_i4(B.seg, i < n_seg ? static_cast<uint32_t>(i) * 16u : kNoWord);
                };
                auto sat_at = [&](long long i) {
                    return buf_u32(B.segsat, i < n_seg ? static_cast<uint32_t>(i) * 4u : kNoWord) != 0u;
                };
                // the end of a segment: merge a multi-segment row's partial OR
                // (the last finisher finalises) or finalise a single-segment row
                auto finish = [&](long long s, int4 sg, uint64_t acc, uint64_t vis_v, Mask flag_old) {
                    const int v = sg.x;
                    const int nseg = sg.w;
                    const size_t base = static_cast<size_t>(v) * NW + k;
#pragma unroll
                    for (int off = NW; off < kLpv; off <<= 1) acc |= shfl_xor_u64(acc, off);
                    if (nseg == 1) {
                        const int3 cw = finalize_vertex<NW, PER_SOURCE>(a, B, v, d, k, sub, gl, gbase, acc, vis_v,
                                                                        s_cnt, flag_old, gcm_k, vis1);
                        if (cw.x) {
                            any = 1;
                            t_pairs += cw.x;
                            t_verts += 1;
                            if (lists && gl == 0) frontier_note(s_fr, par, static_cast<int>(s), 1, (sg.z - sg.y) * cw.y);
                            if (cw.z) mark_saturated<kLpv>(a, static_cast<int>(s), 1, gl, d);
                        }
                    } else {
                        // multi-segment row: merge, the last finisher finalises
                        if (sub == 0 && acc)
                            __hip_atomic_fetch_or(reinterpret_cast<unsigned long long*>(&a.hacc[base]),
                                                  static_cast<unsigned long long>(acc), __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
                        // the wave's OR atomics are performed before the count is
                        // raised (agent-scope atomics complete at the coherence
                        // point; vmcnt(0) waits for their acknowledgement)
                        __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        __builtin_amdgcn_s_waitcnt(0);
                        __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        int old = 0;
                        if (gl == 0)
                            old = __hip_atomic_fetch_add(&a.hcnt[v], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        old = group_bcast<kLpv>(old, gbase, 0);
                        if (old == nseg - 1) {
                            uint64_t full = 0;
                            if (sub == 0)
                                full = __hip_atomic_exchange(reinterpret_cast<unsigned long long*>(&a.hacc[base]), 0ull,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                            for (int off = NW; off < kLpv; off <<= 1) full |= shfl_xor_u64(full, off);
                            const Mask flag_old = flag_nx[v];
                            if (gl == 0) store_agent_i32(&a.hcnt[v], 0);
                            const int3 cw = finalize_vertex<NW, PER_SOURCE>(a, B, v, d, k, sub, gl, gbase, full, vis_v,
                                                                            s_cnt, flag_old, gcm_k, vis1);
                            if (cw.x) {
                                any = 1;
                                t_pairs += cw.x;
                                t_verts += 1;
                                const int first = a.seg_first[v];
                                if (lists && gl == 0) frontier_note(s_fr, par, first, nseg, nseg * seg_len * cw.y);
                                if (cw.z) mark_saturated<kLpv>(a, first, nseg, gl, d);
                            }
                        }
                    }
                };
                bool level1_ids = false;
                if constexpr (NW == 64) level1_ids = d == 1 && !a.listed;
                // one segment: the visited word and the frontier gathers, then
                // its ending (cur holds what the pipeline prefetched for it)
                auto visit = [&](long long s, const SegPre<NW>& cur) {
                    const int v = cur.sg.x;
                    const int nseg = cur.sg.w;
                    const size_t base = static_cast<size_t>(v) * NW + k;
                    bool active = false;
#pragma unroll
                    for (int h = 0; h < Gather<NW>::CH; ++h) active |= cur.fl[h] != 0u;
                    // the visited word is read only when a neighbour is active, the
                    // segment has further rounds or the row has several segments (its
                    // finaliser needs it), together with the gathers
                    const bool need = !cur.sat && (((__ballot(active) & gmask) != 0) ||
                                                   (cur.sg.z - cur.sg.y > Gather<NW>::ROUND) || nseg > 1);
                    uint64_t vis_v = 0;
                    uint64_t acc = 0;
                    if (need) {
                        // the first chunk does not wait for the visited word (no
                        // saturation test); later chunks and rounds use it
                        vis_v = a.vis[base];
                        if constexpr (NW < 64) {
                            // Segments longer than a round (ROUND arcs): each
                            // round's column ids go out with the previous
                            // round's gathers, so a further round waits for its
                            // masks and its gathers only.
                            constexpr int RD = Gather<NW>::ROUND;
                            const int c1 = cur.sg.y + RD;
                            int cidn[Gather<NW>::CH];
                            const bool more = __any(c1 < cur.sg.z);
                            if (more) Gather<NW>::load_ids(B.col, c1, cur.sg.z, gl, cidn);
                            acc = Gather<NW>::round_or(fr_rsrc, cur.cid, cur.fl, k, sub, gbase, false, cur.sg.z - cur.sg.y,
                                                       vis_v);
                            if (more) {
                                for (int c = c1; c < cur.sg.z; c += RD) {
                                    Mask msk[Gather<NW>::CH];
                                    Gather<NW>::load_masks(B.flag_fr, cidn, msk);
                                    int cidnn[Gather<NW>::CH];
                                    Gather<NW>::load_ids(B.col, c + RD, cur.sg.z, gl, cidnn);
                                    acc |= Gather<NW>::round_or(fr_rsrc, cidn, msk, k, sub, gbase, (vis_v | acc) == ~0ull,
                                                                cur.sg.z - c, vis_v | acc);
#pragma unroll
                                    for (int h = 0; h < Gather<NW>::CH; ++h) cidn[h] = cidnn[h];
                                }
                            }
                        } else {
                            acc = Gather<NW>::round_or(fr_rsrc, cur.cid, cur.fl, k, sub, gbase, false, cur.sg.z - cur.sg.y,
                                                       vis_v);
                            for (int c = cur.sg.y + Gather<NW>::ROUND; c < cur.sg.z; c += Gather<NW>::ROUND) {
                                int cid[Gather<NW>::CH];
                                Mask msk[Gather<NW>::CH];
                                Gather<NW>::load_ids(B.col, c, cur.sg.z, gl, cid);
                                Gather<NW>::load_masks(B.flag_fr, cid, msk);
                                acc |= Gather<NW>::round_or(fr_rsrc, cid, msk, k, sub, gbase, (vis_v | acc) == ~0ull,
                                                            cur.sg.z - c, vis_v | acc);
                            }
                        }
                    }
                    finish(s, cur.sg, acc, vis_v, cur.flag_old);
                };
                if constexpr (NW == 64) {
                    // One group per wave: the wave takes its segments s = gid +
                    // j * ngroups in windows of 64, lane j loading record and
                    // saturation level of the window's segment j in one
                    // instruction each, so no record is waited for inside the
                    // sweep.  A segment saturated at level L still clears its
                    // vertex's stale next-frontier word masks at levels L + 1
                    // and L + 2 (no gathers): a single-segment row's lane does
                    // that itself, a longer row goes through the segment ending
                    // (its segments are counted); from L + 3 on it is left out.
                    const int gid_u = __builtin_amdgcn_readfirstlane(static_cast<int>(gid));
                    const int ng = static_cast<int>(ngroups);
                    const int nsg = static_cast<int>(n_seg);
                    const uint32_t dlev = static_cast<uint32_t>(d);
                    // Level 1 of an all-source batch: the frontier is the batch's
                    // sources perm[src0 .. src0 + cnt - 1] with one bit each, so a
                    // neighbour's frontier word follows from its place in perm and
                    // the visited word from the vertex's own (the batch start left
                    // only the sources' own bits): the level reads column ids and
                    // iperm only, in the same window pipeline (ids two segments
                    // ahead, the neighbours' places one ahead).
                    for (int wb = level1_ids ? gid_u : nsg; wb < nsg; wb += 64 * ng) {
                        const int my = wb + lane * ng;
                        const bool ok = my < nsg;
                        const int4 myrec = buf_i4(B.seg, ok ? static_cast<uint32_t>(my) * 16u : kNoWord);
                        uint64_t todo = __ballot(ok);
                        auto take1 = [&](SegPre<NW>& p, int& sp) {
                            int4 rec = make_int4(0, 0, 0, 0);
                            sp = nsg;
                            if (todo != 0) {
                                const int j = __builtin_ctzll(todo);
                                todo &= todo - 1;
                                rec = make_int4(__builtin_amdgcn_readlane(myrec.x, j), __builtin_amdgcn_readlane(myrec.y, j),
                                                __builtin_amdgcn_readlane(myrec.z, j), __builtin_amdgcn_readlane(myrec.w, j));
                                sp = wb + j * ng;
                            }
                            const bool valid = sp < nsg;
                            p.sg = rec;
                            p.sat = false;
                            const int e = rec.y + gl;
                            const uint32_t x = buf_u32(B.col, (valid && e < rec.z) ? static_cast<uint32_t>(e) * 4u : kNoWord);
                            p.cid[0] = (valid && e < rec.z) ? static_cast<int>(x) : -1;
                            p.flag_old = buf_mask<Mask>(B.flag_nx, (valid && rec.w == 1) ? static_cast<uint32_t>(rec.x) * static_cast<uint32_t>(sizeof(Mask))
                                                                                       : kNoWord);
                            p.ipv = valid ? a.iperm[rec.x] : -1;
                            p.fl[0] = 0;
                        };
                        // the neighbours' places among the batches' sources (-1: no arc or no place)
                        auto places = [&](SegPre<NW>& p) {
                            p.fl[0] = static_cast<Mask>(static_cast<uint32_t>(p.cid[0] >= 0 ? a.iperm[p.cid[0]] : -1));
                        };
                        SegPre<NW> cur, nxt;
                        int sc, sn;
                        take1(cur, sc);
                        take1(nxt, sn);
                        places(cur);
                        while (sc < nsg) {
                            SegPre<NW> nn;
                            int snn;
                            take1(nn, snn);                                // ids, 2 ahead
                            places(nxt);                                   // places, 1 ahead
                            const int rel_l = static_cast<int>(static_cast<uint32_t>(cur.fl[0])) - src0;
                            unsigned long long hits = __ballot(cur.cid[0] >= 0 && rel_l >= 0 && rel_l < cnt);
                            uint64_t acc = 0;
                            while (hits) {
                                const int t = __ffsll(static_cast<long long>(hits)) - 1;
                                hits &= hits - 1;
                                const int rel = __builtin_amdgcn_readlane(rel_l, t);
                                if ((rel >> 6) == k) acc |= 1ull << (rel & 63);
                            }
                            const int own = cur.ipv - src0;
                            const uint64_t vis_v = (own >= 0 && own < cnt && (own >> 6) == k) ? (1ull << (own & 63)) : 0ull;
                            finish(sc, cur.sg, acc, vis_v, cur.flag_old);
                            sc = sn;
                            cur = nxt;
                            sn = snn;
                            nxt = nn;
                        }
                    }
                    for (int wb = level1_ids ? nsg : gid_u; wb < nsg; wb += 64 * ng) {
                        const int my = wb + lane * ng;
                        const bool ok = my < nsg;
                        const uint32_t slev = buf_u32(B.segsat, ok ? static_cast<uint32_t>(my) * 4u : kNoWord);
                        const int4 myrec = buf_i4(B.seg, ok ? static_cast<uint32_t>(my) * 16u : kNoWord);
                        const bool clear_only = ok && slev != 0u && dlev <= slev + 2u;
                        const bool own_clear = clear_only && myrec.w == 1;
                        const uint32_t own_off = own_clear ? static_cast<uint32_t>(myrec.x) * static_cast<uint32_t>(sizeof(Mask))
                                                           : kNoWord;
                        const Mask own_old = buf_mask<Mask>(B.flag_nx, own_off);
                        uint64_t todo = __ballot(ok && (slev == 0u || (clear_only && !own_clear)));
                        const uint64_t satm = __ballot(slev != 0u);
                        // the next segment of the window into p (sp = nsg: none left)
                        auto take = [&](SegPre<NW>& p, int& sp) {
                            int4 rec = make_int4(0, 0, 0, 0);
                            bool sat = false;
                            sp = nsg;
                            if (todo != 0) {
                                const int j = __builtin_ctzll(todo);
                                todo &= todo - 1;
                                rec = make_int4(__builtin_amdgcn_readlane(myrec.x, j), __builtin_amdgcn_readlane(myrec.y, j),
                                                __builtin_amdgcn_readlane(myrec.z, j), __builtin_amdgcn_readlane(myrec.w, j));
                                sat = ((satm >> j) & 1ull) != 0;
                                sp = wb + j * ng;
                            }
                            seg_prefetch<NW, PER_SOURCE>(B, rec, sp < nsg, sat, gl, p);
                        };
                        SegPre<NW> cur, nxt;
                        int sc, sn;
                        take(cur, sc);
                        take(nxt, sn);
                        seg_flags<NW>(B, cur);
                        buf_store_mask<Mask>(Mask(0), B.flag_nx, own_old != 0u ? own_off : kNoWord);
                        while (sc < nsg) {
                            SegPre<NW> nn;
                            int snn;
                            take(nn, snn);                                 // ids, 2 ahead
                            seg_flags<NW>(B, nxt);                         // flags, 1 ahead
                            visit(sc, cur);
                            sc = sn;
                            cur = nxt;
                            sn = snn;
                            nxt = nn;
                        }
                    }
                } else {
                    long long s = level1_ids ? n_seg : gid;
                    SegPre<NW> cur, nxt;
                    seg_prefetch<NW, PER_SOURCE>(B, rec_at(s), s < n_seg, sat_at(s), gl, cur);
                    seg_prefetch<NW, PER_SOURCE>(B, rec_at(s + ngroups), s + ngroups < n_seg, sat_at(s + ngroups), gl, nxt);
                    seg_flags<NW>(B, cur);
                    int4 rec2 = rec_at(s + 2 * ngroups);
                    bool sat2 = sat_at(s + 2 * ngroups);
                    while (s < n_seg) {
                        const long long s1 = s + ngroups;
                        const long long s2 = s1 + ngroups;
                        const long long s3 = s2 + ngroups;
                        const int4 rec3 = rec_at(s3);                                      // record, 3 ahead
                        const bool sat3 = sat_at(s3);
                        SegPre<NW> nn;
                        seg_prefetch<NW, PER_SOURCE>(B, rec2, s2 < n_seg, sat2, gl, nn);    // ids, 2 ahead
                        seg_flags<NW>(B, nxt);                                             // flags, 1 ahead

                        visit(s, cur);
                        s = s1;
                        cur = nxt;
                        nxt = nn;
                        rec2 = rec3;
                        sat2 = sat3;
                    }
                }
            }
            if (PER_SOURCE) {
                __syncthreads();
                for (int i = threadIdx.x; i < W; i += BLOCK) {
                    const int c = s_cnt[i];
                    if (c) {
                        s_S[i] += static_cast<int64_t>(d) * c;
                        s_R[i] += c;
                        s_cnt[i] = 0;
                    }
                }
            }
            if (a.trace && trace_row < a.trace_cap) {
                // block totals in LDS, then one global add per block
                __syncthreads();
                if (threadIdx.x == 0) {
                    s_trace[0] = 0;
                    s_trace[1] = 0;
                }
                __syncthreads();
                if (gl == 0 && t_verts) {
                    atomicAdd(reinterpret_cast<unsigned long long*>(&s_trace[0]), static_cast<unsigned long long>(t_verts));
                    atomicAdd(reinterpret_cast<unsigned long long*>(&s_trace[1]), static_cast<unsigned long long>(t_pairs));
                }
                __syncthreads();
                if (threadIdx.x == 0 && s_trace[0]) (void)trace_add(a.trace + 4 * trace_row, s_trace[0], s_trace[1]);
            }
            const hln::dev::BarrierResult br =
                gb.sync(any, PhaseEnd{&s_fr, ctrl, phase, lists}, Decide{ctrl, m_arcs, a.direction, a.alpha, phase});
            if (!br.ok) return false;
            if (a.trace && trace_row < a.trace_cap && blk == 0 && threadIdx.x == 0) {
                a.trace[4 * trace_row] = static_cast<int64_t>(__builtin_amdgcn_s_memrealtime());
                a.trace[4 * trace_row + 3] = push ? 1 : 0;
            }
            push = br.decision;
            ++phase;
            ++trace_row;
            if (!br.any) {
                // level d found nothing new: the batch's largest eccentricity is d - 1
                if (a.levels && blk == 0 && threadIdx.x == 0) a.levels[b] = d;
                break;
            }
            uint64_t* t = fr;
            fr = nx;
            nx = t;
            Mask* tf = flag_fr;
            flag_fr = flag_nx;
            flag_nx = tf;
        }

        if (PER_SOURCE) {
            int64_t* pS = a.part + static_cast<size_t>(blk) * 2 * W;
            int64_t* pR = pS + W;
            for (int i = threadIdx.x; i < W; i += BLOCK) {
                pS[i] = s_S[i];
                pR[i] = s_R[i];
            }
            if (!gb.wait()) return false;
            // one wave per source: its lanes take every 64th block's partial
            // (all in flight at once), then a wave sum (exact: integers)
            for (long long i = tid >> 6; i < cnt; i += nthreads >> 6) {
                uint64_t sS = 0, sR = 0;
                for (unsigned bb = static_cast<unsigned>(lane); bb < nblk; bb += 64) {
                    const int64_t* q = a.part + static_cast<size_t>(bb) * 2 * W;
                    sS += static_cast<uint64_t>(q[i]);
                    sR += static_cast<uint64_t>(q[W + i]);
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    sS += shfl_xor_u64(sS, off);
                    sR += shfl_xor_u64(sR, off);
                }
                if (lane == 0) {
                    const int q = a.perm[src0 + i];          // the source's position in the caller's list
                    a.S[q] = static_cast<int64_t>(sS);
                    a.R[q] = static_cast<int32_t>(1 + static_cast<int64_t>(sR));
                }
            }
            // the partials are rewritten only after the next batch's barriers
        }
        if (b == 0 && n_batches > 1) {
            // member now holds the probe's component (nonzero: 1 + the
            // vertex's distance from the probe), complete since the batch's
            // last level barrier.  All sources: the later batches take the remaining vertices by
            // their distance from the probe (nearest first, distances past
            // kDistClasses - 2 together, vertices outside its component last),
            // keeping the degree-class order among equals.  A batch's level
            // count is 1 + its sources' largest eccentricity, and vertices at
            // one distance from a hub have close eccentricities.
            if constexpr (!PER_SOURCE || NW < 64)
                if (!rank_by_distance<BLOCK>(a, gb, blk, nblk, W, n_src_eff)) return false;
        }
    }

    // ---- closeness (Eq. 1, Wasserman-Faust form, fixed operation order);
    // per-vertex sums (all-source or listed) first fold the last batch's
    // 32-bit sums into S (the same thread reads and writes each vertex, after
    // the final level barrier)
    if (PER_SOURCE) {
        // listed sources: the last writes of S and R are the reduction above
        if (a.cc && !gb.wait()) return false;
    }
    if (!PER_SOURCE || a.cc) {
        const long long n_out = PER_SOURCE ? a.n_src : n;
        for (long long i = tid; i < n_out; i += nthreads) {
            int64_t sv = a.S[i];
            if (!PER_SOURCE) {
                sv += a.S32[i];
                a.S[i] = sv;
                a.S32[i] = 0;
            }
            if (a.cc) {
                const int32_t r = a.R[i];
                double c = 0.0;
                if (r > 1 && sv > 0 && n > 1) {
                    const double reach = static_cast<double>(r - 1);
                    const double q1 = reach / static_cast<double>(sv);
                    const double q2 = reach / static_cast<double>(n - 1);
                    c = q1 * q2;
                }
                a.cc[i] = c;
            }
        }
    }
    return true;
}

// The work index of block `blk` of `nblk` whose consecutive blocks cycle
// through `xcds` XCDs (workgroups are dealt to the XCDs in turn): blocks on
// one XCD take consecutive work indices, so at any moment an XCD's waves
// hold neighbouring segments (vertices close in id, whose gathers share
// lines where the graph's ids carry locality).  The identity when the blocks
// do not divide evenly.
__device__ __forceinline__ unsigned xcd_work_index(unsigned blk, unsigned nblk, unsigned xcds) {
    if (xcds <= 1 || nblk % xcds != 0) return blk;
    return (blk % xcds) * (nblk / xcds) + blk / xcds;
}
constexpr unsigned kXcds = 8;

template <int NW, int BLOCK, bool PER_SOURCE>
__global__ __launch_bounds__(BLOCK) void k_closeness(BfsArgs a) {
    hln::dev::GridBarrier gb{a.bar, a.fault, a.wait_ticks, 0u, 0u, 0u};
    (void)closeness_run<NW, BLOCK, PER_SOURCE>(a, gb, xcd_work_index(blockIdx.x, gridDim.x, kXcds), gridDim.x);
}

__global__ void k_zero_ctrl(Ctrl* c, unsigned long long* bar) {
    int* p = reinterpret_cast<int*>(c);
    for (int i = threadIdx.x; i < static_cast<int>(sizeof(Ctrl) / sizeof(int)); i += blockDim.x) p[i] = 0;
    for (int i = threadIdx.x; i < hln::dev::kBarrierWords; i += blockDim.x) bar[i] = 0;
}

// Several graphs in one cooperative launch (all in the same accumulation
// mode: all sources with per-vertex sums, or listed sources with per-source
// sums):
// the grid is cut into `parts` partitions, partition p holding the blocks b
// with b % parts == p (blocks are dealt to the XCDs in turn, so with 8
// partitions each keeps to one XCD and its L2).  A partition runs its list
// of graphs one after another with the single-graph algorithm and a barrier
// of its own, clearing its control block between two graphs.  All graphs of
// a partition share one workspace slice.
template <int NW, int BLOCK, bool PER_SOURCE>
__global__ __launch_bounds__(BLOCK) void k_closeness_multi(const BfsArgs* __restrict__ args,
                                                           const int* __restrict__ plist,
                                                           const int* __restrict__ pfirst, int parts) {
    const unsigned np = static_cast<unsigned>(parts);
    const unsigned p = blockIdx.x % np;
    const unsigned nblk = gridDim.x / np;
    const unsigned blk = blockIdx.x / np;
    if (blk >= nblk) return;                              // blocks past the last full round take no part
    const int i0 = pfirst[p];
    const int i1 = pfirst[p + 1];
    if (i0 >= i1) return;
    const BfsArgs& first = args[plist[i0]];
    hln::dev::PartBarrier gb{first.bar, first.fault, first.wait_ticks, 0u, nblk, blk};
    // a partition's blocks p, p + np, ... cycle through 8 / gcd(np, 8) XCDs
    unsigned g8 = np;
    for (unsigned r = kXcds; r != 0;) { const unsigned t = g8 % r; g8 = r; r = t; }
    const unsigned work_blk = xcd_work_index(blk, nblk, kXcds / g8);
    for (int i = i0; i < i1; ++i) {
        const BfsArgs a = args[plist[i]];
        if (i > i0) {
            if (!gb.wait()) return;
            if (blk == 0) {
                int* c = reinterpret_cast<int*>(a.ctrl);
                for (int j = threadIdx.x; j < static_cast<int>(sizeof(Ctrl) / sizeof(int)); j += BLOCK) c[j] = 0;
            }
            if (!gb.wait()) return;
        }
        if (!closeness_run<NW, BLOCK, PER_SOURCE>(a, gb, work_blk, nblk)) return;
    }
}

// Control blocks and barrier words of the partitions' slices, before a
// multi-graph launch (block p clears partition p's).
__global__ void k_zero_parts(const BfsArgs* __restrict__ args, const int* __restrict__ plist,
                             const int* __restrict__ pfirst) {
    const int p = blockIdx.x;
    if (pfirst[p] >= pfirst[p + 1]) return;
    const BfsArgs& a = args[plist[pfirst[p]]];
    int* c = reinterpret_cast<int*>(a.ctrl);
    for (int i = threadIdx.x; i < static_cast<int>(sizeof(Ctrl) / sizeof(int)); i += blockDim.x) c[i] = 0;
    for (int i = threadIdx.x; i < hln::dev::kBarrierWords; i += blockDim.x) a.bar[i] = 0;
}

struct Layout {
    size_t words;     // n * NW
    size_t seg_cap;
};

// A kernel with grid barriers needs every block of its grid resident at
// once.  The cooperative launch is the runtime's guarantee of that; inside a
// stream capture the runtime may refuse it, and the same grid then goes out
// as an ordinary kernel node.  Either way the grid never exceeds the
// residency bound (hln::residency: the occupancy query, and the blocks the
// kernel's own VGPRs and LDS allow per compute unit, times the compute
// units), and every wait in the kernel is bounded, so a grid that did not
// all start ends with fault code 1 rather than hanging.
hln_status launch_persistent(const void* f, int grid, int block, void** kargs, int bound_grid, hipStream_t stream) {
    if (grid < 1 || grid > bound_grid)
        return hln::fail(HLN_EUNSUPPORTED, "grid of %d blocks exceeds the co-residency bound %d", grid, bound_grid);
    hipError_t e = hipLaunchCooperativeKernel(f, dim3(grid), dim3(block), kargs, 0, stream);
    int path = 1;
    if (e != hipSuccess) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &cap) == hipSuccess && cap == hipStreamCaptureStatusActive) {
            (void)hipGetLastError();
            e = hipLaunchKernel(f, dim3(grid), dim3(block), kargs, 0, stream);
            path = 2;
        }
    }
    if (e != hipSuccess) return hln::fail(HLN_EDEVICE, "persistent launch failed: %s", hipGetErrorString(e));
    hln::note_launch_path(path);
    return HLN_OK;
}

template <int NW, int BLOCK, bool PS>
const void* closeness_fn() {
    return reinterpret_cast<const void*>(&k_closeness<NW, BLOCK, PS>);
}

// Blocks per compute unit of a persistent launch: the residency bound,
// at most one 1024-thread block's worth of threads per CU by default (the
// measured best: fewest barrier participants for the same waves).
// HLN_BLOCKS_PER_CU overrides the default up to the bound; a value above
// the bound is refused (0 is returned and the error set).
int blocks_per_cu(const void* f, int block) {
    hln::Residency r;
    if (hln::residency(f, block, 0, r) != HLN_OK) return 0;
    if (r.bound < 1) {
        hln::fail(HLN_EUNSUPPORTED, "kernel does not fit a compute unit (%d VGPRs, %d B LDS, block %d)", r.vgprs,
                  r.lds, block);
        return 0;
    }
    int per_cu = std::min(r.bound, std::max(1, 1024 / block));
    if (const char* e = getenv("HLN_BLOCKS_PER_CU")) {
        const int want = atoi(e);
        if (want < 1 || want > r.bound) {
            hln::fail(HLN_EUNSUPPORTED, "HLN_BLOCKS_PER_CU=%d is outside [1, %d] (the co-residency bound: %d VGPRs, "
                                        "%d B LDS, block %d)", want, r.bound, r.vgprs, r.lds, block);
            return 0;
        }
        per_cu = want;
    }
    return per_cu;
}

template <int NW, int BLOCK>
hln_status dispatch(const BfsArgs& a, bool ps, int want, int grid_cap, int cus, hipStream_t st) {
    const void* f = ps ? closeness_fn<NW, BLOCK, true>() : closeness_fn<NW, BLOCK, false>();
    const int per_cu = blocks_per_cu(f, BLOCK);
    if (per_cu < 1) return HLN_EUNSUPPORTED;
    const int bound_grid = per_cu * cus;
    const int grid = std::max(1, std::min({want, bound_grid, grid_cap}));
    if (getenv("HLN_VERBOSE"))
        fprintf(stderr, "[hln] closeness NW=%d block=%d per_source=%d n=%d n_src=%d grid=%d\n", NW, BLOCK,
                ps ? 1 : 0, a.n, a.n_src, grid);
    void* kargs[] = {const_cast<BfsArgs*>(&a)};
    return launch_persistent(f, grid, BLOCK, kargs, bound_grid, st);
}

template <int NW, int BLOCK>
bool fits(bool ps) {
    hln::Residency r;
    const void* f = ps ? closeness_fn<NW, BLOCK, true>() : closeness_fn<NW, BLOCK, false>();
    return hln::residency(f, BLOCK, 0, r) == HLN_OK && r.bound >= 1;
}

// Block size: 1024 threads by default (fewest barrier participants for the
// same number of waves), smaller if the kernel's registers do not allow it.
template <int NW>
hln_status dispatch_block(const BfsArgs& a, bool ps, long long want_threads, int grid_cap, int cus, hipStream_t st) {
    int block = 1024;
    if (const char* e = getenv("HLN_BLOCK")) block = atoi(e);
    if (block >= 1024 && !fits<NW, 1024>(ps)) block = 512;
    if (block >= 512 && block < 1024 && !fits<NW, 512>(ps)) block = 256;
    auto want = [&](int b) { return static_cast<int>(std::min<long long>((want_threads + b - 1) / b, 1 << 20)); };
    switch (block) {
        case 256: return dispatch<NW, 256>(a, ps, want(256), grid_cap, cus, st);
        case 512: return dispatch<NW, 512>(a, ps, want(512), grid_cap, cus, st);
        default: return dispatch<NW, 1024>(a, ps, want(1024), grid_cap, cus, st);
    }
}

int width_words(const hln_opts* o) {
    int w = (o && o->width_bits) ? o->width_bits : 512;
    switch (w) {
        case 64: return 1;
        case 128: return 2;
        case 256: return 4;
        case 512: return 8;
        case 1024: return 16;
        case 2048: return 32;
        case 4096: return 64;
        default: return 0;
    }
}

size_t workspace_bytes(int32_t n, int64_t nnz, int nw, int grid_cap, int32_t n_src) {
    using hln::Arena;
    size_t words = static_cast<size_t>(n) * nw;
    size_t seg_cap = static_cast<size_t>(n) + static_cast<size_t>(nnz / kSegLen) + 1;
    size_t b = 0;
    b += Arena::round(sizeof(Ctrl));
    b += Arena::round(hln::dev::kBarrierWords * sizeof(unsigned long long));
    b += 4 * Arena::round(words * sizeof(uint64_t));            // A, B, vis, hacc
    b += 2 * Arena::round(static_cast<size_t>(n) * 8);          // word masks of A, B
    b += 3 * Arena::round(static_cast<size_t>(n) * sizeof(int32_t)); // hcnt, seg_first, S32
    b += Arena::round(seg_cap * sizeof(int4));
    b += Arena::round(seg_cap * sizeof(uint32_t));                    // saturated segments
    b += Arena::round(static_cast<size_t>(n) * sizeof(uint32_t));    // probe component membership
    b += Arena::round(static_cast<size_t>(grid_cap) * 2 * 64 * nw * sizeof(int64_t));  // per-source partials
    b += 2 * Arena::round(static_cast<size_t>(std::max(n, n_src)) * sizeof(int32_t));   // perm, iperm
    b += Arena::round(static_cast<size_t>(grid_cap) * std::max(kRankClasses, kDistClasses) * sizeof(int32_t)); // per-block class counts
    return b;
}

int grid_cap_for(int cus) { return cus * 4; }

// Carves one graph's working set out of `workspace` (laid out as
// workspace_bytes() counts it) and fills its launch arguments.
hln_status fill_args(BfsArgs& a, const hln_csr* g, const int32_t* sources, int32_t n_src, bool per_vertex, int nw,
                     const hln_opts* opts, int64_t* S, int32_t* R, double* cc, int32_t* h2, void* workspace,
                     size_t workspace_bytes_in, int grid_cap, int* fault) {
    using hln::fail;
    a = BfsArgs{};
    const int n = g->n;
    hln::Arena ar{static_cast<char*>(workspace), workspace_bytes_in};
    const size_t words = static_cast<size_t>(n) * nw;
    a.n = n;
    a.n_src = n_src;
    a.row_ptr = g->row_ptr;
    a.col_idx = g->col_idx;
    a.sources = sources;
    a.listed = (sources != nullptr || per_vertex) ? 1 : 0;
    a.ctrl = ar.take<Ctrl>(1);
    a.bar = ar.take<unsigned long long>(hln::dev::kBarrierWords);
    a.bufA = ar.take<uint64_t>(words);
    a.bufB = ar.take<uint64_t>(words);
    a.vis = ar.take<uint64_t>(words);
    a.hacc = ar.take<uint64_t>(words);
    a.flagA = ar.take<uint64_t>(n);
    a.flagB = ar.take<uint64_t>(n);
    a.hcnt = ar.take<int32_t>(n);
    a.seg_cap = static_cast<long long>(n) + g->nnz / kSegLen + 1;
    a.seg = ar.take<int4>(static_cast<size_t>(a.seg_cap));
    a.segsat = ar.take<uint32_t>(static_cast<size_t>(a.seg_cap));
    a.member = ar.take<uint32_t>(n);
    a.seg_first = ar.take<int32_t>(n);
    a.S32 = ar.take<uint32_t>(n);
    a.nnz_cap = g->nnz;
    a.part = ar.take<int64_t>(static_cast<size_t>(grid_cap) * 2 * 64 * nw);
    a.perm = ar.take<int32_t>(static_cast<size_t>(std::max(n, n_src)));
    a.iperm = ar.take<int32_t>(static_cast<size_t>(std::max(n, n_src)));
    a.bcount = ar.take<int32_t>(static_cast<size_t>(grid_cap) * std::max(kRankClasses, kDistClasses));
    a.S = S;
    a.R = R;
    a.H2 = h2;
    a.cc = cc;
    a.fault = fault;
    a.wait_ticks = 1000000000ull;   // 10 s at 100 MHz
    a.direction = opts ? opts->direction : 0;
    a.levels = opts ? opts->levels : nullptr;
    a.trace = opts ? opts->trace : nullptr;
    a.trace_cap = opts ? opts->trace_cap : 0;
    a.seg_len = kSegLen;
    // Automatic direction: with all sources at W = 4096 every level runs
    // bottom-up (its sweep leaves long-saturated segments out, so a nearly
    // finished level costs less than a push's two barriers, and level 1 reads
    // ids only); listed sources and narrower widths push when 32 * frontier
    // arc-words < arcs (a listed batch's first frontier is a few thousand
    // vertices of a large graph).  Measured on configs 2-5.
    a.alpha = (nw == 64 && !a.listed) ? 0 : 32;
    if (const char* e = getenv("HLN_ALPHA")) a.alpha = std::max(1, atoi(e));
    a.s32_levels = kS32Levels;
    if (const char* e = getenv("HLN_S32_LEVELS")) a.s32_levels = std::min(kS32Levels, std::max(1, atoi(e)));
    if (!a.ctrl || !a.bar || !a.part || !a.flagB || !a.seg_first || !a.S32 || !a.segsat || !a.member || !a.perm ||
        !a.iperm || !a.bcount)
        return fail(HLN_ENOMEM, "workspace carve failed");
    return HLN_OK;
}


// Scratch of hln_closeness_layer_static: one array per device, which the
// runtime allocates with the code object and keeps until the process ends.
// Host code never uses this name as an address: the array's device address
// on the current device comes from hipGetSymbolAddress (static_scratch()).
constexpr size_t kStaticScratchBytes = size_t(HLN_STATIC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current), or nullptr with the error set.
void* static_scratch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) {
        hln::fail(HLN_EDEVICE, "hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            hln::fail(HLN_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

hln_status hln_closeness_layer_static(const hln_csr* g, const int32_t* sources, int32_t n_src, const hln_opts* opts,
                                      int64_t* S, int32_t* R, double* cc, int32_t* h2, void* stream) {
    using hln::fail;
    hln::clear_error();
    if (!g) return fail(HLN_EINVAL, "graph is NULL");
    if (g->n < 1 || g->nnz < 0) return fail(HLN_EINVAL, "bad graph size (n %d, nnz %lld)", g->n, (long long)g->nnz);
    const int nw = width_words(opts);
    if (nw == 0) return fail(HLN_EINVAL, "width_bits must be 64, 128, 256, 512, 1024, 2048 or 4096");
    const hln::DeviceInfo* di = hln::device_info();
    if (!di) return HLN_EDEVICE;
    const size_t need = workspace_bytes(g->n, g->nnz, nw, grid_cap_for(di->cus), std::max(n_src, 0));
    if (need > kStaticScratchBytes)
        return fail(HLN_ENOMEM, "graph needs %zu bytes of scratch, more than the static %zu (n %d, nnz %lld, width %d): "
                                "use hln_closeness_layer with a workspace", need, kStaticScratchBytes, g->n,
                    (long long)g->nnz, nw * 64);
    void* ptr = static_scratch();
    if (!ptr) return HLN_EDEVICE;
    // the same kernels as hln_closeness_layer, on the static scratch; they
    // clear everything they read before using it (control block and barrier
    // words by k_zero_ctrl, the rest in phase 0), so the previous call's
    // contents do not matter
    return hln_closeness_layer(g, sources, n_src, opts, S, R, cc, h2, ptr, kStaticScratchBytes, stream);
}

hln_status hln_closeness_kernel_residency(int32_t width_bits, int32_t block_threads, int32_t mode, int32_t* info) {
    using hln::fail;
    hln::clear_error();
    if (!info) return fail(HLN_EINVAL, "info is NULL");
    hln_opts o{width_bits, 0, 0, nullptr, nullptr, 0};
    const int nw = width_words(&o);
    if (nw == 0) return fail(HLN_EINVAL, "bad width %d", width_bits);
    if (mode < 0 || mode > 3) return fail(HLN_EINVAL, "mode must be 0, 1, 2 or 3");
    if (block_threads != 256 && block_threads != 512 && block_threads != 1024)
        return fail(HLN_EINVAL, "block must be 256, 512 or 1024");
    const void* f = nullptr;
    auto pick = [&](auto nwc) {
        constexpr int N = decltype(nwc)::value;
        if (mode >= 2) {
            if constexpr (N == 8 || N == 16 || N == 32 || N == 64) {
                if (block_threads == 1024)
                    f = mode == 3 ? reinterpret_cast<const void*>(&k_closeness_multi<N, 1024, true>)
                                  : reinterpret_cast<const void*>(&k_closeness_multi<N, 1024, false>);
            }
            return;
        }
        const bool ps = mode == 1;
        switch (block_threads) {
            case 256: f = ps ? closeness_fn<N, 256, true>() : closeness_fn<N, 256, false>(); break;
            case 512: f = ps ? closeness_fn<N, 512, true>() : closeness_fn<N, 512, false>(); break;
            default: f = ps ? closeness_fn<N, 1024, true>() : closeness_fn<N, 1024, false>(); break;
        }
    };
    switch (nw) {
        case 1: pick(std::integral_constant<int, 1>{}); break;
        case 2: pick(std::integral_constant<int, 2>{}); break;
        case 4: pick(std::integral_constant<int, 4>{}); break;
        case 8: pick(std::integral_constant<int, 8>{}); break;
        case 16: pick(std::integral_constant<int, 16>{}); break;
        case 32: pick(std::integral_constant<int, 32>{}); break;
        default: pick(std::integral_constant<int, 64>{}); break;
    }
    if (!f) return fail(HLN_EUNSUPPORTED, "no such kernel (multi-graph: widths 512-4096, block 1024)");
    hln::Residency r;
    const hln_status st = hln::residency(f, block_threads, 0, r);
    if (st != HLN_OK) return st;
    info[0] = r.vgprs;
    info[1] = r.lds;
    info[2] = r.scratch;
    info[3] = r.query;
    info[4] = r.bound;
    return HLN_OK;
}

size_t hln_closeness_workspace_size(int32_t n, int64_t nnz, int32_t n_src, const hln_opts* opts) {
    int nw = width_words(opts);
    if (nw == 0 || n < 0 || nnz < 0 || n_src < 0) return 0;
    const hln::DeviceInfo* di = hln::device_info();
    int cus = di ? di->cus : 256;
    return workspace_bytes(n, nnz, nw, grid_cap_for(cus), n_src);
}

hln_status hln_closeness_layer(const hln_csr* g, const int32_t* sources, int32_t n_src, const hln_opts* opts,
                               int64_t* S, int32_t* R, double* cc, int32_t* h2, void* workspace,
                               size_t workspace_bytes_in, void* stream) {
    using hln::fail;
    hln::clear_error();
    if (!g) return fail(HLN_EINVAL, "graph is NULL");
    if (g->n < 1) return fail(HLN_EINVAL, "n must be >= 1 (got %d)", g->n);
    if (g->nnz < 0 || g->nnz > 0x7fffffffLL) return fail(HLN_EINVAL, "nnz out of range (%lld)", (long long)g->nnz);
    if (!g->row_ptr || (g->nnz > 0 && !g->col_idx)) return fail(HLN_EINVAL, "graph arrays are NULL");
    if (!S || !R) return fail(HLN_EINVAL, "S and R outputs are required");
    const int32_t flags = opts ? opts->flags : 0;
    if (flags & ~HLN_FLAG_PER_VERTEX) return fail(HLN_EINVAL, "unknown opts->flags bits 0x%x", flags);
    const bool per_vertex = (flags & HLN_FLAG_PER_VERTEX) != 0;
    if (n_src < 0) return fail(HLN_EINVAL, "n_src < 0");
    // per-vertex sums always take a list; an empty one may be NULL
    if (per_vertex && !sources && n_src > 0) return fail(HLN_EINVAL, "HLN_FLAG_PER_VERTEX needs listed sources");
    // NULL with n_src == n is all-source; NULL with n_src == 0 an empty list (n >= 1)
    if (!sources && !per_vertex && n_src != g->n && n_src != 0)
        return fail(HLN_EINVAL, "all-source mode needs n_src == n (%d != %d)", n_src, g->n);
    if ((sources || per_vertex) && h2) return fail(HLN_EUNSUPPORTED, "h2 is produced in all-source mode only");
    if (per_vertex && cc) return fail(HLN_EINVAL, "HLN_FLAG_PER_VERTEX gives sums only: cc must be NULL");
    if (opts && (opts->direction < 0 || opts->direction > 2)) return fail(HLN_EINVAL, "bad direction %d", opts->direction);
    const int nw = width_words(opts);
    if (nw == 0) return fail(HLN_EINVAL, "width_bits must be 64, 128, 256, 512, 1024, 2048 or 4096");
    if (g->nnz >= (1LL << 29) || static_cast<long long>(g->n) + g->nnz / kSegLen + 1 >= (1LL << 27))
        return fail(HLN_EUNSUPPORTED, "graph too large for 32-bit buffer offsets (nnz %lld)", (long long)g->nnz);
    if (static_cast<long long>(g->n) * nw * 8 >= (1LL << 31))
        return fail(HLN_EUNSUPPORTED, "n * width_bits / 8 must be below 2^31 bytes (n = %d, width %d): use a narrower width",
                    g->n, nw * 64);
    if (!workspace) return fail(HLN_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % hln::Arena::kAlign) return fail(HLN_EINVAL, "workspace not 256-byte aligned");
    const hln::DeviceInfo* di = hln::device_info();
    if (!di) return HLN_EDEVICE;
    const int grid_cap = grid_cap_for(di->cus);
    const size_t need = workspace_bytes(g->n, g->nnz, nw, grid_cap, n_src);
    if (workspace_bytes_in < need)
        return fail(HLN_ENOMEM, "workspace too small: %zu < %zu bytes", workspace_bytes_in, need);
    if (n_src == 0 && !per_vertex) return HLN_OK;    // per-vertex mode still writes zero sums
    int* fault = hln::fault_word();
    if (!fault) return HLN_EDEVICE;

    BfsArgs a{};
    {
        const hln_status fs = fill_args(a, g, sources, n_src, per_vertex, nw, opts, S, R, cc, h2, workspace,
                                        workspace_bytes_in, grid_cap, fault);
        if (fs != HLN_OK) return fs;
    }
    const int n = g->n;

    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_zero_ctrl, dim3(1), dim3(256), 0, st, a.ctrl, a.bar);
    HLN_TRY_HIP(hipGetLastError());

    // enough groups to cover the segments, capped by co-residency
    const long long want_threads = (static_cast<long long>(n) + g->nnz / kSegLen + 1) * std::max(8, nw);
    const bool ps = sources != nullptr && !per_vertex;
    switch (nw) {
        case 1: return dispatch_block<1>(a, ps, want_threads, grid_cap, di->cus, st);
        case 2: return dispatch_block<2>(a, ps, want_threads, grid_cap, di->cus, st);
        case 4: return dispatch_block<4>(a, ps, want_threads, grid_cap, di->cus, st);
        case 8: return dispatch_block<8>(a, ps, want_threads, grid_cap, di->cus, st);
        case 16: return dispatch_block<16>(a, ps, want_threads, grid_cap, di->cus, st);
        case 32: return dispatch_block<32>(a, ps, want_threads, grid_cap, di->cus, st);
        case 64: return dispatch_block<64>(a, ps, want_threads, grid_cap, di->cus, st);
        default: return fail(HLN_EINVAL, "unsupported width");
    }
}

}  // extern "C"

namespace {

template <int NW, bool PS>
hln_status launch_multi(const void* args_dev, const int* plist_dev, const int* pfirst_dev, int parts, int cus,
                        hipStream_t st) {
    constexpr int BLOCK = 1024;
    const void* f = reinterpret_cast<const void*>(&k_closeness_multi<NW, BLOCK, PS>);
    const int per_cu = blocks_per_cu(f, BLOCK);
    if (per_cu < 1) return HLN_EUNSUPPORTED;
    // one block per compute unit, as the single-graph launch; a whole number
    // of rounds of partitions
    const int grid = std::max(parts, (cus / parts) * parts);
    if (getenv("HLN_VERBOSE"))
        fprintf(stderr, "[hln] closeness multi NW=%d per_source=%d parts=%d grid=%d\n", NW, PS ? 1 : 0, parts, grid);
    const BfsArgs* args = static_cast<const BfsArgs*>(args_dev);
    hipLaunchKernelGGL(k_zero_parts, dim3(parts), dim3(256), 0, st, args, plist_dev, pfirst_dev);
    HLN_TRY_HIP(hipGetLastError());
    void* kargs[] = {const_cast<BfsArgs**>(&args), const_cast<int**>(&plist_dev), const_cast<int**>(&pfirst_dev),
                     &parts};
    return launch_persistent(f, grid, BLOCK, kargs, per_cu * cus, st);
}

}  // namespace

namespace hln {

size_t multi_args_bytes(int n_graphs) { return sizeof(BfsArgs) * static_cast<size_t>(n_graphs > 0 ? n_graphs : 1); }

size_t multi_slice_bytes(int32_t n, int64_t nnz, int width_bits) {
    hln_opts o{width_bits, 0, 0, nullptr, nullptr, 0};
    const int nw = width_words(&o);
    if (nw == 0 || n < 1 || nnz < 0) return 0;
    const DeviceInfo* di = device_info();
    return Arena::round(workspace_bytes(n, nnz, nw, grid_cap_for(di ? di->cus : 256), n));
}

hln_status multi_fill(const hln_csr& g, const int32_t* sources, int32_t n_src, int64_t* S, int32_t* R, double* cc,
                      int32_t* h2, int width_bits, void* slice, size_t slice_bytes, void* args_host, int index) {
    hln_opts o{width_bits, 0, 0, nullptr, nullptr, 0};
    const int nw = width_words(&o);
    if (nw == 0) return fail(HLN_EINVAL, "unsupported width %d", width_bits);
    if (g.nnz >= (1LL << 29) || static_cast<long long>(g.n) + g.nnz / kSegLen + 1 >= (1LL << 27) ||
        static_cast<long long>(g.n) * nw * 8 >= (1LL << 31))
        return fail(HLN_EUNSUPPORTED, "graph too large for 32-bit buffer offsets");
    const DeviceInfo* di = device_info();
    if (!di) return HLN_EDEVICE;
    int* fault = fault_word();
    if (!fault) return HLN_EDEVICE;
    if (sources && h2) return fail(HLN_EUNSUPPORTED, "h2 is produced in all-source mode only");
    BfsArgs* a = static_cast<BfsArgs*>(args_host) + index;
    return fill_args(*a, &g, sources, sources ? n_src : g.n, false, nw, &o, S, R, cc, h2, slice, slice_bytes,
                     grid_cap_for(di->cus), fault);
}

hln_status multi_launch(int width_bits, bool per_source, const void* args_dev, const int* plist_dev,
                        const int* pfirst_dev, int parts, hipStream_t st) {
    const DeviceInfo* di = device_info();
    if (!di) return HLN_EDEVICE;
    if (parts < 1 || parts > di->cus) return fail(HLN_EINVAL, "bad partition count %d", parts);
    const int c = di->cus;
    if (per_source) {
        switch (width_bits) {
            case 512: return launch_multi<8, true>(args_dev, plist_dev, pfirst_dev, parts, c, st);
            case 1024: return launch_multi<16, true>(args_dev, plist_dev, pfirst_dev, parts, c, st);
            case 2048: return launch_multi<32, true>(args_dev, plist_dev, pfirst_dev, parts, c, st);
            case 4096: return launch_multi<64, true>(args_dev, plist_dev, pfirst_dev, parts, c, st);
            default: return fail(HLN_EUNSUPPORTED, "multi-graph launch at width %d", width_bits);
        }
    }
    switch (width_bits) {
        case 512: return launch_multi<8, false>(args_dev, plist_dev, pfirst_dev, parts, c, st);
        case 1024: return launch_multi<16, false>(args_dev, plist_dev, pfirst_dev, parts, c, st);
        case 2048: return launch_multi<32, false>(args_dev, plist_dev, pfirst_dev, parts, c, st);
        case 4096: return launch_multi<64, false>(args_dev, plist_dev, pfirst_dev, parts, c, st);
        default: return fail(HLN_EUNSUPPORTED, "multi-graph launch at width %d", width_bits);
    }
}

}  // namespace hln
