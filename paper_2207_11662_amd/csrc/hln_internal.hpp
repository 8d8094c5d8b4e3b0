// Internal helpers shared by the library's translation units: error
// reporting, device facts, workspace carving and a few wave-level device
// primitives.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

#include "../../include/hln.h"

namespace hln {

// Records a printf-style message as this thread's last error and returns s.
hln_status fail(hln_status s, const char* fmt, ...);
void clear_error();

struct DeviceInfo {
    int device = -1;
    int cus = 0;
    int max_threads_per_cu = 0;
    size_t lds_per_block = 0;
    size_t lds_per_cu = 0;
};
// Facts about the current device (cached per device).
const DeviceInfo* device_info();

// Co-residency of a kernel's blocks on one compute unit (CDNA4: 4 SIMDs of
// 512 VGPRs per lane, allocated in granules of 8, at most 8 waves per SIMD;
// LDS allocated per block in granules of 512 bytes).  A block of B threads
// holds ceil(ceil(B/64) / 4) wave slots on each SIMD.
int resident_blocks(int vgprs, size_t lds_bytes, int block, size_t lds_per_cu);

// What a compiled kernel needs and how many of its blocks fit a compute
// unit: vgprs and lds from hipFuncGetAttributes (VGPRs per lane, static
// LDS per block; dynamic LDS is added by the caller through `dyn_lds`),
// scratch bytes per lane, the runtime's occupancy answer (`query`) and the
// bound a cooperative grid is held to: the smaller of that answer and
// resident_blocks() of the kernel's own registers and LDS.
struct Residency {
    int vgprs = 0;
    int lds = 0;
    int scratch = 0;
    int query = 0;
    int bound = 0;
};
hln_status residency(const void* kernel, int block, size_t dyn_lds, Residency& r);

// How the last persistent (grid-barrier) launch of this thread went out:
// 1 cooperative launch, 2 ordinary launch inside a stream capture (the
// runtime refused the cooperative one; the grid is within the residency
// bound).
void note_launch_path(int path);

// Device address of the library's fault word on the current device; kernels
// store a nonzero code there when a bounded wait runs out or an input is
// out of range.  nullptr (with the error set) on failure.
int* fault_word();

// Several graphs' closeness in one cooperative launch, for the batched path
// (hln_msbfs.hip): all graphs of a launch either use every source (sums
// per vertex) or a list of sources (sums per listed source, per_source).
// The caller stages an array of launch arguments (multi_args_bytes(n)
// bytes, filled on the host by multi_fill for each graph: its working set is
// carved from the workspace slice of the partition that runs it, each slice
// multi_slice_bytes() for the largest graph it serves) and, in device
// memory, the partitions' graph lists: plist (argument indices) and pfirst
// (parts + 1 offsets into plist).  Widths 512, 1024, 2048 and 4096.
size_t multi_args_bytes(int n_graphs);
size_t multi_slice_bytes(int32_t n, int64_t nnz, int width_bits);
hln_status multi_fill(const hln_csr& g, const int32_t* sources, int32_t n_src, int64_t* S, int32_t* R, double* cc,
                      int32_t* h2, int width_bits, void* slice, size_t slice_bytes, void* args_host, int index);
hln_status multi_launch(int width_bits, bool per_source, const void* args_dev, const int* plist_dev,
                        const int* pfirst_dev, int parts, hipStream_t st);

// Bump allocator over a caller workspace (256-byte alignment).
struct Arena {
    char* base;
    size_t size;
    size_t off = 0;
    static constexpr size_t kAlign = 256;
    static size_t round(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
    template <typename T>
    T* take(size_t count) {
        size_t b = round(count * sizeof(T));
        if (off + b > size) return nullptr;
        T* p = reinterpret_cast<T*>(base + off);
        off += b;
        return p;
    }
};

}  // namespace hln

#define HLN_TRY_HIP(call)                                                                  \
    do {                                                                                   \
        hipError_t hln_e_ = (call);                                                        \
        if (hln_e_ != hipSuccess)                                                          \
            return ::hln::fail(HLN_EDEVICE, "%s failed: %s", #call, hipGetErrorString(hln_e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// device-side helpers
// ---------------------------------------------------------------------------
namespace hln {
namespace dev {

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int mask) {
    int lo = __shfl_xor(static_cast<int>(static_cast<uint32_t>(x)), mask, 64);
    int hi = __shfl_xor(static_cast<int>(static_cast<uint32_t>(x >> 32)), mask, 64);
    return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

__device__ __forceinline__ int shfl_xor_i32(int x, int mask) { return __shfl_xor(x, mask, 64); }

// Agent-scope atomic helpers.
__device__ __forceinline__ unsigned long long atomic_add_agent(unsigned long long* p, unsigned long long v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long load_agent(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int load_agent_i32(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent_i32(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier for a cooperative launch that also ORs a per-block flag
// over the grid and hands every block one bit decided by the last arrival.
// Two levels, so that no counter takes more than ~grid/kSubs arrivals, and
// two counter sets used by alternate barriers (every block counts the
// barriers it has passed, so all agree on the parity):
//   bar[kSub*(i + kSubs*p)]      sub-group i (blocks with blockIdx % kSubs
//                                == i), parity p: low 32 bits arrivals,
//                                high 32 bits flagged arrivals;
//   bar[kSub*(2*kSubs + p)]      the same for the sub-groups' last arrivals;
//   bar[kSub*(2*kSubs + 2)]      release word: 4*(barriers completed) +
//                                2*decision + OR of the flags.
// The last arrival at a counter resets it to zero for the barrier after
// next (every block passes the next barrier first, so the reset is done
// before the counter's next use).  Words sit 4 KB apart.  `pre()` runs on
// each block's thread 0 after the block has synchronised and before it
// arrives (its memory operations complete before the arrival counts);
// `decide()` runs on the releasing thread after every block has arrived,
// and its result is returned to all blocks.  The wait is bounded in
// wall-clock time (s_memrealtime, 100 MHz): after `limit` ticks the block
// records fault code 1; when another block has already recorded a fault it
// stops waiting.  Either way ok = false and the caller leaves the kernel,
// so every block exits.
constexpr int kSubs = 16;
constexpr int kSub = 512;                       // 4 KB of unsigned long long
constexpr int kBarrierWords = kSub * (2 * kSubs + 3);

struct BarrierResult {
    bool ok;
    bool any;
    bool decision;
};

struct NoHook {
    __device__ void operator()() const {}
};
struct NoDecision {
    __device__ bool operator()() const { return false; }
};

// kWholeGrid: every block of the grid takes part (their number and this
// block's index come from the dispatch); otherwise `nb` blocks of one
// partition of the grid, this one being `bid` among them.
template <bool kWholeGrid>
struct GridBarrierT {
    unsigned long long* bar;
    int* fault;
    uint64_t limit;
    unsigned passed;                            // barriers this block has passed (thread 0's copy is used)
    unsigned nb_part;                           // partition only: blocks taking part
    unsigned bid_part;                          // partition only: this block's index among them

    template <class Pre = NoHook, class Decide = NoDecision>
    __device__ __forceinline__ BarrierResult sync(int flag, Pre pre = Pre(), Decide decide = Decide()) {
        __shared__ int s_ok;
        __shared__ int s_any;
        __shared__ int s_dec;
        const int blk_flag = __syncthreads_or(flag);
        if (threadIdx.x == 0) {
            pre();
            // release: this block's writes reach the device coherence point
            // (L2 write-back) before its arrival is counted
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned e = passed;
            const unsigned par = e & 1u;
            const unsigned nb = kWholeGrid ? gridDim.x : nb_part;
            const unsigned bid = kWholeGrid ? blockIdx.x : bid_part;
            const unsigned groups = nb < kSubs ? nb : kSubs;
            const unsigned g = bid % groups;
            const unsigned members = nb / groups + (g < nb % groups ? 1u : 0u);
            unsigned long long* sub = bar + kSub * (g + kSubs * par);
            unsigned long long* root = bar + kSub * (2 * kSubs + par);
            unsigned long long* release = bar + kSub * (2 * kSubs + 2);
            const unsigned long long add = 1ull + (blk_flag ? (1ull << 32) : 0ull);
            const unsigned long long old = atomic_add_agent(sub, add);
            int ok = 1;
            unsigned long long rel = 0;
            bool released = false;
            if (static_cast<unsigned>(old) == members - 1) {
                const unsigned long long radd = 1ull + (((old + add) >> 32) ? (1ull << 32) : 0ull);
                __hip_atomic_store(sub, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned long long r = atomic_add_agent(root, radd);
                if (static_cast<unsigned>(r) == groups - 1) {
                    const bool any = ((r + radd) >> 32) != 0;
                    __hip_atomic_store(root, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    // decide() reads agent-scope atomics only, which every
                    // block completed before its arrival
                    rel = 4ull * (e + 1ull) + (decide() ? 2ull : 0ull) + (any ? 1ull : 0ull);
                    __hip_atomic_store(release, rel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    released = true;
                }
            }
            if (!released) {
                const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                while (((rel = load_agent(release)) >> 2) < e + 1ull) {
                    __builtin_amdgcn_s_sleep(4);
                    if (load_agent_i32(fault) != 0) {  // another block failed: keep its code
                        ok = 0;
                        break;
                    }
                    if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
                        store_agent_i32(fault, 1);
                        ok = 0;
                        break;
                    }
                }
            }
            passed = e + 1;
            // acquire: drop stale L2 lines so that later loads see every
            // block's writes
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_ok = ok;
            s_any = static_cast<int>(rel & 1ull);
            s_dec = static_cast<int>((rel >> 1) & 1ull);
        }
        __syncthreads();
        return BarrierResult{s_ok != 0, s_any != 0, s_dec != 0};
    }

    __device__ __forceinline__ bool wait() { return sync(0).ok; }
};
using GridBarrier = GridBarrierT<true>;
using PartBarrier = GridBarrierT<false>;

}  // namespace dev
}  // namespace hln
