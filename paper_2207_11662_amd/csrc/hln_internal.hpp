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
};
// Facts about the current device (cached per device).
const DeviceInfo* device_info();

// Device address of the library's fault word on the current device; kernels
// store a nonzero code there when a bounded wait runs out or an input is
// out of range.  nullptr (with the error set) on failure.
int* fault_word();

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
// over the grid.  Two levels, so that no counter takes more than
// ~grid/kSubs arrivals:
//   bar[kSub*i]          sub-group i (blocks with blockIdx % kSubs == i):
//                        low 32 bits arrivals, high 32 bits flagged arrivals,
//   bar[kSub*kSubs]      the same for the last arrival of each sub-group,
//   bar[kSub*(kSubs+1)]  release word: 2*(barriers completed) + OR of flags,
//   bar[kSub*(kSubs+2)+i] flagged totals seen at the previous barrier.
// Counters grow monotonically during a launch (never reset) and sit 4 KB
// apart.  The wait is bounded in wall-clock time (s_memrealtime, 100 MHz):
// after `limit_ticks` the block records fault code 1; when another block has
// already recorded a fault it stops waiting.  Either way ok = false and the
// caller leaves the kernel, so every block exits.
constexpr int kSubs = 16;
constexpr int kSub = 512;                       // 4 KB of unsigned long long
constexpr int kBarrierWords = kSub * (kSubs + 3);

struct BarrierResult {
    bool ok;
    bool any;
};

__device__ __forceinline__ unsigned long long flagged_delta(unsigned long long* prev, unsigned long long total) {
    const unsigned long long before = load_agent(prev);
    __hip_atomic_store(prev, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);
    return total - before;
}

__device__ __forceinline__ BarrierResult grid_barrier_or(unsigned long long* bar, int flag, int* fault,
                                                         uint64_t limit_ticks) {
    __shared__ int s_ok;
    __shared__ int s_any;
    const int blk_flag = __syncthreads_or(flag);
    if (threadIdx.x == 0) {
        __threadfence();  // publish this block's writes device-wide
        const unsigned nb = gridDim.x;
        const unsigned groups = nb < kSubs ? nb : kSubs;
        const unsigned g = blockIdx.x % groups;
        const unsigned members = nb / groups + (g < nb % groups ? 1u : 0u);
        const unsigned long long add = 1ull + (blk_flag ? (1ull << 32) : 0ull);
        const unsigned long long old = atomic_add_agent(bar + kSub * g, add);
        const unsigned cnt = static_cast<unsigned>(old);
        const unsigned long long epoch = cnt / members + 1ull;   // barriers completed once this one is
        unsigned long long* release = bar + kSub * (kSubs + 1);
        int ok = 1;
        int any = 0;
        bool released = false;
        if (cnt % members == members - 1) {
            const unsigned long long d = flagged_delta(bar + kSub * (kSubs + 2) + g, (old + add) >> 32);
            const unsigned long long radd = 1ull + (d ? (1ull << 32) : 0ull);
            const unsigned long long r = atomic_add_agent(bar + kSub * kSubs, radd);
            if (static_cast<unsigned>(r) % groups == groups - 1) {
                const unsigned long long dr = flagged_delta(bar + kSub * (kSubs + 2) + kSubs, (r + radd) >> 32);
                any = dr != 0;
                __hip_atomic_store(release, 2ull * epoch + (any ? 1ull : 0ull), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                released = true;
            }
        }
        if (!released) {
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            unsigned long long rel;
            while (((rel = load_agent(release)) >> 1) < epoch) {
                __builtin_amdgcn_s_sleep(8);
                if (load_agent_i32(fault) != 0) {  // another block failed: keep its code
                    ok = 0;
                    break;
                }
                if (__builtin_amdgcn_s_memrealtime() - t0 > limit_ticks) {
                    store_agent_i32(fault, 1);
                    ok = 0;
                    break;
                }
            }
            any = static_cast<int>(rel & 1ull);
        }
        __threadfence();  // see every other block's writes
        s_ok = ok;
        s_any = any;
    }
    __syncthreads();
    return BarrierResult{s_ok != 0, s_any != 0};
}

__device__ __forceinline__ bool grid_barrier(unsigned long long* bar, int* fault, uint64_t limit_ticks) {
    return grid_barrier_or(bar, 0, fault, limit_ticks).ok;
}

}  // namespace dev
}  // namespace hln
