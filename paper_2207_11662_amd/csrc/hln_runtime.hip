// Runtime pieces of the C ABI: error strings, device facts, the device
// fault word and the status query.
#include "hln_internal.hpp"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <mutex>

namespace {

thread_local char t_error[512] = "";

// Fault word read back by hln_device_status; one copy per device (a
// device global), addressed through hipGetSymbolAddress.
__device__ int g_fault_word[64];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
hln::DeviceInfo g_info[kMaxDevices];
int* g_fault_ptr[kMaxDevices] = {};

}  // namespace

namespace hln {

hln_status fail(hln_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_error, sizeof(t_error), fmt, ap);
    va_end(ap);
    return s;
}

void clear_error() { t_error[0] = 0; }

const DeviceInfo* device_info() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        fail(HLN_EDEVICE, "hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceInfo& d = g_info[dev];
    if (d.device < 0) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
            fail(HLN_EDEVICE, "hipGetDeviceProperties failed");
            return nullptr;
        }
        d.cus = p.multiProcessorCount;
        d.max_threads_per_cu = p.maxThreadsPerMultiProcessor;
        d.lds_per_block = p.sharedMemPerBlock;
        d.lds_per_cu = p.maxSharedMemoryPerMultiProcessor > 0 ? p.maxSharedMemoryPerMultiProcessor : 160 * 1024;
        d.device = dev;
    }
    return &d;
}

int* fault_word() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        fail(HLN_EDEVICE, "hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_fault_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_fault_word));
        if (e != hipSuccess || !p) {
            fail(HLN_EDEVICE, "hipGetSymbolAddress(fault word) failed: %s", hipGetErrorString(e));
            return nullptr;
        }
        g_fault_ptr[dev] = static_cast<int*>(p);
    }
    return g_fault_ptr[dev];
}

int resident_blocks(int vgprs, size_t lds_bytes, int block, size_t lds_per_cu) {
    constexpr int kSimds = 4, kVgprFile = 512, kVgprGranule = 8, kMaxWavesPerSimd = 8;
    constexpr size_t kLdsGranule = 512;
    if (block < 1 || block > 1024 || vgprs < 0 || vgprs > kVgprFile) return 0;
    const int waves = (block + 63) / 64;
    const int slots = (waves + kSimds - 1) / kSimds;      // wave slots per SIMD per block
    const int alloc = std::max(kVgprGranule, (vgprs + kVgprGranule - 1) / kVgprGranule * kVgprGranule);
    const int waves_per_simd = std::min(kMaxWavesPerSimd, kVgprFile / alloc);
    int blocks = waves_per_simd / slots;
    if (lds_bytes > 0) {
        const size_t a = (lds_bytes + kLdsGranule - 1) / kLdsGranule * kLdsGranule;
        blocks = std::min<long long>(blocks, static_cast<long long>(lds_per_cu / a));
    }
    return blocks;
}

hln_status residency(const void* kernel, int block, size_t dyn_lds, Residency& r) {
    const DeviceInfo* di = device_info();
    if (!di) return HLN_EDEVICE;
    hipFuncAttributes at{};
    HLN_TRY_HIP(hipFuncGetAttributes(&at, kernel));
    int q = 0;
    HLN_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, kernel, block, dyn_lds));
    r.vgprs = at.numRegs;
    r.lds = static_cast<int>(at.sharedSizeBytes);
    r.scratch = static_cast<int>(at.localSizeBytes);
    r.query = q;
    r.bound = std::min(q, resident_blocks(at.numRegs, at.sharedSizeBytes + dyn_lds, block, di->lds_per_cu));
    return HLN_OK;
}

namespace {
thread_local int t_launch_path = 0;
}

void note_launch_path(int path) { t_launch_path = path; }

}  // namespace hln

extern "C" {

int32_t hln_resident_blocks(int32_t vgprs, int32_t lds_bytes, int32_t block_threads) {
    if (lds_bytes < 0) return 0;
    return hln::resident_blocks(vgprs, static_cast<size_t>(lds_bytes), block_threads, 160 * 1024);
}

int32_t hln_last_launch_path(void) { return hln::t_launch_path; }

const char* hln_last_error(void) { return t_error; }

int32_t hln_version(void) { return 0x000100; }

int32_t hln_device_cu_count(void) {
    const hln::DeviceInfo* d = hln::device_info();
    return d ? d->cus : 0;
}

hln_status hln_device_status(void* stream) {
    int* fw = hln::fault_word();
    if (!fw) return HLN_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HLN_TRY_HIP(hipStreamSynchronize(s));
    int code = 0;
    HLN_TRY_HIP(hipMemcpy(&code, fw, sizeof(int), hipMemcpyDeviceToHost));
    if (code != 0) {
        int zero = 0;
        HLN_TRY_HIP(hipMemcpy(fw, &zero, sizeof(int), hipMemcpyHostToDevice));
        return hln::fail(HLN_EDEVICE, "device-side fault code %d (1 = bounded wait ran out, 2 = id out of range)", code);
    }
    return HLN_OK;
}

}  // extern "C"
