// Runtime pieces of the C ABI: error strings, device facts, the device
// fault word and the status query.
#include "hln_internal.hpp"

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

}  // namespace hln

extern "C" {

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
