// Sampling-based estimate of every vertex's closeness (the linear-time
// sampling approximations of closeness that Sec. 2 cites: Eppstein and
// Wang's estimator, and Cohen et al.'s sampling for closeness at scale).
//
// Input: per-vertex sums over a sample Q of k distinct source vertices drawn
// uniformly from a population of n_pop vertices (the listed-source BFS with
// per-vertex sums gives them in one launch):
//   S[v] = sum over s in Q reaching v of d(s, v),
//   R[v] = number of s in Q reaching v (v itself counts when v is in Q).
// With q = R[v] - [v in Q] and k' = k - [v in Q], the sampled sources other
// than v are a uniform sample of the population without v, so
//   S[v] / q      estimates the mean distance from v to what it reaches,
//   q / k'        estimates the fraction of the population it reaches,
// and the Wasserman-Faust closeness (Eq. 1 in its disconnected-graph form)
// is estimated by
//   cc[v] = (q / S[v]) * (q / k') * ((n_pop - 1) / (n - 1)),
// rounded in that order (IEEE division, two multiplications), 0 when q = 0,
// S[v] = 0, k' = 0 or n = 1.  Vertices outside the population reach none of
// it and get 0.  When Q is every vertex (k = n_pop = n) the estimate is the
// exact closeness: q = R - 1, k' = n - 1.
//
// Three small launches on the caller's stream: zero cc, mark the sample
// (cc[s] = 1 as a flag), then every thread turns its own vertex's flag into
// the estimate.  No workspace.
#include "hln_internal.hpp"

#include <algorithm>

namespace {

constexpr int kBlock = 256;

__global__ void k_fill_zero(int n, double* cc) {
    for (long long v = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
         v += static_cast<long long>(gridDim.x) * blockDim.x)
        cc[v] = 0.0;
}

// An id outside [0, n) is fault code 2 and marks nothing.
__global__ void k_mark_sample(int n, int k, const int32_t* __restrict__ sources, double* cc, int* fault) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < k;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int s = sources[i];
        if (static_cast<unsigned>(s) < static_cast<unsigned>(n))
            cc[s] = 1.0;
        else
            hln::dev::store_agent_i32(fault, 2);
    }
}

__global__ void k_estimate(int n, int n_pop, int k, const int64_t* __restrict__ S, const int32_t* __restrict__ R,
                           double* cc) {
    for (long long v = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
         v += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int self = cc[v] != 0.0 ? 1 : 0;
        const int32_t q = R[v] - self;
        const int32_t kp = k - self;
        const int64_t sv = S[v];
        double c = 0.0;
        if (q > 0 && sv > 0 && kp > 0 && n > 1) {
            const double mean_inv = static_cast<double>(q) / static_cast<double>(sv);
            const double reach = static_cast<double>(q) / static_cast<double>(kp);
            const double pop = static_cast<double>(n_pop - 1) / static_cast<double>(n - 1);
            c = (mean_inv * reach) * pop;
        }
        cc[v] = c;
    }
}

int grid_for(long long items, int cus) {
    const long long g = (items + kBlock - 1) / kBlock;
    return static_cast<int>(std::max<long long>(1, std::min<long long>(g, static_cast<long long>(cus) * 16)));
}

}  // namespace

extern "C" {

hln_status hln_closeness_estimate(int32_t n, int32_t n_pop, const int32_t* sources, int32_t k, const int64_t* S,
                                  const int32_t* R, double* cc, void* stream) {
    using hln::fail;
    hln::clear_error();
    if (n < 1) return fail(HLN_EINVAL, "n must be >= 1 (got %d)", n);
    if (n_pop < 1 || n_pop > n) return fail(HLN_EINVAL, "n_pop must be in [1, n] (got %d, n = %d)", n_pop, n);
    if (k < 0 || k > n_pop) return fail(HLN_EINVAL, "k must be in [0, n_pop] (got %d, n_pop = %d)", k, n_pop);
    if (k > 0 && !sources) return fail(HLN_EINVAL, "sources is NULL");
    if (!S || !R || !cc) return fail(HLN_EINVAL, "S, R and cc are required");
    const hln::DeviceInfo* di = hln::device_info();
    if (!di) return HLN_EDEVICE;
    int* fault = hln::fault_word();
    if (!fault) return HLN_EDEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(n, di->cus)), dim3(kBlock), 0, st, n, cc);
    HLN_TRY_HIP(hipGetLastError());
    if (k > 0) {
        hipLaunchKernelGGL(k_mark_sample, dim3(grid_for(k, di->cus)), dim3(kBlock), 0, st, n, k, sources, cc, fault);
        HLN_TRY_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_estimate, dim3(grid_for(n, di->cus)), dim3(kBlock), 0, st, n, n_pop, k, S, R, cc);
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

}  // extern "C"
