// Learned candidate proposer: a small FP32 MLP that ranks vertices for
// exact closeness in the AND graph from per-layer quantities the method has
// already computed (the Psi step: degree, distance sums and reach, 2-hop
// count).  Its
// top candidates are then scored by exact BFS on the AND graph; the
// exhaustive computation stays the fallback and the precision reference.
// (Not in the paper: the features echo CC1's degree bound, Sec. 5.1, and
// CC2's per-layer distance sums, Sec. 5.2.)
//
// Model: 12 features -> 64 ReLU -> 64 ReLU -> 1, FP32.  Parameters, in
// order: W1[12][64], b1[64], W2[64][64], b2[64], w3[64], b3.
// Training step (mean squared error): a block takes 64 vertices, runs the
// forward and backward passes with activations in LDS, and writes its
// partial gradient; one kernel then sums the partials over blocks in block
// order (deterministic) and applies Adam.
#include "hln_internal.hpp"
#include "hln_prim.hpp"

#include <algorithm>
#include <cmath>

namespace {

constexpr int F = 12;
constexpr int NQ = 3;                          // per-layer quantities
constexpr int H = 64;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + F * H;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + H;
constexpr int NPARAM = OFF_B3 + 1;            // 5057
constexpr int TB = 64;                         // vertices per training block
constexpr int BLK = 256;
constexpr int kMaxLayers = 64;

struct Layers {
    int r;
    const int32_t* rp[kMaxLayers];
    const int64_t* S[kMaxLayers];
    const int32_t* R[kMaxLayers];
    const int32_t* h2[kMaxLayers];
    float inv_mean_deg[kMaxLayers];
};

// Per layer and vertex: log1p(deg / mean degree); the Wasserman-Faust
// closeness ((R-1)/S)((R-1)/(n-1)) (Sec. 4, Eq. 1); log1p(h2 / mean
// degree^2).
__device__ __forceinline__ void layer_values(const Layers& L, int l, int u, int n, float v[NQ]) {
    const float deg = static_cast<float>(L.rp[l][u + 1] - L.rp[l][u]);
    const double S = static_cast<double>(L.S[l][u]);
    const double R = static_cast<double>(L.R[l][u]);
    const double nm1 = static_cast<double>(n - 1);
    v[0] = log1pf(deg * L.inv_mean_deg[l]);
    v[1] = (R > 1.0 && n > 1) ? static_cast<float>(((R - 1.0) / S) * ((R - 1.0) / nm1)) : 0.f;
    v[2] = log1pf(static_cast<float>(L.h2[l][u]) * L.inv_mean_deg[l] * L.inv_mean_deg[l]);
}

// 12 features per vertex: min, max, mean and standard deviation of each
// quantity over the r layers (two passes, so that the deviation does not
// cancel against the mean).
__global__ void k_features(int n, Layers L, float* X) {
    for (long long uu = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; uu < n;
         uu += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int u = static_cast<int>(uu);
        float mn[NQ], mx[NQ], sm[NQ], sq[NQ];
        for (int q = 0; q < NQ; ++q) {
            mn[q] = 3.4e38f;
            mx[q] = -3.4e38f;
            sm[q] = 0.f;
            sq[q] = 0.f;
        }
        for (int l = 0; l < L.r; ++l) {
            float v[NQ];
            layer_values(L, l, u, n, v);
            for (int q = 0; q < NQ; ++q) {
                mn[q] = fminf(mn[q], v[q]);
                mx[q] = fmaxf(mx[q], v[q]);
                sm[q] += v[q];
            }
        }
        const float inv_r = 1.0f / static_cast<float>(L.r);
        for (int q = 0; q < NQ; ++q) sm[q] *= inv_r;
        for (int l = 0; l < L.r; ++l) {
            float v[NQ];
            layer_values(L, l, u, n, v);
            for (int q = 0; q < NQ; ++q) {
                const float d = v[q] - sm[q];
                sq[q] = fmaf(d, d, sq[q]);
            }
        }
        float* x = X + static_cast<size_t>(u) * F;
        for (int q = 0; q < NQ; ++q) {
            x[4 * q + 0] = mn[q];
            x[4 * q + 1] = mx[q];
            x[4 * q + 2] = sm[q];
            x[4 * q + 3] = sqrtf(sq[q] * inv_r);
        }
    }
}

__device__ __forceinline__ void load_params(const float* __restrict__ p, float* s_p) {
    for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) s_p[i] = p[i];
    __syncthreads();
}

// one thread per vertex
__global__ __launch_bounds__(BLK) void k_mlp_fwd(const float* __restrict__ params, const float* __restrict__ X, int n,
                                                 float* y) {
    __shared__ float s_p[NPARAM];
    load_params(params, s_p);
    for (long long uu = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; uu < n;
         uu += static_cast<long long>(gridDim.x) * blockDim.x) {
        const float* x = X + static_cast<size_t>(uu) * F;
        float xf[F];
        for (int f = 0; f < F; ++f) xf[f] = x[f];
        float h1[H];
        for (int j = 0; j < H; ++j) {
            float a = s_p[OFF_B1 + j];
            for (int f = 0; f < F; ++f) a = fmaf(xf[f], s_p[OFF_W1 + f * H + j], a);
            h1[j] = fmaxf(a, 0.f);
        }
        float out = s_p[OFF_B3];
        for (int j = 0; j < H; ++j) {
            float a = s_p[OFF_B2 + j];
            for (int k = 0; k < H; ++k) a = fmaf(h1[k], s_p[OFF_W2 + k * H + j], a);
            out = fmaf(fmaxf(a, 0.f), s_p[OFF_W3 + j], out);
        }
        y[uu] = out;
    }
}

// Forward + backward for 64 vertices per block; partial gradient of the
// block's share of the loss  (1/N) * sum (y - t)^2  to part[block][NPARAM],
// partial loss to lpart[block].
__global__ __launch_bounds__(BLK) void k_mlp_grad(const float* __restrict__ params, const float* __restrict__ X,
                                                  const float* __restrict__ target, int n, float inv_n,
                                                  float* part, float* lpart) {
    __shared__ float s_p[NPARAM];
    __shared__ float s_x[TB][F];
    __shared__ float s_h1[TB][H];
    __shared__ float s_h2[TB][H];
    __shared__ float s_d2[TB][H];
    __shared__ float s_d1[TB][H];
    __shared__ float s_dy[TB];
    load_params(params, s_p);
    const int base = blockIdx.x * TB;
    const int t = threadIdx.x;
    for (int i = t; i < TB * F; i += BLK) {
        const int v = base + i / F;
        s_x[i / F][i % F] = v < n ? X[static_cast<size_t>(v) * F + i % F] : 0.f;
    }
    __syncthreads();
    // thread t: vertex i = t / 4, units c*16 .. c*16+15
    const int i = t >> 2;
    const int c0 = (t & 3) * 16;
    for (int j = c0; j < c0 + 16; ++j) {
        float a = s_p[OFF_B1 + j];
        for (int f = 0; f < F; ++f) a = fmaf(s_x[i][f], s_p[OFF_W1 + f * H + j], a);
        s_h1[i][j] = fmaxf(a, 0.f);
    }
    __syncthreads();
    for (int j = c0; j < c0 + 16; ++j) {
        float a = s_p[OFF_B2 + j];
        for (int k = 0; k < H; ++k) a = fmaf(s_h1[i][k], s_p[OFF_W2 + k * H + j], a);
        s_h2[i][j] = fmaxf(a, 0.f);
    }
    __syncthreads();
    if (t < TB) {
        float y = s_p[OFF_B3];
        for (int j = 0; j < H; ++j) y = fmaf(s_h2[t][j], s_p[OFF_W3 + j], y);
        const int v = base + t;
        const float r = v < n ? y - target[v] : 0.f;
        s_dy[t] = 2.f * r * inv_n;
        // this vertex's share of the loss, summed below by thread 0 in
        // vertex order (s_d1 is free until the backward pass)
        s_d1[t][0] = r * r * inv_n;
    }
    __syncthreads();
    if (t == 0) {
        float l = 0.f;
        for (int k = 0; k < TB; ++k) l += s_d1[k][0];
        lpart[blockIdx.x] = l;
    }
    __syncthreads();
    for (int j = c0; j < c0 + 16; ++j)
        s_d2[i][j] = s_h2[i][j] > 0.f ? s_dy[i] * s_p[OFF_W3 + j] : 0.f;
    __syncthreads();
    for (int k = c0; k < c0 + 16; ++k) {
        float a = 0.f;
        for (int j = 0; j < H; ++j) a = fmaf(s_d2[i][j], s_p[OFF_W2 + k * H + j], a);
        s_d1[i][k] = s_h1[i][k] > 0.f ? a : 0.f;
    }
    __syncthreads();
    float* g = part + static_cast<size_t>(blockIdx.x) * NPARAM;
    // dW2[k][j] = sum_i h1[i][k] d2[i][j]: 16 entries per thread
    for (int e = t; e < H * H; e += BLK) {
        const int k = e / H, j = e % H;
        float a = 0.f;
        for (int q = 0; q < TB; ++q) a = fmaf(s_h1[q][k], s_d2[q][j], a);
        g[OFF_W2 + e] = a;
    }
    for (int e = t; e < F * H; e += BLK) {
        const int f = e / H, k = e % H;
        float a = 0.f;
        for (int q = 0; q < TB; ++q) a = fmaf(s_x[q][f], s_d1[q][k], a);
        g[OFF_W1 + e] = a;
    }
    if (t < H) {
        float a1 = 0.f, a2 = 0.f, a3 = 0.f;
        for (int q = 0; q < TB; ++q) {
            a1 += s_d1[q][t];
            a2 += s_d2[q][t];
            a3 = fmaf(s_h2[q][t], s_dy[q], a3);
        }
        g[OFF_B1 + t] = a1;
        g[OFF_B2 + t] = a2;
        g[OFF_W3 + t] = a3;
    }
    if (t == 0) {
        float a = 0.f;
        for (int q = 0; q < TB; ++q) a += s_dy[q];
        g[OFF_B3] = a;
    }
}

// sum partial gradients over blocks in order, then one Adam step
__global__ void k_mlp_adam(float* params, float* m, float* v, const float* __restrict__ part, int nblocks, int step,
                           float lr, float b1, float b2, float eps, const float* lpart, float* loss_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NPARAM) {
        float g = 0.f;
        for (int b = 0; b < nblocks; ++b) g += part[static_cast<size_t>(b) * NPARAM + p];
        const float mm = b1 * m[p] + (1.f - b1) * g;
        const float vv = b2 * v[p] + (1.f - b2) * g * g;
        m[p] = mm;
        v[p] = vv;
        const float mh = mm / (1.f - powf(b1, static_cast<float>(step)));
        const float vh = vv / (1.f - powf(b2, static_cast<float>(step)));
        params[p] -= lr * mh / (sqrtf(vh) + eps);
    }
    if (p == 0 && loss_out) {
        float l = 0.f;
        for (int b = 0; b < nblocks; ++b) l += lpart[b];
        *loss_out = l;
    }
}

// splitmix64 (Steele, Lea, Flood 2014) as a counter-based generator
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

// Glorot-uniform weights, zero biases, zero Adam moments
__global__ void k_mlp_init(float* params, float* m, float* v, unsigned long long seed) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    float val = 0.f;
    float fan = 0.f;
    if (p < OFF_B1) fan = F + H;
    else if (p >= OFF_W2 && p < OFF_B2) fan = H + H;
    else if (p >= OFF_W3 && p < OFF_B3) fan = H + 1;
    if (fan > 0.f) {
        const unsigned long long r = splitmix64(seed * 0x100000001b3ull + static_cast<unsigned long long>(p));
        const float u = static_cast<float>(r >> 40) * (1.0f / 16777216.0f);     // [0, 1)
        const float lim = sqrtf(6.0f / fan);
        val = (2.f * u - 1.f) * lim;
    }
    params[p] = val;
    if (m) m[p] = 0.f;
    if (v) v[p] = 0.f;
}

// ---- generic top-k of scores (descending, ties by ascending index) ----
__global__ void k_score_keys(int n, const void* score, int dtype, unsigned long long* key, int32_t* val) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        unsigned long long k;
        // -0.0 is keyed as +0.0 so that the two tie like any equal scores
        if (dtype == 0) {
            const double x = static_cast<const double*>(score)[i];
            const unsigned long long b = x == 0.0 ? 0ull : static_cast<unsigned long long>(__double_as_longlong(x));
            const unsigned long long ord = (b >> 63) ? ~b : (b | 0x8000000000000000ull);   // ascending in the value
            k = ~ord;                                                                      // descending
        } else {
            const float x = static_cast<const float*>(score)[i];
            const unsigned b = x == 0.f ? 0u : __float_as_uint(x);
            const unsigned ord = (b >> 31) ? ~b : (b | 0x80000000u);
            k = static_cast<unsigned long long>(~ord);
        }
        key[i] = k;
        val[i] = static_cast<int32_t>(i);
    }
}

__global__ void k_take_ids(int k, const int32_t* __restrict__ order, int32_t* ids) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < k;
         i += static_cast<long long>(gridDim.x) * blockDim.x)
        ids[i] = order[i];
}

// With g = the first sorted position holding key[i] (the number of
// vertices with a strictly larger score): label = log((n+1)/(g+1)) /
// log(n+1), 1 for the best vertex and near 0 for the last; the logarithm
// spreads the top of the ranking, which decides the answer, over most of
// the label range.
__global__ void k_rank_labels(int n, const unsigned long long* __restrict__ key, const int32_t* __restrict__ val,
                              float* label) {
    for (long long ii = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; ii < n;
         ii += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int i = static_cast<int>(ii);
        const unsigned long long k = key[i];
        int lo = 0, hi = i;                       // first j in [0, i] with key[j] == k
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (key[mid] < k) lo = mid + 1;
            else hi = mid;
        }
        const double n1 = static_cast<double>(n) + 1.0;
        label[val[i]] = static_cast<float>(log(n1 / (static_cast<double>(lo) + 1.0)) / log(n1));
    }
}

unsigned grid_for(long long count, int block = 256) {
    return static_cast<unsigned>(std::max<long long>(1, std::min<long long>((count + block - 1) / block, 8192)));
}

// key = value = the id, for sorting a list of ids ascending
__global__ void k_id_keys(int k, const int32_t* __restrict__ ids, unsigned long long* key, int32_t* val) {
    for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < k;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        key[i] = static_cast<unsigned long long>(static_cast<uint32_t>(ids[i]));
        val[i] = ids[i];
    }
}

size_t topk_ws(int32_t n) {
    if (n < 1) return 0;
    return hln::Arena::round(static_cast<size_t>(n) * 8) + hln::Arena::round(static_cast<size_t>(n) * 4) +
           hln::prim::sort_workspace(n);
}

// keys that sort ascending in (score descending, index ascending), sorted
// with their indices
hln_status sort_scores(int32_t n, const void* score, int32_t dtype, void* workspace, size_t workspace_bytes,
                       hipStream_t st, unsigned long long** key_out, int32_t** val_out) {
    using hln::fail;
    if (n < 1 || !score) return fail(HLN_EINVAL, "bad arguments");
    if (dtype != 0 && dtype != 1) return fail(HLN_EINVAL, "dtype must be 0 (f64) or 1 (f32)");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % hln::Arena::kAlign)
        return fail(HLN_EINVAL, "workspace NULL or not 256-byte aligned");
    const size_t need = topk_ws(n);
    if (workspace_bytes < need) return fail(HLN_ENOMEM, "workspace too small: %zu < %zu", workspace_bytes, need);
    hln::Arena ar{static_cast<char*>(workspace), workspace_bytes};
    unsigned long long* key = ar.take<unsigned long long>(n);
    int32_t* val = ar.take<int32_t>(n);
    hipLaunchKernelGGL(k_score_keys, dim3(grid_for(n)), dim3(256), 0, st, n, score, dtype, key, val);
    HLN_TRY_HIP(hipGetLastError());
    const hln_status s =
        hln::prim::sort_pairs(key, val, n, dtype == 0 ? 64 : 32, ar.base + ar.off, workspace_bytes - ar.off, st);
    *key_out = key;
    *val_out = val;
    return s;
}

}  // namespace

extern "C" {

int32_t hln_mlp_param_count(void) { return NPARAM; }

hln_status hln_proposer_features(int32_t n, int32_t r, const int32_t* const* row_ptr, const int64_t* const* S,
                                 const int32_t* const* R, const int32_t* const* h2, const int64_t* nnz, float* X,
                                 void* stream) {
    using hln::fail;
    hln::clear_error();
    if (n < 1 || r < 1 || r > kMaxLayers) return fail(HLN_EINVAL, "bad n or r");
    if (!row_ptr || !S || !R || !h2 || !nnz || !X) return fail(HLN_EINVAL, "NULL argument");
    Layers L;
    L.r = r;
    for (int l = 0; l < r; ++l) {
        if (!row_ptr[l] || !S[l] || !R[l] || !h2[l]) return fail(HLN_EINVAL, "layer %d: NULL array", l);
        L.rp[l] = row_ptr[l];
        L.S[l] = S[l];
        L.R[l] = R[l];
        L.h2[l] = h2[l];
        const double mean_deg = static_cast<double>(nnz[l]) / static_cast<double>(n);
        L.inv_mean_deg[l] = mean_deg > 0 ? static_cast<float>(1.0 / mean_deg) : 0.f;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_features, dim3(grid_for(n)), dim3(256), 0, st, n, L, X);
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

hln_status hln_mlp_init(float* params, float* adam_m, float* adam_v, uint64_t seed, void* stream) {
    hln::clear_error();
    if (!params) return hln::fail(HLN_EINVAL, "params is NULL");
    hipLaunchKernelGGL(k_mlp_init, dim3((NPARAM + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), params,
                       adam_m, adam_v, static_cast<unsigned long long>(seed));
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

hln_status hln_mlp_forward(const float* params, const float* X, int32_t n, float* y, void* stream) {
    hln::clear_error();
    if (!params || !X || !y || n < 0) return hln::fail(HLN_EINVAL, "bad arguments");
    if (n == 0) return HLN_OK;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(grid_for(n, BLK)), dim3(BLK), 0, static_cast<hipStream_t>(stream), params, X,
                       n, y);
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

size_t hln_mlp_train_workspace_size(int32_t n) {
    if (n < 1) return 0;
    const size_t blocks = (static_cast<size_t>(n) + TB - 1) / TB;
    return hln::Arena::round(blocks * NPARAM * 4) + hln::Arena::round(blocks * 4 + 4);
}

hln_status hln_mlp_train_step(float* params, float* adam_m, float* adam_v, int32_t step, float lr, const float* X,
                              const float* target, int32_t n, float* loss, void* workspace, size_t workspace_bytes,
                              void* stream) {
    using hln::fail;
    hln::clear_error();
    if (!params || !adam_m || !adam_v || !X || !target || n < 1 || step < 1) return fail(HLN_EINVAL, "bad arguments");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % hln::Arena::kAlign)
        return fail(HLN_EINVAL, "workspace NULL or not 256-byte aligned");
    const size_t need = hln_mlp_train_workspace_size(n);
    if (workspace_bytes < need) return fail(HLN_ENOMEM, "workspace too small: %zu < %zu", workspace_bytes, need);
    const int blocks = (n + TB - 1) / TB;
    hln::Arena ar{static_cast<char*>(workspace), workspace_bytes};
    float* part = ar.take<float>(static_cast<size_t>(blocks) * NPARAM);
    float* lpart = ar.take<float>(blocks + 1);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(BLK), 0, st, params, X, target, n, 1.0f / static_cast<float>(n),
                       part, lpart);
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, params, adam_m, adam_v, part, blocks,
                       step, lr, 0.9f, 0.999f, 1e-8f, lpart, loss);
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

size_t hln_topk_workspace_size(int32_t n) { return topk_ws(n); }

hln_status hln_topk(int32_t n, const void* score, int32_t dtype, int32_t k, int32_t* ids, void* workspace,
                    size_t workspace_bytes, void* stream) {
    hln::clear_error();
    if (k < 0 || k > n) return hln::fail(HLN_EINVAL, "k must be in [0, n]");
    if (!ids) return hln::fail(HLN_EINVAL, "ids is NULL");
    const bool as_set = (dtype & HLN_TOPK_SET) != 0;
    dtype &= ~HLN_TOPK_SET;
    unsigned long long* key;
    int32_t* val;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hln_status s = sort_scores(n, score, dtype, workspace, workspace_bytes, st, &key, &val);
    if (s != HLN_OK) return s;
    if (k > 0) hipLaunchKernelGGL(k_take_ids, dim3(grid_for(k)), dim3(256), 0, st, k, val, ids);
    if (as_set && k > 1) {
        // the same k ids in ascending order: one more radix sort, of the ids
        // themselves, in the key and value arrays the ranking is done with
        hipLaunchKernelGGL(k_id_keys, dim3(grid_for(k)), dim3(256), 0, st, k, ids, key, val);
        int bits = 1;
        while (bits < 31 && ((n - 1) >> bits) != 0) ++bits;
        hln::Arena ar{static_cast<char*>(workspace), workspace_bytes};
        (void)ar.take<unsigned long long>(n);
        (void)ar.take<int32_t>(n);
        s = hln::prim::sort_pairs(key, val, k, bits, ar.base + ar.off, workspace_bytes - ar.off, st);
        if (s != HLN_OK) return s;
        hipLaunchKernelGGL(k_take_ids, dim3(grid_for(k)), dim3(256), 0, st, k, val, ids);
    }
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

hln_status hln_rank_labels(int32_t n, const void* score, int32_t dtype, float* label, void* workspace,
                           size_t workspace_bytes, void* stream) {
    hln::clear_error();
    if (!label) return hln::fail(HLN_EINVAL, "label is NULL");
    unsigned long long* key;
    int32_t* val;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const hln_status s = sort_scores(n, score, dtype, workspace, workspace_bytes, st, &key, &val);
    if (s != HLN_OK) return s;
    hipLaunchKernelGGL(k_rank_labels, dim3(grid_for(n)), dim3(256), 0, st, n, key, val, label);
    HLN_TRY_HIP(hipGetLastError());
    return HLN_OK;
}

}  // extern "C"
