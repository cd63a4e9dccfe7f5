// Cost-model network on the GPU: forward, backward and Adam, in FP32.
//
//   h1 = relu(W1 x + b1)   (64 x 32)      x: 32 chunk statistics
//   h2 = relu(W2 h1 + b2)  (64 x 64)
//   y  = W3 h2 + b3        (24 x 64)      y: predicted log time per (codec, schedule)
//
// Loss over n samples: (1/n) sum_i (y_i[k_i] - t_i)^2, only the measured
// output k_i of each sample counts.  One workgroup of 256 threads handles 64
// samples with every weight and activation in LDS; the per-workgroup partial
// gradients are summed over workgroups in a fixed order, so a training run is
// bit-reproducible.  The tensors are tiny: this is plain FP32 FMA work, not a
// matrix-core job.
#include <hip/hip_runtime.h>

#include <cstdint>

#include <mutex>
#include <string>

#include "zf.h"

namespace zf {
void set_last_error(const std::string &m);

static zf_status fail_with(zf_status st, const char *msg) {
    set_last_error(msg);
    return st;
}
static zf_status launched() {
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return ZF_OK;
    set_last_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
    return ZF_E_HIP;
}

constexpr int NI = 32, NH = 64, NO = 24, TS = 64;  // inputs, hidden, outputs, samples per block
constexpr int OW1 = 0, OB1 = OW1 + NH * NI, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NO * NH, NP = OB3 + NO;
static_assert(NP == 7832, "parameter count");

struct MlpShared {
    float p[NP];
    float x[TS][NI];
    float h1[TS][NH];
    float h2[TS][NH];   // later reused for dL/dz1
    float d2[TS][NH];   // dL/dz2 (masked by relu')
    float e[TS];        // y[k] - t per sample (NaN for an out-of-range k)
    int k[TS];
};

// Forward pass of the block's samples; leaves h1, h2 in LDS and returns
// nothing; y values are written by the callers as they need them.
__device__ void mlp_forward_block(MlpShared &S, const float *P, const float *X, uint32_t n,
                                  uint32_t s0) {
    const int t = threadIdx.x;
    for (int i = t; i < NP; i += 256) S.p[i] = P[i];
    for (int i = t; i < TS * NI; i += 256) {
        const uint32_t s = s0 + uint32_t(i / NI);
        S.x[i / NI][i % NI] = s < n ? X[uint64_t(s) * NI + (i % NI)] : 0.f;
    }
    __syncthreads();
    const int j = t % NH, r0 = t / NH;  // neuron j, samples r0, r0+4, ...
    for (int s = r0; s < TS; s += 4) {
        float a = S.p[OB1 + j];
        for (int i = 0; i < NI; i++) a = fmaf(S.p[OW1 + j * NI + i], S.x[s][i], a);
        S.h1[s][j] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    for (int s = r0; s < TS; s += 4) {
        float a = S.p[OB2 + j];
        for (int i = 0; i < NH; i++) a = fmaf(S.p[OW2 + j * NH + i], S.h1[s][i], a);
        S.h2[s][j] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
}

__device__ float mlp_out(const MlpShared &S, int s, int o) {
    float a = S.p[OB3 + o];
    for (int i = 0; i < NH; i++) a = fmaf(S.p[OW3 + o * NH + i], S.h2[s][i], a);
    return a;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float *P, const float *X, uint32_t n,
                                                     float *Y) {
    __shared__ MlpShared S;
    const uint32_t s0 = blockIdx.x * TS;
    mlp_forward_block(S, P, X, n, s0);
    for (int i = threadIdx.x; i < TS * NO; i += 256) {
        const int s = i / NO, o = i % NO;
        if (s0 + s < n) Y[uint64_t(s0 + s) * NO + o] = mlp_out(S, s, o);
    }
}

// Partial gradient of the block's samples -> work[block][NP + 1] (last = loss).
__global__ __launch_bounds__(256) void k_mlp_grad(const float *P, const float *X, const int32_t *K,
                                                  const float *T, uint32_t n, float *work) {
    __shared__ MlpShared S;
    const uint32_t s0 = blockIdx.x * TS;
    const int t = threadIdx.x;
    mlp_forward_block(S, P, X, n, s0);
    const float inv_n = 1.f / float(n);
    float(&d1)[TS][NH] = S.h2;  // h2 is dead once dz2 and dW3 are done
    if (t < TS) {
        const uint32_t s = s0 + t;
        float e = 0.f;
        int k = -1;
        if (s < n) {
            k = K[s];
            e = (k >= 0 && k < NO) ? mlp_out(S, t, k) - T[s] : __builtin_nanf("");
        }
        S.e[t] = e;
        S.k[t] = (k >= 0 && k < NO) ? k : -1;
    }
    __syncthreads();
    float *g = work + uint64_t(blockIdx.x) * (NP + 1);
    if (t == 0) {
        float l = 0.f;
        for (int s = 0; s < TS; s++)
            if (s0 + s < n) l = fmaf(S.e[s] * inv_n, S.e[s], l);
        g[NP] = l;
    }
    // layer 3: dW3[o][j] = sum_s [k_s == o] dy_s h2[s][j]; db3[o] = sum_s [k_s == o] dy_s
    for (int i = t; i < NO * NH; i += 256) {
        const int o = i / NH, jj = i % NH;
        float a = 0.f;
        for (int s = 0; s < TS; s++)
            if (S.k[s] == o) a = fmaf(2.f * S.e[s] * inv_n, S.h2[s][jj], a);
        g[OW3 + i] = a;
    }
    if (t < NO) {
        float a = 0.f;
        for (int s = 0; s < TS; s++)
            if (S.k[s] == t) a += 2.f * S.e[s] * inv_n;
        g[OB3 + t] = a;
    }
    // dz2[s][j] = dy_s W3[k_s][j] relu'(z2)
    for (int i = t; i < TS * NH; i += 256) {
        const int s = i / NH, jj = i % NH;
        const int k = S.k[s];
        S.d2[s][jj] = (k >= 0 && S.h2[s][jj] > 0.f) ? 2.f * S.e[s] * inv_n * S.p[OW3 + k * NH + jj] : 0.f;
    }
    __syncthreads();  // h2 is no longer read after this point
    // layer 2: dW2[j][i] = sum_s dz2[s][j] h1[s][i]; db2[j] = sum_s dz2[s][j]
    for (int q = t; q < NH * NH; q += 256) {
        const int jj = q / NH, i = q % NH;
        float a = 0.f;
        for (int s = 0; s < TS; s++) a = fmaf(S.d2[s][jj], S.h1[s][i], a);
        g[OW2 + q] = a;
    }
    if (t < NH) {
        float a = 0.f;
        for (int s = 0; s < TS; s++) a += S.d2[s][t];
        g[OB2 + t] = a;
    }
    // dz1[s][i] = (sum_j dz2[s][j] W2[j][i]) relu'(z1)
    for (int q = t; q < TS * NH; q += 256) {
        const int s = q / NH, i = q % NH;
        float a = 0.f;
        for (int jj = 0; jj < NH; jj++) a = fmaf(S.d2[s][jj], S.p[OW2 + jj * NH + i], a);
        d1[s][i] = S.h1[s][i] > 0.f ? a : 0.f;
    }
    __syncthreads();
    // layer 1: dW1[i][c] = sum_s dz1[s][i] x[s][c]; db1[i] = sum_s dz1[s][i]
    for (int q = t; q < NH * NI; q += 256) {
        const int i = q / NI, c = q % NI;
        float a = 0.f;
        for (int s = 0; s < TS; s++) a = fmaf(d1[s][i], S.x[s][c], a);
        g[OW1 + q] = a;
    }
    if (t < NH) {
        float a = 0.f;
        for (int s = 0; s < TS; s++) a += d1[s][t];
        g[OB1 + t] = a;
    }
}

// grad[p] = sum over blocks of the partials, in block order.
__global__ void k_mlp_reduce(const float *work, uint32_t nblocks, float *grad, float *loss) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > uint32_t(NP)) return;
    float a = 0.f;
    for (uint32_t b = 0; b < nblocks; b++) a += work[uint64_t(b) * (NP + 1) + p];
    if (p < uint32_t(NP)) grad[p] = a;
    else *loss = a;
}

__global__ void k_mlp_adam(float *P, const float *G, float *M, float *V, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= uint32_t(NP)) return;
    const float g = G[p];
    const float m = b1 * M[p] + (1.f - b1) * g;
    const float v = b2 * V[p] + (1.f - b2) * g * g;
    M[p] = m;
    V[p] = v;
    P[p] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

// Allocation-free gradient (zf_mlp_grad_noalloc): the per-workgroup partials
// live in this file-scope device array instead of a caller workspace.  Every
// partial a launch reads is written by the same launch first, so nothing has
// to be cleared between calls.  In host code `scratch` only names the symbol;
// its device address comes from hipGetSymbolAddress, once per device.
constexpr uint32_t kStaticBlocks = (ZF_MLP_STATIC_MAX_N + TS - 1) / TS;
static __device__ __align__(256) float scratch[uint64_t(kStaticBlocks) * (NP + 1)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call per device).
static zf_status static_scratch(float **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_with(ZF_E_HIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return fail_with(ZF_E_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_last_error(std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
            return ZF_E_HIP;
        }
        g_scratch_ptr[dev] = static_cast<float *>(p);
    }
    *out = g_scratch_ptr[dev];
    return ZF_OK;
}

}  // namespace zf

using namespace zf;

extern "C" {

zf_status zf_mlp_forward(const float *d_params, const float *d_x, uint32_t n, float *d_y,
                         zf_stream_t stream) {
    if (!n) return ZF_OK;
    if (!d_params || !d_x || !d_y) return fail_with(ZF_E_INVALID, "null pointer");
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + TS - 1) / TS), dim3(256), 0,
                       static_cast<hipStream_t>(stream), d_params, d_x, n, d_y);
    return launched();
}

uint64_t zf_mlp_grad_work_bytes(uint32_t n) {
    return uint64_t((n + TS - 1) / TS) * (NP + 1) * sizeof(float);
}

zf_status zf_mlp_grad(const float *d_params, const float *d_x, const int32_t *d_k, const float *d_t,
                      uint32_t n, float *d_grad, float *d_loss, void *d_work, uint64_t work_bytes,
                      zf_stream_t stream) {
    if (!n || !d_params || !d_x || !d_k || !d_t || !d_grad || !d_loss || !d_work)
        return fail_with(ZF_E_INVALID, "null pointer or empty batch");
    if (work_bytes < zf_mlp_grad_work_bytes(n)) return fail_with(ZF_E_TOO_SMALL, "workspace too small");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t nb = (n + TS - 1) / TS;
    float *work = static_cast<float *>(d_work);
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, st, d_params, d_x, d_k, d_t, n, work);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NP + 1 + 255) / 256), dim3(256), 0, st, work, nb, d_grad,
                       d_loss);
    return launched();
}

zf_status zf_mlp_grad_noalloc(const float *d_params, const float *d_x, const int32_t *d_k,
                              const float *d_t, uint32_t n, float *d_grad, float *d_loss,
                              zf_stream_t stream) {
    if (!n || !d_params || !d_x || !d_k || !d_t || !d_grad || !d_loss)
        return fail_with(ZF_E_INVALID, "null pointer or empty batch");
    if (n > ZF_MLP_STATIC_MAX_N) {
        set_last_error("zf_mlp_grad_noalloc: " + std::to_string(n) + " samples exceed the static scratch "
                       "limit of " + std::to_string(ZF_MLP_STATIC_MAX_N) + " (use zf_mlp_grad with a workspace)");
        return ZF_E_UNSUPPORTED;
    }
    float *work = nullptr;
    const zf_status st0 = static_scratch(&work);
    if (st0 != ZF_OK) return st0;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t nb = (n + TS - 1) / TS;
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, st, d_params, d_x, d_k, d_t, n, work);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NP + 1 + 255) / 256), dim3(256), 0, st, work, nb, d_grad,
                       d_loss);
    return launched();
}

zf_status zf_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, uint32_t step,
                      float lr, float beta1, float beta2, float eps, zf_stream_t stream) {
    if (!d_params || !d_grad || !d_m || !d_v || step == 0)
        return fail_with(ZF_E_INVALID, "null pointer or step 0");
    const double c1 = 1.0 / (1.0 - __builtin_pow(double(beta1), double(step)));
    const double c2 = 1.0 / (1.0 - __builtin_pow(double(beta2), double(step)));
    hipLaunchKernelGGL(k_mlp_adam, dim3((NP + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), d_params, d_grad, d_m, d_v, lr, beta1, beta2,
                       eps, float(c1), float(c2));
    return launched();
}

}  // extern "C"
