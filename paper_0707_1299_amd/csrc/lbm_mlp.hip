// Mobility-correction network: 4 -> 64 tanh -> 64 tanh -> 1 (linear output).
// Weights are held as bfloat16 for the forward pass and as FP32 master
// copies for training; every product accumulates in FP32.
//
// Parameter layout (flat, LBML_NPARAM = 4545):
//   W1[64][4] b1[64] W2[64][64] b2[64] W3[1][64] b3[1]
//
// Training is full-batch mean-squared error.  The gradient pass first stores,
// per sample, the activations and the back-propagated pre-activation
// gradients, then forms each parameter's gradient as a sum over samples in
// sample order (one thread per parameter and fixed chunking), so repeated
// calls give bit-identical gradients.
#include <math.h>

#include <mutex>

#include "../../include/lbm.h"
#include "lbm_device.h"

namespace {

constexpr int NP = 4545;
constexpr int O_W1 = 0, O_B1 = 256, O_W2 = 320, O_B2 = 4416, O_W3 = 4480, O_B3 = 4544;

__device__ __forceinline__ float bf16f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// round to nearest, ties to even
__device__ __forceinline__ uint16_t f2bf16(float x)
{
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7F800000u) == 0x7F800000u) return uint16_t((b >> 16) | ((b & 0xFFFFu) ? 0x40u : 0u));
    b += 0x7FFFu + ((b >> 16) & 1u);
    return uint16_t(b >> 16);
}

__global__ void k_round(const float* __restrict__ m, uint16_t* __restrict__ w, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = f2bf16(m[i]);
}

__device__ __forceinline__ void stage(const uint16_t* __restrict__ w16, float* W)
{
    for (int k = threadIdx.x; k < NP; k += blockDim.x) W[k] = bf16f(w16[k]);
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_forward(const uint16_t* __restrict__ w16, long long n,
                                                 const float* __restrict__ x, float* __restrict__ y)
{
    __shared__ float W[NP];
    stage(w16, W);
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float xin[4] = {x[4 * i], x[4 * i + 1], x[4 * i + 2], x[4 * i + 3]};
    float h1[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        float s = W[O_B1 + j];
#pragma unroll
        for (int k = 0; k < 4; ++k) s = fmaf(W[O_W1 + 4 * j + k], xin[k], s);
        h1[j] = tanhf(s);
    }
    float out = W[O_B3];
    for (int j = 0; j < 64; ++j) {
        float s = W[O_B2 + j];
#pragma unroll
        for (int k = 0; k < 64; ++k) s = fmaf(W[O_W2 + 64 * j + k], h1[k], s);
        out = fmaf(W[O_W3 + j], tanhf(s), out);
    }
    y[i] = out;
}

// per sample: h1, h2, dz1, dz2 (64 each) and dy into work
//   work layout: h1[n][64] h2[n][64] dz1[n][64] dz2[n][64] dy[n] sq[n]
__global__ __launch_bounds__(256) void k_backprop(const uint16_t* __restrict__ w16, long long n,
                                                  const float* __restrict__ x, const float* __restrict__ target,
                                                  float* __restrict__ work)
{
    __shared__ float W[NP];
    stage(w16, W);
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float* H1 = work;
    float* H2 = H1 + 64 * n;
    float* D1 = H2 + 64 * n;
    float* D2 = D1 + 64 * n;
    float* DY = D2 + 64 * n;
    float* SQ = DY + n;
    float xin[4] = {x[4 * i], x[4 * i + 1], x[4 * i + 2], x[4 * i + 3]};
    float h1[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        float s = W[O_B1 + j];
#pragma unroll
        for (int k = 0; k < 4; ++k) s = fmaf(W[O_W1 + 4 * j + k], xin[k], s);
        h1[j] = tanhf(s);
        H1[64 * i + j] = h1[j];
    }
    float out = W[O_B3];
    for (int j = 0; j < 64; ++j) {
        float s = W[O_B2 + j];
#pragma unroll
        for (int k = 0; k < 64; ++k) s = fmaf(W[O_W2 + 64 * j + k], h1[k], s);
        const float h = tanhf(s);
        H2[64 * i + j] = h;
        out = fmaf(W[O_W3 + j], h, out);
    }
    const float r = out - target[i];
    const float dy = 2.0f * r / float(n);
    DY[i] = dy;
    SQ[i] = r * r;
    // dz2_j = dy W3_j (1 - h2_j^2); dz1_k = (sum_j dz2_j W2_jk)(1 - h1_k^2)
    float d1[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) d1[k] = 0.0f;
    for (int j = 0; j < 64; ++j) {
        const float h = H2[64 * i + j];
        const float d2 = dy * W[O_W3 + j] * (1.0f - h * h);
        D2[64 * i + j] = d2;
#pragma unroll
        for (int k = 0; k < 64; ++k) d1[k] = fmaf(d2, W[O_W2 + 64 * j + k], d1[k]);
    }
#pragma unroll
    for (int k = 0; k < 64; ++k) D1[64 * i + k] = d1[k] * (1.0f - h1[k] * h1[k]);
}

// one thread per parameter: sum over samples in order
__global__ __launch_bounds__(256) void k_grad(long long n, const float* __restrict__ x, const float* __restrict__ work,
                                              float* __restrict__ grad, float* __restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const float* H1 = work;
    const float* H2 = H1 + 64 * n;
    const float* D1 = H2 + 64 * n;
    const float* D2 = D1 + 64 * n;
    const float* DY = D2 + 64 * n;
    const float* SQ = DY + n;
    if (p == NP) {
        float s = 0.0f;
        for (long long i = 0; i < n; ++i) s += SQ[i];
        *loss = s / float(n);
        return;
    }
    if (p > NP) return;
    float s = 0.0f;
    if (p < O_B1) {
        const int j = p / 4, k = p % 4;
        for (long long i = 0; i < n; ++i) s = fmaf(D1[64 * i + j], x[4 * i + k], s);
    } else if (p < O_W2) {
        const int j = p - O_B1;
        for (long long i = 0; i < n; ++i) s += D1[64 * i + j];
    } else if (p < O_B2) {
        const int j = (p - O_W2) / 64, k = (p - O_W2) % 64;
        for (long long i = 0; i < n; ++i) s = fmaf(D2[64 * i + j], H1[64 * i + k], s);
    } else if (p < O_W3) {
        const int j = p - O_B2;
        for (long long i = 0; i < n; ++i) s += D2[64 * i + j];
    } else if (p < O_B3) {
        const int j = p - O_W3;
        for (long long i = 0; i < n; ++i) s = fmaf(DY[i], H2[64 * i + j], s);
    } else {
        for (long long i = 0; i < n; ++i) s += DY[i];
    }
    grad[p] = s;
}

__global__ void k_adam(float* __restrict__ m0, float* __restrict__ m1, float* __restrict__ v1,
                       const float* __restrict__ g, uint16_t* __restrict__ w16, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NP) return;
    const float gi = g[i];
    const float m = b1 * m1[i] + (1.0f - b1) * gi;
    const float v = b2 * v1[i] + (1.0f - b2) * gi * gi;
    m1[i] = m;
    v1[i] = v;
    const float mh = m / c1, vh = v / c2;
    const float w = m0[i] - lr * mh / (sqrtf(vh) + eps);
    m0[i] = w;
    w16[i] = f2bf16(w);
}

// the two passes of the gradient: per-sample quantities into work, then the per-parameter sums
void launch_loss_grad(const uint16_t* d_w16, long long n, const float* d_x, const float* d_target, float* d_grad,
                      float* d_loss, float* d_work, hipStream_t s)
{
    hipLaunchKernelGGL(k_backprop, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_w16, n, d_x, d_target,
                       d_work);
    hipLaunchKernelGGL(k_grad, dim3((NP + 1 + 255) / 256), dim3(256), 0, s, n, d_x, (const float*)d_work, d_grad,
                       d_loss);
}

}  // namespace

// Work memory of lbml_loss_grad_static: a device array in the library itself, sized for
// LBML_STATIC_MAX_N samples (lbml_work_floats of that many).  Its name is a host-side stand-in:
// kernels receive the device address that hipGetSymbolAddress returns, taken once per device
// (with that device current) and kept in scratch_dev.  Every call on one device shares the array;
// the gradient pass writes every value it reads, so nothing needs clearing between calls.
static __device__ __align__(256) float scratch[258LL * LBML_STATIC_MAX_N];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
float* scratch_dev[MAX_DEVICES] = {};

int scratch_ptr(float** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return LB_ERR_HIP;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return LB_ERR_HIP;
        scratch_dev[dev] = static_cast<float*>(p);
    }
    *out = scratch_dev[dev];
    return LB_OK;
}

}  // namespace

extern "C" {

int64_t lbml_work_floats(int64_t n) { return n < 0 ? -1 : 256 * n + 2 * n; }

int lbml_round_bf16(const float* d_master, uint16_t* d_w16, void* hip_stream)
{
    if (!d_master || !d_w16) return LB_ERR_ARG;
    hipLaunchKernelGGL(k_round, dim3((NP + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream, d_master, d_w16, NP);
    return hipGetLastError() == hipSuccess ? LB_OK : LB_ERR_HIP;
}

int lbml_forward(const uint16_t* d_w16, int64_t n, const float* d_x, float* d_y, void* hip_stream)
{
    if (n < 0 || (n > 0 && (!d_w16 || !d_x || !d_y))) return LB_ERR_ARG;
    if (n == 0) return LB_OK;
    hipLaunchKernelGGL(k_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)hip_stream, d_w16,
                       (long long)n, d_x, d_y);
    return hipGetLastError() == hipSuccess ? LB_OK : LB_ERR_HIP;
}

int lbml_loss_grad(const uint16_t* d_w16, int64_t n, const float* d_x, const float* d_target, float* d_grad,
                   float* d_loss, float* d_work, void* hip_stream)
{
    if (n <= 0 || !d_w16 || !d_x || !d_target || !d_grad || !d_loss || !d_work) return LB_ERR_ARG;
    (void)hipGetLastError();
    launch_loss_grad(d_w16, (long long)n, d_x, d_target, d_grad, d_loss, d_work, (hipStream_t)hip_stream);
    return hipGetLastError() == hipSuccess ? LB_OK : LB_ERR_HIP;
}

int lbml_loss_grad_static(const uint16_t* d_w16, int64_t n, const float* d_x, const float* d_target, float* d_grad,
                          float* d_loss, void* hip_stream)
{
    if (n <= 0 || !d_w16 || !d_x || !d_target || !d_grad || !d_loss) return LB_ERR_ARG;
    if (n > LBML_STATIC_MAX_N) return LB_ERR_SIZE;
    float* work = nullptr;
    const int r = scratch_ptr(&work);
    if (r) return r;
    (void)hipGetLastError();
    launch_loss_grad(d_w16, (long long)n, d_x, d_target, d_grad, d_loss, work, (hipStream_t)hip_stream);
    return hipGetLastError() == hipSuccess ? LB_OK : LB_ERR_HIP;
}

int lbml_adam_step(float* d_master, float* d_m, float* d_v, const float* d_grad, uint16_t* d_w16, int32_t t, float lr,
                   float beta1, float beta2, float eps, void* hip_stream)
{
    if (!d_master || !d_m || !d_v || !d_grad || !d_w16 || t < 1) return LB_ERR_ARG;
    const float c1 = 1.0f - powf(beta1, (float)t);
    const float c2 = 1.0f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream, d_master, d_m, d_v,
                       d_grad, d_w16, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? LB_OK : LB_ERR_HIP;
}

}  // extern "C"
