// Candidate-ranking MLP: 3 features -> 64 -> 64 -> 1 (ReLU), weights held
// in bf16 for the forward pass, FP32 accumulation, FP32 master weights and
// Adam moments for training.  Used to order the candidate list of each
// edge before a level's lexicographic enumeration (the order changes only
// which separating set is found first and how many tests run before it;
// the stable schedule makes the skeleton independent of it).
//
// Model buffer (device, fpc_mlp_bytes() bytes, 256-byte aligned parts):
//   float  master[kParams]     W1[3][64], b1[64], W2[64][64], b2[64], W3[64], b3
//   float  adam_m[kParams], adam_v[kParams]
//   bf16   W1h[3*64], W2h[64*64], W3h[64]   (rounded copies used by the passes)
//   int    step
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "fpc_internal.h"

namespace fpc {

namespace {

constexpr int kIn = 3, kH = 64;
constexpr int oW1 = 0, ob1 = oW1 + kIn * kH, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH, ob3 = oW3 + kH;
constexpr int kParams = ob3 + 1;  // 4481

inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t kMasterBytes = ((size_t)kParams * 4 + 255) / 256 * 256;
constexpr size_t kOffM = kMasterBytes, kOffV = 2 * kMasterBytes, kOffH = 3 * kMasterBytes;
constexpr size_t kHalfBytes = ((size_t)(kIn * kH + kH * kH + kH) * 2 + 255) / 256 * 256;
constexpr size_t kOffStep = kOffH + kHalfBytes;
constexpr size_t kModelBytes = kOffStep + 256;

struct ModelView {
    float *master, *m, *v;
    __bf16 *W1h, *W2h, *W3h;
    int *step;
};

inline ModelView view(void *model)
{
    char *b = static_cast<char *>(model);
    ModelView mv;
    mv.master = reinterpret_cast<float *>(b);
    mv.m = reinterpret_cast<float *>(b + kOffM);
    mv.v = reinterpret_cast<float *>(b + kOffV);
    mv.W1h = reinterpret_cast<__bf16 *>(b + kOffH);
    mv.W2h = mv.W1h + kIn * kH;
    mv.W3h = mv.W2h + kH * kH;
    mv.step = reinterpret_cast<int *>(b + kOffStep);
    return mv;
}

// bf16 copies of the weight matrices from the FP32 master weights
__global__ void round_weights(const float *__restrict__ master, __bf16 *__restrict__ W1h, __bf16 *__restrict__ W2h,
                              __bf16 *__restrict__ W3h)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < kIn * kH) W1h[t] = (__bf16)master[oW1 + t];
    if (t < kH * kH) W2h[t] = (__bf16)master[oW2 + t];
    if (t < kH) W3h[t] = (__bf16)master[oW3 + t];
}

// Weights staged in LDS as FP32 values of the bf16 copies.
struct SmemW {
    alignas(16) float W2[kH * kH];  // first, 16-byte aligned: read as float4 rows
    float W1[kIn * kH], b1[kH], b2[kH], W3[kH], b3;
};

__device__ void load_weights(SmemW &s, const float *__restrict__ master, const __bf16 *__restrict__ W1h,
                             const __bf16 *__restrict__ W2h, const __bf16 *__restrict__ W3h)
{
    for (int t = threadIdx.x; t < kH * kH; t += blockDim.x) s.W2[t] = (float)W2h[t];
    for (int t = threadIdx.x; t < kIn * kH; t += blockDim.x) s.W1[t] = (float)W1h[t];
    for (int t = threadIdx.x; t < kH; t += blockDim.x) {
        s.b1[t] = master[ob1 + t];
        s.b2[t] = master[ob2 + t];
        s.W3[t] = (float)W3h[t];
    }
    if (threadIdx.x == 0) s.b3 = master[ob3];
    __syncthreads();
}

// h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), z = h2 . W3 + b3
__device__ __forceinline__ float forward_one(const SmemW &s, const float *x, float *h1, float *h2)
{
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        float a = s.b1[o];
#pragma unroll
        for (int i = 0; i < kIn; ++i) a = fmaf(x[i], s.W1[i * kH + o], a);
        h1[o] = fmaxf(a, 0.f);
    }
    float z = s.b3;
#pragma unroll 4
    for (int o = 0; o < kH; ++o) {
        float a = s.b2[o];
#pragma unroll
        for (int i = 0; i < kH; ++i) a = fmaf(h1[i], s.W2[i * kH + o], a);
        h2[o] = fmaxf(a, 0.f);
        z = fmaf(h2[o], s.W3[o], z);
    }
    return z;
}

// The same forward pass with the hidden layer's loops swapped: all 64
// sums of layer 2 stay in registers and each row of W2 is read from LDS as
// 16-byte words (four FMAs per read instead of one).  Every sum takes its
// terms in the same order as forward_one, so the results are identical.
__device__ __forceinline__ float forward_rows(const SmemW &s, const float *x)
{
    float h1[kH];
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        float a = s.b1[o];
#pragma unroll
        for (int i = 0; i < kIn; ++i) a = fmaf(x[i], s.W1[i * kH + o], a);
        h1[o] = fmaxf(a, 0.f);
    }
    // layer 2 in four slices of 16 outputs; the output sum takes them in order
    float z = s.b3;
#pragma unroll 1
    for (int q = 0; q < kH / 16; ++q) {
        float acc[16];
#pragma unroll
        for (int o = 0; o < 16; ++o) acc[o] = s.b2[16 * q + o];
#pragma unroll
        for (int i = 0; i < kH; ++i) {
            const float4 *w = reinterpret_cast<const float4 *>(s.W2 + i * kH + 16 * q);
#pragma unroll
            for (int o4 = 0; o4 < 4; ++o4) {
                const float4 v = w[o4];
                acc[4 * o4 + 0] = fmaf(h1[i], v.x, acc[4 * o4 + 0]);
                acc[4 * o4 + 1] = fmaf(h1[i], v.y, acc[4 * o4 + 1]);
                acc[4 * o4 + 2] = fmaf(h1[i], v.z, acc[4 * o4 + 2]);
                acc[4 * o4 + 3] = fmaf(h1[i], v.w, acc[4 * o4 + 3]);
            }
            // keeps the scheduler from hoisting later rows' reads past this row
            if (i % 4 == 3) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int o = 0; o < 16; ++o) z = fmaf(fmaxf(acc[o], 0.f), s.W3[16 * q + o], z);
    }
    return z;
}

// at most 128 registers (four waves per SIMD): left alone, the compiler
// hoists the unrolled stream of W2 reads into all 256
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void mlp_forward_kernel(
    const float *__restrict__ X, int64_t N,
                                                          const float *__restrict__ master,
                                                          const __bf16 *__restrict__ W1h,
                                                          const __bf16 *__restrict__ W2h,
                                                          const __bf16 *__restrict__ W3h, float *__restrict__ out)
{
    __shared__ SmemW s;
    load_weights(s, master, W1h, W2h, W3h);
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < N; r += (int64_t)gridDim.x * 256) {
        float x[kIn];
#pragma unroll
        for (int i = 0; i < kIn; ++i) x[i] = X[r * kIn + i];
        out[r] = forward_rows(s, x);
    }
}

// Mean binary cross-entropy with logits and its gradient.  Each block
// handles kBS samples and writes its partial loss and gradient to
// part[block]; a second kernel sums the partials in block order.
constexpr int kBS = 32;

__global__ __launch_bounds__(256) void mlp_grad_kernel(const float *__restrict__ X, const float *__restrict__ Y,
                                                       int64_t N, const float *__restrict__ master,
                                                       const __bf16 *__restrict__ W1h,
                                                       const __bf16 *__restrict__ W2h,
                                                       const __bf16 *__restrict__ W3h, float *__restrict__ part)
{
    __shared__ SmemW s;
    __shared__ float H1[kBS][kH + 1], D2[kBS][kH + 1], D1[kBS][kH + 1], XS[kBS][kIn], LS[kBS];
    load_weights(s, master, W1h, W2h, W3h);
    const int64_t r0 = (int64_t)blockIdx.x * kBS;
    const float invN = 1.0f / (float)N;
    // per-sample forward and backward to the hidden layers (threads 0..kBS-1)
    if (threadIdx.x < kBS) {
        const int t = threadIdx.x;
        const int64_t r = r0 + t;
        float x[kIn] = {0.f, 0.f, 0.f}, h1[kH], h2[kH];
        float y = 0.f, w = 0.f;
        if (r < N) {
#pragma unroll
            for (int i = 0; i < kIn; ++i) x[i] = X[r * kIn + i];
            y = Y[r];
            w = invN;
        }
        const float z = forward_one(s, x, h1, h2);
        // loss = log(1 + e^z) - y z ; dz = sigmoid(z) - y
        const float sz = 1.f / (1.f + __expf(-z));
        LS[t] = w * (fmaxf(z, 0.f) + log1pf(__expf(-fabsf(z))) - y * z);
        const float dz = w * (sz - y);
#pragma unroll
        for (int o = 0; o < kH; ++o) {
            H1[t][o] = h1[o];
            D2[t][o] = h2[o] > 0.f ? dz * s.W3[o] : 0.f;  // dL/d(pre-activation of layer 2)
        }
        // keep dz and h2 for the output layer: reuse D1 row as scratch
#pragma unroll
        for (int o = 0; o < kH; ++o) D1[t][o] = dz * h2[o];  // dW3 contribution
        XS[t][0] = x[0];
        XS[t][1] = x[1];
        XS[t][2] = x[2];
        H1[t][kH] = dz;  // db3 contribution
    }
    __syncthreads();
    float *g = part + (size_t)blockIdx.x * (kParams + 1);
    // output layer: dW3[o] = sum_t dz h2, db3 = sum_t dz
    for (int o = threadIdx.x; o < kH; o += blockDim.x) {
        float a = 0.f;
        for (int t = 0; t < kBS; ++t) a += D1[t][o];
        g[oW3 + o] = a;
    }
    if (threadIdx.x == 0) {
        float a = 0.f, l = 0.f;
        for (int t = 0; t < kBS; ++t) {
            a += H1[t][kH];
            l += LS[t];
        }
        g[ob3] = a;
        g[kParams] = l;
    }
    // dW2[i][o] = sum_t h1[t][i] D2[t][o] ; db2[o] = sum_t D2[t][o]
    for (int idx = threadIdx.x; idx < kH * kH; idx += blockDim.x) {
        const int i = idx / kH, o = idx % kH;
        float a = 0.f;
        for (int t = 0; t < kBS; ++t) a = fmaf(H1[t][i], D2[t][o], a);
        g[oW2 + idx] = a;
    }
    for (int o = threadIdx.x; o < kH; o += blockDim.x) {
        float a = 0.f;
        for (int t = 0; t < kBS; ++t) a += D2[t][o];
        g[ob2 + o] = a;
    }
    __syncthreads();
    // D1[t][i] = (sum_o W2[i][o] D2[t][o]) * [h1 > 0]
    for (int idx = threadIdx.x; idx < kBS * kH; idx += blockDim.x) {
        const int t = idx / kH, i = idx % kH;
        float a = 0.f;
        for (int o = 0; o < kH; ++o) a = fmaf(s.W2[i * kH + o], D2[t][o], a);
        D1[t][i] = H1[t][i] > 0.f ? a : 0.f;
    }
    __syncthreads();
    // dW1[i][o] = sum_t x[t][i] D1[t][o] ; db1[o] = sum_t D1[t][o]
    for (int idx = threadIdx.x; idx < kIn * kH; idx += blockDim.x) {
        const int i = idx / kH, o = idx % kH;
        float a = 0.f;
        for (int t = 0; t < kBS; ++t) a = fmaf(XS[t][i], D1[t][o], a);
        g[oW1 + idx] = a;
    }
    for (int o = threadIdx.x; o < kH; o += blockDim.x) {
        float a = 0.f;
        for (int t = 0; t < kBS; ++t) a += D1[t][o];
        g[ob1 + o] = a;
    }
}

__global__ __launch_bounds__(256) void sum_partials(const float *__restrict__ part, int nblk, float *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > kParams) return;
    float a = 0.f;
    for (int b = 0; b < nblk; ++b) a += part[(size_t)b * (kParams + 1) + k];
    out[k] = a;
}

__global__ __launch_bounds__(256) void adam_step(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                                 const float *__restrict__ g, int *__restrict__ step, float lr)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = *step + 1;
    if (k < kParams) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float mk = b1 * m[k] + (1.f - b1) * g[k];
        const float vk = b2 * v[k] + (1.f - b2) * g[k] * g[k];
        m[k] = mk;
        v[k] = vk;
        const float mh = mk / (1.f - powf(b1, (float)t));
        const float vh = vk / (1.f - powf(b2, (float)t));
        w[k] -= lr * mh / (sqrtf(vh) + eps);
    }
}

__global__ void bump_step(int *step) { *step += 1; }

}  // namespace

size_t mlp_model_bytes() { return kModelBytes; }
int mlp_params() { return kParams; }

int mlp_forward(fpc_ctx *ctx, const float *X, int64_t N, const void *model, float *out)
{
    if (N < 0 || !model) return FPC_EINVAL;
    if (N == 0) return FPC_OK;  // empty buffers may be NULL
    if (!X || !out) return FPC_EINVAL;
    ModelView mv = view(const_cast<void *>(model));
    const int64_t grid = std::min<int64_t>((N + 255) / 256, 4 * (int64_t)ctx->num_cus);
    mlp_forward_kernel<<<(unsigned)grid, 256, 0, ctx->stream>>>(X, N, mv.master, mv.W1h, mv.W2h, mv.W3h, out);
    FPC_HIP(hipGetLastError());
    return FPC_OK;
}

int mlp_grad(fpc_ctx *ctx, const float *X, const float *Y, int64_t N, const void *model, float *grad_out)
{
    if (!X || !Y || !model || !grad_out || N <= 0) return FPC_EINVAL;
    ModelView mv = view(const_cast<void *>(model));
    const int64_t nblk = (N + kBS - 1) / kBS;
    if (nblk > 0x7fffffff) return FPC_EINVAL;
    int rc = ctx->batch_tmp.ensure(sizeof(float) * (size_t)nblk * (kParams + 1));
    if (rc) return rc;
    float *part = ctx->batch_tmp.as<float>();
    mlp_grad_kernel<<<(unsigned)nblk, 256, 0, ctx->stream>>>(X, Y, N, mv.master, mv.W1h, mv.W2h, mv.W3h, part);
    sum_partials<<<(kParams + 1 + 255) / 256, 256, 0, ctx->stream>>>(part, (int)nblk, grad_out);
    FPC_HIP(hipGetLastError());
    return FPC_OK;
}

}  // namespace fpc

using namespace fpc;

extern "C" size_t fpc_mlp_bytes(void) { return mlp_model_bytes(); }
extern "C" int fpc_mlp_params(void) { return mlp_params(); }

extern "C" int fpc_mlp_init(fpc_ctx *ctx, void *model, const float *params)
{
    if (!ctx || !model || !params) return FPC_EINVAL;
    for (int k = 0; k < kParams; ++k)
        if (!std::isfinite(params[k])) return FPC_EINVAL;
    FPC_HIP(hipMemsetAsync(model, 0, mlp_model_bytes(), ctx->stream));
    ModelView mv = view(model);
    FPC_HIP(hipMemcpyAsync(mv.master, params, sizeof(float) * kParams, hipMemcpyHostToDevice, ctx->stream));
    round_weights<<<(kH * kH + 255) / 256, 256, 0, ctx->stream>>>(mv.master, mv.W1h, mv.W2h, mv.W3h);
    FPC_HIP(hipGetLastError());
    FPC_HIP(hipStreamSynchronize(ctx->stream));
    return FPC_OK;
}

extern "C" int fpc_mlp_get(fpc_ctx *ctx, const void *model, float *params_out)
{
    if (!ctx || !model || !params_out) return FPC_EINVAL;
    FPC_HIP(hipMemcpyAsync(params_out, model, sizeof(float) * kParams, hipMemcpyDeviceToHost, ctx->stream));
    FPC_HIP(hipStreamSynchronize(ctx->stream));
    return FPC_OK;
}

extern "C" int fpc_mlp_forward(fpc_ctx *ctx, const float *X, int64_t n, const void *model, float *logits_out)
{
    if (!ctx) return FPC_EINVAL;
    int rc = mlp_forward(ctx, X, n, model, logits_out);
    if (rc) return rc;
    FPC_HIP(hipStreamSynchronize(ctx->stream));
    return FPC_OK;
}

extern "C" int fpc_mlp_grad(fpc_ctx *ctx, const float *X, const float *y, int64_t n, const void *model,
                            float *grad_out)
{
    if (!ctx) return FPC_EINVAL;
    int rc = mlp_grad(ctx, X, y, n, model, grad_out);
    if (rc) return rc;
    FPC_HIP(hipStreamSynchronize(ctx->stream));
    return FPC_OK;
}

extern "C" int fpc_mlp_train_step(fpc_ctx *ctx, const float *X, const float *y, int64_t n, void *model, float lr,
                                  float *loss_out)
{
    if (!ctx || !model || !(lr > 0.f)) return FPC_EINVAL;
    int rc = ctx->flag.ensure(64);
    if (rc) return rc;
    // gradient (+ loss in the last slot) into a scratch vector after the partials
    if ((rc = ctx->mlp_grad.ensure(sizeof(float) * (kParams + 1)))) return rc;
    float *g = ctx->mlp_grad.as<float>();
    if ((rc = mlp_grad(ctx, X, y, n, model, g))) return rc;
    ModelView mv = view(model);
    adam_step<<<(kParams + 255) / 256, 256, 0, ctx->stream>>>(mv.master, mv.m, mv.v, g, mv.step, lr);
    bump_step<<<1, 1, 0, ctx->stream>>>(mv.step);
    round_weights<<<(kH * kH + 255) / 256, 256, 0, ctx->stream>>>(mv.master, mv.W1h, mv.W2h, mv.W3h);
    FPC_HIP(hipGetLastError());
    if (loss_out) FPC_HIP(hipMemcpyAsync(loss_out, g + kParams, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    FPC_HIP(hipStreamSynchronize(ctx->stream));
    return FPC_OK;
}
