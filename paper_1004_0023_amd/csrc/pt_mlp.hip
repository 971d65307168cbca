// pt_mlp.hip -- FP32 training and inference kernels of the ladder network.
//
// The network maps 32 instance features to 64 outputs: 32 -> 128 -> 128 -> 64 with ReLU
// after the two hidden layers.  Parameters, flat FP32 in this order:
//   W1[128][32], b1[128], W2[128][128], b2[128], W3[64][128], b3[64]   (28,992 floats)
// Two training losses (targets q[batch][64]):
//   PT_MLP_LOSS_SOFTMAX:  -sum_j q_j log softmax(z)_j                 (q rows sum to 1)
//   PT_MLP_LOSS_SIGMOID:  -sum_j [q_j log s(z_j) + (1-q_j) log(1-s(z_j))], s = logistic
// both averaged over the batch; either has gradient (p - q)/B in the logits.
//
// Every dense product runs on the matrix cores: one wave computes a 16x16 tile of
// C = op(A) op(B) with v_mfma_f32_16x16x4f32 (K = 4 per instruction); transposes are
// strides.  Elementwise steps (softmax, masks, bias sums, Adam) are plain VALU kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <mutex>
#include <string>

#include "../../include/ptqmc.h"
#include "pt_internal.h"

namespace {

// PT_OK, or PT_EHIP with the HIP error recorded as the last error
int launched(hipError_t e, const char *what)
{
    if (e == hipSuccess) return PT_OK;
    return ptq::report_error(PT_EHIP, (std::string(what) + ": " + hipGetErrorString(e)).c_str());
}

constexpr int kIn = 32, kH = 128, kOut = 64;
constexpr int kW1 = 0, kB1 = kW1 + kH * kIn, kW2 = kB1 + kH, kB2 = kW2 + kH * kH,
              kW3 = kB2 + kH, kB3 = kW3 + kOut * kH, kParams = kB3 + kOut;

typedef float v4f __attribute__((ext_vector_type(4)));

// C[m][n] = sum_k A(m, k) B(k, n) (+ bias[n]) (ReLU if relu), for m < M, n < N, with
// A(m, k) = A[m*am + k*ak] and B(k, n) = B[k*bk + n*bn].  If mask is given, the result is
// multiplied by (mask[m*cm + n] > 0) (the ReLU derivative of a stored activation).
// Grid: (ceil(N/16), ceil(M/16)); block: one 64-lane wave.
__global__ void __launch_bounds__(64) gemm16_kernel(const float *A, int am, int ak,
                                                    const float *B, int bk, int bn,
                                                    float *C, int cm, int M, int N, int K,
                                                    const float *bias, int relu,
                                                    const float *mask)
{
    const int lane = threadIdx.x;
    const int r16 = lane & 15;
    const int kq = lane >> 4;  // 0..3
    const int m0 = blockIdx.y * 16, n0 = blockIdx.x * 16;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    const int am_row = m0 + r16, bn_col = n0 + r16;
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int k = k0 + kq;
        const float a = (am_row < M && k < K) ? A[(int64_t)am_row * am + (int64_t)k * ak] : 0.f;
        const float b = (bn_col < N && k < K) ? B[(int64_t)k * bk + (int64_t)bn_col * bn] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
    // D[i][j] sits in lane j + 16 * (i / 4), element i % 4
    const int col = n0 + r16;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = m0 + 4 * kq + e;
        if (row < M && col < N) {
            float v = acc[e];
            if (bias) v += bias[col];
            if (relu) v = v > 0.f ? v : 0.f;
            if (mask) v = mask[(int64_t)row * cm + col] > 0.f ? v : 0.f;
            C[(int64_t)row * cm + col] = v;
        }
    }
}

// Row-wise softmax cross entropy against soft targets q: dz = (p - q) / B, loss[row].
__global__ void softmax_xent_kernel(const float *z, const float *q, float *dz, float *loss,
                                    int B)
{
    const int row = blockIdx.x;
    const int j = threadIdx.x;  // 64 lanes, one logit each
    if (row >= B) return;
    const float v = z[row * kOut + j];
    float mx = v;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    const float ex = __expf(v - mx);
    float sum = ex;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    const float p = ex / sum;
    const float tq = q[row * kOut + j];
    dz[row * kOut + j] = (p - tq) / (float)B;
    float l = (tq > 0.f) ? -tq * (v - mx - __logf(sum)) : 0.f;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
    if (j == 0) loss[row] = l;
}

// Per-output logistic cross entropy against targets q in [0, 1].
__global__ void sigmoid_xent_kernel(const float *z, const float *q, float *dz, float *loss,
                                    int B)
{
    const int row = blockIdx.x;
    const int j = threadIdx.x;
    if (row >= B) return;
    const float v = z[row * kOut + j];
    const float tq = q[row * kOut + j];
    const float p = 1.f / (1.f + __expf(-v));
    dz[row * kOut + j] = (p - tq) / (float)B;
    // log(1 + e^{-|v|}) + max(v, 0) - q v  is the cross entropy, computed stably
    float l = __logf(1.f + __expf(-fabsf(v))) + fmaxf(v, 0.f) - tq * v;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
    if (j == 0) loss[row] = l;
}

// db[n] = sum_m dz[m][n]
__global__ void colsum_kernel(const float *dz, float *db, int M, int N)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += dz[(int64_t)m * N + n];
    db[n] = s;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int n, float lr,
                            float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t gemm(hipStream_t s, const float *A, int am, int ak, const float *B, int bk, int bn,
                float *C, int cm, int M, int N, int K, const float *bias, int relu,
                const float *mask)
{
    dim3 grid((N + 15) / 16, (M + 15) / 16);
    hipLaunchKernelGGL(gemm16_kernel, grid, dim3(64), 0, s, A, am, ak, B, bk, bn, C, cm, M, N, K,
                       bias, relu, mask);
    return hipGetLastError();
}

struct Acts {
    float *h1, *h2, *z3, *dz3, *dz2, *dz1, *loss;
};

Acts carve(void *ws, int B)
{
    float *f = (float *)ws;
    Acts a;
    a.h1 = f;
    a.h2 = a.h1 + (size_t)B * kH;
    a.z3 = a.h2 + (size_t)B * kH;
    a.dz3 = a.z3 + (size_t)B * kOut;
    a.dz2 = a.dz3 + (size_t)B * kOut;
    a.dz1 = a.dz2 + (size_t)B * kH;
    a.loss = a.dz1 + (size_t)B * kH;
    return a;
}

// Device memory of pt_mlp_forward_static: the two hidden activations (h1, h2) of at most
// PT_MLP_STATIC_MAX_BATCH rows, in a file-scope array that each GPU holds for the life of
// the process.  Host code never passes the array's name to a kernel (on the host it names
// a host-side stand-in): it uses the device address hipGetSymbolAddress returns, taken
// once per device with that device current.
constexpr int kStaticMaxBatch = PT_MLP_STATIC_MAX_BATCH;
static __device__ __align__(256) float scratch[2 * (size_t)kStaticMaxBatch * kH];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on the first call on a device).
int static_scratch(float **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return launched(e, "pt_mlp_forward_static: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return ptq::report_error(PT_EINVAL, "pt_mlp_forward_static: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return launched(e, "pt_mlp_forward_static: hipGetSymbolAddress");
        if (!ptr)
            return ptq::report_error(PT_EHIP, "pt_mlp_forward_static: no device address for the scratch array");
        g_scratch_dev[dev] = static_cast<float *>(ptr);
    }
    *out = g_scratch_dev[dev];
    return PT_OK;
}

hipError_t forward(hipStream_t s, const float *P, const float *x, const Acts &a, float *out, int B)
{
    hipError_t e;
    // h1 = relu(x W1^T + b1): A = x [B x 32], B(k, n) = W1[n][k]
    if ((e = gemm(s, x, kIn, 1, P + kW1, 1, kIn, a.h1, kH, B, kH, kIn, P + kB1, 1, nullptr))) return e;
    if ((e = gemm(s, a.h1, kH, 1, P + kW2, 1, kH, a.h2, kH, B, kH, kH, P + kB2, 1, nullptr))) return e;
    return gemm(s, a.h2, kH, 1, P + kW3, 1, kH, out, kOut, B, kOut, kH, P + kB3, 0, nullptr);
}

}  // namespace

extern "C" {

int32_t pt_mlp_param_count(void) { return kParams; }

size_t pt_mlp_workspace_bytes(int32_t batch)
{
    if (batch < 1) return 0;
    return sizeof(float) * ((size_t)batch * (kH + kH + kOut + kOut + kH + kH) + (size_t)batch);
}

int pt_mlp_forward(const float *params, const float *x, float *logits, int32_t batch,
                   void *workspace, void *stream)
{
    if (!params || !x || !logits || !workspace)
        return ptq::report_error(PT_EINVAL, "pt_mlp_forward: null pointer");
    if (batch < 1) return ptq::report_error(PT_EINVAL, "pt_mlp_forward: batch < 1");
    hipStream_t s = (hipStream_t)stream;
    const Acts a = carve(workspace, batch);
    return launched(forward(s, params, x, a, logits, batch), "pt_mlp_forward");
}

int pt_mlp_forward_static(const float *params, const float *x, float *logits, int32_t batch,
                          void *stream)
{
    if (!params || !x || !logits)
        return ptq::report_error(PT_EINVAL, "pt_mlp_forward_static: null pointer");
    if (batch < 1) return ptq::report_error(PT_EINVAL, "pt_mlp_forward_static: batch < 1");
    if (batch > kStaticMaxBatch)
        return ptq::report_error(PT_EINVAL, ("pt_mlp_forward_static: batch " + std::to_string(batch) +
                                             " exceeds PT_MLP_STATIC_MAX_BATCH (" +
                                             std::to_string(kStaticMaxBatch) + ")").c_str());
    float *ws = nullptr;
    const int rc = static_scratch(&ws);
    if (rc) return rc;
    // the forward pass reads only h1 and h2, each written in full before it is read, so
    // nothing left by an earlier call needs clearing
    Acts a{};
    a.h1 = ws;
    a.h2 = ws + (size_t)batch * kH;
    return launched(forward((hipStream_t)stream, params, x, a, logits, batch), "pt_mlp_forward_static");
}

int pt_mlp_loss_grad(const float *params, const float *x, const float *target, int32_t batch,
                     int32_t loss_kind, float *grads, float *loss, void *workspace, void *stream)
{
    if (!params || !x || !target || !grads || !loss || !workspace)
        return ptq::report_error(PT_EINVAL, "pt_mlp_loss_grad: null pointer");
    if (batch < 1) return ptq::report_error(PT_EINVAL, "pt_mlp_loss_grad: batch < 1");
    if (loss_kind != PT_MLP_LOSS_SOFTMAX && loss_kind != PT_MLP_LOSS_SIGMOID)
        return ptq::report_error(PT_EINVAL, "pt_mlp_loss_grad: unknown loss kind");
    hipStream_t s = (hipStream_t)stream;
    const Acts a = carve(workspace, batch);
    const float *P = params;
    float *G = grads;
    const int B = batch;
    hipError_t e = forward(s, P, x, a, a.z3, B);
    if (e != hipSuccess) return launched(e, "pt_mlp_loss_grad");
    if (loss_kind == PT_MLP_LOSS_SOFTMAX)
        hipLaunchKernelGGL(softmax_xent_kernel, dim3(B), dim3(64), 0, s, a.z3, target, a.dz3, a.loss, B);
    else
        hipLaunchKernelGGL(sigmoid_xent_kernel, dim3(B), dim3(64), 0, s, a.z3, target, a.dz3, a.loss, B);
    e = hipGetLastError();
    // layer 3: dW3[o][k] = sum_b dz3[b][o] h2[b][k]; db3; dz2 = (dz3 W3) * [h2 > 0]
    if (!e) e = gemm(s, a.dz3, 1, kOut, a.h2, kH, 1, G + kW3, kH, kOut, kH, B, nullptr, 0, nullptr);
    if (!e) { hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(kOut), 0, s, a.dz3, G + kB3, B, kOut); e = hipGetLastError(); }
    if (!e) e = gemm(s, a.dz3, kOut, 1, P + kW3, kH, 1, a.dz2, kH, B, kH, kOut, nullptr, 0, a.h2);
    // layer 2
    if (!e) e = gemm(s, a.dz2, 1, kH, a.h1, kH, 1, G + kW2, kH, kH, kH, B, nullptr, 0, nullptr);
    if (!e) { hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(kH), 0, s, a.dz2, G + kB2, B, kH); e = hipGetLastError(); }
    if (!e) e = gemm(s, a.dz2, kH, 1, P + kW2, kH, 1, a.dz1, kH, B, kH, kH, nullptr, 0, a.h1);
    // layer 1
    if (!e) e = gemm(s, a.dz1, 1, kH, x, kIn, 1, G + kW1, kIn, kH, kIn, B, nullptr, 0, nullptr);
    if (!e) { hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(kH), 0, s, a.dz1, G + kB1, B, kH); e = hipGetLastError(); }
    // loss[0] = sum over the batch of the per-sample cross entropies
    if (!e) { hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(1), 0, s, a.loss, loss, B, 1); e = hipGetLastError(); }
    return launched(e, "pt_mlp_loss_grad");
}

int pt_mlp_adam(float *params, const float *grads, float *m, float *v, int32_t n, float lr,
                float beta1, float beta2, float eps, int32_t step, void *stream)
{
    if (!params || !grads || !m || !v) return ptq::report_error(PT_EINVAL, "pt_mlp_adam: null pointer");
    if (n < 1 || step < 1) return ptq::report_error(PT_EINVAL, "pt_mlp_adam: n < 1 or step < 1");
    // bias corrections 1 - beta^step
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       params, grads, m, v, n, lr, beta1, beta2, eps, c1, c2);
    return launched(hipGetLastError(), "pt_mlp_adam");
}

}  // extern "C"
