// Cost-model MLP: forward, backward and Adam on the GPU, FP32.
//
// The learned fusion planner scores candidate plans with a three-layer
// perceptron (features -> H -> H -> 1, ReLU) trained on pass timings the
// simulator measures itself.  Its products are small dense contractions, so
// they run on MFMA 16x16x4 FP32 tiles (one wave per 16x16 output tile,
// bounds-checked loads, fused bias / ReLU / ReLU-mask epilogues).
//   forward:  Z1 = X W1 + b1, H1 = relu(Z1), Z2 = H1 W2 + b2, H2 = relu(Z2),
//             y = H2 W3 + b3
//   loss:     L = (1/B) sum (y - t)^2
//   backward: dy = 2/B (y - t); dW3 = H2^T dy; db3 = sum dy; dZ2 = (dy W3^T) . [Z2 > 0];
//             dW2 = H1^T dZ2; db2 = colsum dZ2; dZ1 = (dZ2 W2^T) . [Z1 > 0];
//             dW1 = X^T dZ1; db1 = colsum dZ1
//   Adam (Kingma & Ba 2015) with bias correction.
// Parameters are packed [W1 (d x H), b1 (H), W2 (H x H), b2 (H), W3 (H x 1), b3 (1)],
// row-major.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.hpp"

namespace qvm {

typedef float mf32x4 __attribute__((ext_vector_type(4)));

struct GemmArgs {
    int M, N, K;
    const float* A;
    long long sai, sak;       // A(i, k) = A[i * sai + k * sak]
    const float* B;
    long long sbk, sbj;       // B(k, j) = B[k * sbk + j * sbj]
    float* C;                 // C[i * N + j]
    const float* bias;        // added per column (nullable)
    float* H;                 // mode 1: relu(C) stored here
    const float* Zm;          // mode 2: C *= [Zm[i * N + j] > 0]
    int mode;
};

// One wave per 16x16 output tile; 4 waves per block.
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int tn = (g.N + 15) / 16;
    const int tm = (g.M + 15) / 16;
    if (tile >= tm * tn) return;
    const int i0 = (tile / tn) * 16, j0 = (tile % tn) * 16;
    const int ri = i0 + (lane & 15), cj = j0 + (lane & 15), kk = lane >> 4;
    mf32x4 acc = {0, 0, 0, 0};
    for (int k0 = 0; k0 < g.K; k0 += 4) {
        const int k = k0 + kk;
        const float a = (ri < g.M && k < g.K) ? g.A[ri * g.sai + k * g.sak] : 0.f;
        const float b = (cj < g.N && k < g.K) ? g.B[k * g.sbk + cj * g.sbj] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + 4 * (lane >> 4) + r, j = j0 + (lane & 15);
        if (i >= g.M || j >= g.N) continue;
        float v = acc[r];
        if (g.bias) v += g.bias[j];
        if (g.mode == 2 && !(g.Zm[(long long)i * g.N + j] > 0.f)) v = 0.f;
        g.C[(long long)i * g.N + j] = v;
        if (g.mode == 1) g.H[(long long)i * g.N + j] = v > 0.f ? v : 0.f;
    }
}

// out[j] = sum_i D[i * N + j], rows in order.
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ D, int M, int N,
                                                float* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int i = 0; i < M; ++i) s += D[(long long)i * N + j];
    out[j] = s;
}

// dy = 2/B (y - t); loss = mean (y - t)^2 (single block, fixed order).
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             int B, float* __restrict__ dy, float* __restrict__ loss) {
    __shared__ float sh[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < B; i += 256) {
        const float r = y[i] - t[i];
        dy[i] = 2.f * r / (float)B;
        s += r * r;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) *loss = sh[0] / (float)B;
}

__global__ __launch_bounds__(256) void k_adam(size_t n, float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static qvm_status gemm(GemmArgs g, hipStream_t s) {
    const int tiles = ((g.M + 15) / 16) * ((g.N + 15) / 16);
    hipLaunchKernelGGL(k_gemm, dim3((tiles + 3) / 4), dim3(256), 0, s, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(QVM_EDEVICE, std::string("mlp gemm launch: ") + hipGetErrorString(e));
    return QVM_OK;
}

struct MlpView {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};

static MlpView view(const float* P, int d, int H) {
    MlpView v;
    v.W1 = P;
    v.b1 = v.W1 + (size_t)d * H;
    v.W2 = v.b1 + H;
    v.b2 = v.W2 + (size_t)H * H;
    v.W3 = v.b2 + H;
    v.b3 = v.W3 + H;
    return v;
}

static qvm_status check_dims(int B, int d, int H) {
    if (B < 1 || d < 1 || H < 1 || B > (1 << 24) || d > 4096 || H > 4096)
        return fail(QVM_EARG, "mlp: batch/features/hidden out of range");
    return QVM_OK;
}

}  // namespace qvm

using namespace qvm;

extern "C" {

size_t qvm_mlp_param_count(int d, int hidden) {
    return (size_t)d * hidden + hidden + (size_t)hidden * hidden + hidden + hidden + 1;
}

qvm_status qvm_mlp_forward(int B, int d, int H, const float* X, const float* params, float* act,
                           float* y, void* stream) {
    qvm_status st = check_dims(B, d, H);
    if (st) return st;
    if (!X || !params || !act || !y) return fail(QVM_EARG, "mlp: NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    MlpView P = view(params, d, H);
    float *Z1 = act, *H1 = Z1 + (size_t)B * H, *Z2 = H1 + (size_t)B * H, *H2 = Z2 + (size_t)B * H;
    if ((st = gemm({B, H, d, X, d, 1, P.W1, H, 1, Z1, P.b1, H1, nullptr, 1}, s))) return st;
    if ((st = gemm({B, H, H, H1, H, 1, P.W2, H, 1, Z2, P.b2, H2, nullptr, 1}, s))) return st;
    return gemm({B, 1, H, H2, H, 1, P.W3, 1, 1, y, P.b3, nullptr, nullptr, 0}, s);
}

qvm_status qvm_mlp_backward(int B, int d, int H, const float* X, const float* t, const float* params,
                            const float* act, const float* y, float* grads, float* work,
                            float* loss_dev, void* stream) {
    qvm_status st = check_dims(B, d, H);
    if (st) return st;
    if (!X || !t || !params || !act || !y || !grads || !work) return fail(QVM_EARG, "mlp: NULL pointer");
    hipStream_t s = (hipStream_t)stream;
    MlpView P = view(params, d, H);
    const float *Z1 = act, *H1 = Z1 + (size_t)B * H, *Z2 = H1 + (size_t)B * H, *H2 = Z2 + (size_t)B * H;
    float* gW1 = grads;
    float* gb1 = gW1 + (size_t)d * H;
    float* gW2 = gb1 + H;
    float* gb2 = gW2 + (size_t)H * H;
    float* gW3 = gb2 + H;
    float* gb3 = gW3 + H;
    float *dZ2 = work, *dZ1 = dZ2 + (size_t)B * H, *dy = dZ1 + (size_t)B * H;
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, s, y, t, B, dy, loss_dev);
    // dW3 = H2^T dy  [H x 1];  db3 = sum dy
    if ((st = gemm({H, 1, B, H2, 1, H, dy, 1, 1, gW3, nullptr, nullptr, nullptr, 0}, s))) return st;
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, s, dy, B, 1, gb3);
    // dZ2 = (dy W3^T) . [Z2 > 0]  [B x H]
    if ((st = gemm({B, H, 1, dy, 1, 1, P.W3, 1, 1, dZ2, nullptr, nullptr, Z2, 2}, s))) return st;
    if ((st = gemm({H, H, B, H1, 1, H, dZ2, H, 1, gW2, nullptr, nullptr, nullptr, 0}, s))) return st;
    hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, dZ2, B, H, gb2);
    // dZ1 = (dZ2 W2^T) . [Z1 > 0]: W2^T(k, j) = W2[j * H + k]
    if ((st = gemm({B, H, H, dZ2, H, 1, P.W2, 1, H, dZ1, nullptr, nullptr, Z1, 2}, s))) return st;
    if ((st = gemm({d, H, B, X, 1, d, dZ1, H, 1, gW1, nullptr, nullptr, nullptr, 0}, s))) return st;
    hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, dZ1, B, H, gb1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(QVM_EDEVICE, std::string("mlp backward: ") + hipGetErrorString(e));
    return QVM_OK;
}

qvm_status qvm_mlp_adam_step(size_t n, float* params, const float* grads, float* m, float* v, int step,
                             float lr, float beta1, float beta2, float eps, void* stream) {
    if (!params || !grads || !m || !v) return fail(QVM_EARG, "adam: NULL pointer");
    if (step < 1) return fail(QVM_EARG, "adam: step counts from 1");
    const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n,
                       params, grads, m, v, lr, beta1, beta2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(QVM_EDEVICE, std::string("adam: ") + hipGetErrorString(e));
    return QVM_OK;
}

}  // extern "C"
