// Training of the facet-law surrogate MLP on the GPU: BF16 MFMA forward and
// backward, FP32 accumulation, FP32 master weights and Adam.  C-ABI in
// include/ldpm.h (ldpm_mlp_*).
//
// One wave (64 samples) per block.  Forward activations are kept in LDS in
// row layout (A operand of the next layer) and transposed layout (B operand
// of the weight gradient, whose K dimension is the batch).  Each block writes
// its partial gradient; a second kernel sums the partials over blocks in a
// fixed order (bitwise reproducible), a third applies Adam.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/ldpm.h"
#include "mlp.hpp"

using namespace ldpm;

ldpm_status ldpm_fail(ldpm_status st, const char* fmt, ...);  // ldpm.hip

#define HIP_TRY_M(expr)                                                                          \
    do {                                                                                         \
        hipError_t _e = (expr);                                                                  \
        if (_e != hipSuccess)                                                                    \
            return ldpm_fail(LDPM_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));   \
    } while (0)

namespace {

constexpr int NPB = MLP_NPARAM + 1;  // partial gradient + loss per block

struct TrainLds {
    MlpBf16 W;                  // forward weights
    __bf16 w4t[MLP_H * PA1];    // [k][n]  W4 transposed (n = 3 of 32 used)
    __bf16 w3t[MLP_H * PA];     // [k][n]  W3 transposed
    __bf16 w2t[MLP_H * PA];     // [k][n]  W2 transposed
    __bf16 x[64 * PA1];         // [m][k]
    __bf16 xt[K1 * PA];         // [k][m]
    __bf16 h[3][64 * PA];       // [m][k]
    __bf16 ht[3][64 * PA];      // [k][m]
    __bf16 dz[64 * PA];         // [m][n]
    __bf16 dzt[64 * PA];        // [n][m]
    __bf16 dy[64 * PA1];        // [m][j]
    __bf16 dyt[N4 * PA];        // [j][m]
    float loss[64];
};

__device__ __forceinline__ void load_transposed(const float* __restrict__ p, TrainLds& S, int tid, int nth)
{
    for (int i = tid; i < MLP_H * PA1; i += nth) {
        const int k = i / PA1, n = i % PA1;
        S.w4t[i] = to_bf16(n < MLP_OUT ? p[P_W4 + n * MLP_H + k] : 0.f);
    }
    for (int i = tid; i < MLP_H * PA; i += nth) {
        const int k = i / PA, n = i % PA;
        S.w3t[i] = to_bf16(n < MLP_H ? p[P_W3 + n * MLP_H + k] : 0.f);
        S.w2t[i] = to_bf16(n < MLP_H ? p[P_W2 + n * MLP_H + k] : 0.f);
    }
}

// Forward + backward of 64 samples; writes the block's partial gradient of
// L = sum_m sum_j (y_mj - target_mj)^2 / norm.
__global__ __launch_bounds__(64) void k_mlp_train_block(const float* __restrict__ params,
                                                        const float* __restrict__ X, const float* __restrict__ Y,
                                                        int64_t n, int64_t off, float norm,
                                                        float* __restrict__ partial)
{
    extern __shared__ __align__(16) unsigned char smem[];
    TrainLds& S = *(TrainLds*)smem;
    const int l = threadIdx.x;
    mlp_load_bf16(params, S.W, l, 64);
    load_transposed(params, S, l, 64);
    // samples of this block (wrapping around the data set)
    const int64_t row = (off + (int64_t)blockIdx.x * 64 + l) % n;
    float xin[MLP_IN], tgt[MLP_OUT];
#pragma unroll
    for (int k = 0; k < MLP_IN; k++) xin[k] = X[row * MLP_IN + k];
#pragma unroll
    for (int j = 0; j < MLP_OUT; j++) tgt[j] = Y[row * MLP_OUT + j];
    for (int k = 0; k < PA1; k++) S.x[l * PA1 + k] = to_bf16(k < MLP_IN ? xin[k] : 0.f);
    for (int k = 0; k < K1; k++) S.xt[k * PA + l] = to_bf16(k < MLP_IN ? xin[k] : 0.f);
    __syncthreads();
    // ---- forward ----
    wave_gemm64<1, 4>(S.x, PA1, S.W.w1, PA1, [&](int m, int c, float v) {
        const __bf16 h = to_bf16(act_tanh(v + S.W.b1[c]));
        S.h[0][m * PA + c] = h;
        S.ht[0][c * PA + m] = h;
    });
    __syncthreads();
    wave_gemm64<2, 4>(S.h[0], PA, S.W.w2, PA, [&](int m, int c, float v) {
        const __bf16 h = to_bf16(act_tanh(v + S.W.b2[c]));
        S.h[1][m * PA + c] = h;
        S.ht[1][c * PA + m] = h;
    });
    __syncthreads();
    wave_gemm64<2, 4>(S.h[1], PA, S.W.w3, PA, [&](int m, int c, float v) {
        const __bf16 h = to_bf16(act_tanh(v + S.W.b3[c]));
        S.h[2][m * PA + c] = h;
        S.ht[2][c * PA + m] = h;
    });
    __syncthreads();
    // output and dL/dy = 2 (y - target) / norm
    float* yo = (float*)S.dz;  // scratch for the 64 x 3 outputs (before dz is used)
    wave_gemm64<2, 1>(S.h[2], PA, S.W.w4, PA, [&](int m, int c, float v) {
        if (c < MLP_OUT) yo[m * 4 + c] = v + S.W.b4[c];
    });
    __syncthreads();
    float lsum = 0.f;
    float dyv[MLP_OUT];
#pragma unroll
    for (int j = 0; j < MLP_OUT; j++) {
        const float r = yo[l * 4 + j] - tgt[j];
        lsum += r * r;
        dyv[j] = 2.f * r / norm;
    }
    S.loss[l] = lsum;
    __syncthreads();
    for (int k = 0; k < PA1; k++) S.dy[l * PA1 + k] = to_bf16(k < MLP_OUT ? dyv[k] : 0.f);
    for (int j = 0; j < N4; j++) S.dyt[j * PA + l] = to_bf16(j < MLP_OUT ? dyv[j] : 0.f);
    __syncthreads();
    float* gout = partial + (int64_t)blockIdx.x * NPB;
    // ---- layer 4: dW4[j][k] = sum_m dy[m][j] h3[m][k], db4[j] = sum_m dy ----
    wave_gemm64<2, 1>(S.ht[2], PA, S.dyt, PA, [&](int k, int j, float v) {
        if (j < MLP_OUT) gout[P_W4 + j * MLP_H + k] = v;
    });
    if (l < MLP_OUT) {
        float s = 0.f;
        for (int m = 0; m < 64; m++) s += from_bf16(S.dyt[l * PA + m]);
        gout[P_B4 + l] = s;
    }
    // dz3 = (dy W4) (1 - h3^2)
    wave_gemm64<1, 4>(S.dy, PA1, S.w4t, PA1, [&](int m, int c, float v) {
        const float h = from_bf16(S.h[2][m * PA + c]);
        const __bf16 d = to_bf16(v * (1.f - h * h));
        S.dz[m * PA + c] = d;
        S.dzt[c * PA + m] = d;
    });
    __syncthreads();
    // ---- layers 3, 2: dW = dz^T h_prev, db = sum dz, dz_prev = (dz W)(1 - h_prev^2) ----
    for (int layer = 2; layer >= 1; layer--) {
        const int pw = layer == 2 ? P_W3 : P_W2;
        const int pb = layer == 2 ? P_B3 : P_B2;
        wave_gemm64<2, 4>(S.dzt, PA, S.ht[layer - 1], PA, [&](int o, int k, float v) {
            gout[pw + o * MLP_H + k] = v;
        });
        {
            float s = 0.f;
            for (int m = 0; m < 64; m++) s += from_bf16(S.dzt[l * PA + m]);
            gout[pb + l] = s;
        }
        __syncthreads();
        const __bf16* wt = layer == 2 ? S.w3t : S.w2t;
        wave_gemm64<2, 4>(S.dz, PA, wt, PA, [&](int m, int c, float v) {
            const float h = from_bf16(S.h[layer - 1][m * PA + c]);
            const __bf16 d = to_bf16(v * (1.f - h * h));
            S.dz[m * PA + c] = d;
            S.dzt[c * PA + m] = d;
        });
        __syncthreads();
    }
    // ---- layer 1: dW1[o][k] = sum_m dz1[m][o] x[m][k] ----
    wave_gemm64<2, 2>(S.dzt, PA, S.xt, PA, [&](int o, int k, float v) {
        if (k < MLP_IN) gout[P_W1 + o * MLP_IN + k] = v;
    });
    {
        float s = 0.f;
        for (int m = 0; m < 64; m++) s += from_bf16(S.dzt[l * PA + m]);
        gout[P_B1 + l] = s;
    }
    if (l == 0) {
        float s = 0.f;
        for (int m = 0; m < 64; m++) s += S.loss[m];
        gout[MLP_NPARAM] = s / norm;
    }
}

// grad[p] = sum over blocks in ascending order
__global__ void k_mlp_reduce(const float* __restrict__ partial, int nblocks, float* __restrict__ grad)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPB) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; b++) s += partial[(int64_t)b * NPB + p];
    grad[p] = s;
}

__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_NPARAM) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// forward only (4 waves of 64 rows per block), the same code path as the
// surrogate facet kernel's inference
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ params, const float* __restrict__ X,
                                                     int64_t n, float* __restrict__ Y)
{
    __shared__ MlpFrag W;
    const int tid = threadIdx.x;
    mlp_load_frag(params, W, tid, 256);
    const int64_t row = (int64_t)blockIdx.x * 256 + tid;
    float x[MLP_IN], y[MLP_OUT];
    for (int k = 0; k < MLP_IN; k++) x[k] = row < n ? X[row * MLP_IN + k] : 0.f;
    __syncthreads();
    mlp_infer_wave(W, x, y);
    if (row < n)
        for (int j = 0; j < MLP_OUT; j++) Y[row * MLP_OUT + j] = y[j];
}

}  // namespace

struct ldpm_mlp {
    hipStream_t stream = nullptr;
    float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *partial = nullptr;
    float *X = nullptr, *Y = nullptr;
    int64_t n = 0, off = 0, t = 0;
    int max_blocks = 0;
};

static size_t train_lds() { return sizeof(TrainLds); }

extern "C" {

ldpm_status ldpm_mlp_create(const float* init, void* stream, ldpm_mlp** out)
{
    if (!init || !out) return ldpm_fail(LDPM_ERR_ARG, "null argument");
    *out = nullptr;
    ldpm_mlp* M = new ldpm_mlp();
    M->stream = (hipStream_t)stream;
    const size_t pb = MLP_NPARAM * sizeof(float);
    if (hipMalloc(&M->params, pb) != hipSuccess || hipMalloc(&M->m, pb) != hipSuccess ||
        hipMalloc(&M->v, pb) != hipSuccess || hipMalloc(&M->grad, NPB * sizeof(float)) != hipSuccess) {
        ldpm_mlp_free(M);
        return ldpm_fail(LDPM_ERR_ALLOC, "mlp: device allocation failed");
    }
    HIP_TRY_M(hipMemcpyAsync(M->params, init, pb, hipMemcpyHostToDevice, M->stream));
    HIP_TRY_M(hipMemsetAsync(M->m, 0, pb, M->stream));
    HIP_TRY_M(hipMemsetAsync(M->v, 0, pb, M->stream));
    HIP_TRY_M(hipStreamSynchronize(M->stream));
    HIP_TRY_M(hipFuncSetAttribute((const void*)k_mlp_train_block, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)train_lds()));
    *out = M;
    return LDPM_OK;
}

ldpm_status ldpm_mlp_set_data(ldpm_mlp* M, const float* x, const float* y, int64_t n)
{
    if (!M || !x || !y || n <= 0) return ldpm_fail(LDPM_ERR_ARG, "mlp: bad data");
    (void)hipFree(M->X);
    (void)hipFree(M->Y);
    M->X = M->Y = nullptr;
    if (hipMalloc(&M->X, n * MLP_IN * sizeof(float)) != hipSuccess ||
        hipMalloc(&M->Y, n * MLP_OUT * sizeof(float)) != hipSuccess)
        return ldpm_fail(LDPM_ERR_ALLOC, "mlp: data allocation failed");
    HIP_TRY_M(hipMemcpyAsync(M->X, x, n * MLP_IN * sizeof(float), hipMemcpyHostToDevice, M->stream));
    HIP_TRY_M(hipMemcpyAsync(M->Y, y, n * MLP_OUT * sizeof(float), hipMemcpyHostToDevice, M->stream));
    HIP_TRY_M(hipStreamSynchronize(M->stream));
    M->n = n;
    M->off = 0;
    return LDPM_OK;
}

static ldpm_status ensure_partials(ldpm_mlp* M, int nb)
{
    if (nb <= M->max_blocks) return LDPM_OK;
    (void)hipFree(M->partial);
    M->partial = nullptr;
    if (hipMalloc(&M->partial, (size_t)nb * NPB * sizeof(float)) != hipSuccess)
        return ldpm_fail(LDPM_ERR_ALLOC, "mlp: partial allocation failed");
    M->max_blocks = nb;
    return LDPM_OK;
}

// gradient of the loss over batch samples starting at off (no update)
static ldpm_status grad_pass(ldpm_mlp* M, int32_t batch, int64_t off)
{
    const int nb = (batch + 63) / 64;
    ldpm_status st = ensure_partials(M, nb);
    if (st != LDPM_OK) return st;
    const float norm = (float)(nb * 64);
    hipLaunchKernelGGL(k_mlp_train_block, dim3(nb), dim3(64), train_lds(), M->stream, M->params, M->X, M->Y, M->n,
                       off, norm, M->partial);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NPB + 255) / 256), dim3(256), 0, M->stream, M->partial, nb, M->grad);
    HIP_TRY_M(hipGetLastError());
    return LDPM_OK;
}

ldpm_status ldpm_mlp_grad(ldpm_mlp* M, int32_t batch, int64_t offset, float* grad, float* loss)
{
    if (!M || !grad || batch <= 0 || M->n <= 0) return ldpm_fail(LDPM_ERR_ARG, "mlp: bad gradient request");
    ldpm_status st = grad_pass(M, batch, offset);
    if (st != LDPM_OK) return st;
    std::vector<float> g(NPB);
    HIP_TRY_M(hipMemcpyAsync(g.data(), M->grad, NPB * sizeof(float), hipMemcpyDeviceToHost, M->stream));
    HIP_TRY_M(hipStreamSynchronize(M->stream));
    memcpy(grad, g.data(), MLP_NPARAM * sizeof(float));
    if (loss) *loss = g[MLP_NPARAM];
    return LDPM_OK;
}

ldpm_status ldpm_mlp_train(ldpm_mlp* M, int64_t steps, int32_t batch, float lr, float* last_loss)
{
    if (!M || steps < 0 || batch <= 0 || M->n <= 0 || !(lr > 0)) return ldpm_fail(LDPM_ERR_ARG, "mlp: bad training request");
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const int nb = (batch + 63) / 64;
    for (int64_t s = 0; s < steps; s++) {
        ldpm_status st = grad_pass(M, batch, M->off);
        if (st != LDPM_OK) return st;
        M->t++;
        const float c1 = 1.f - powf(b1, (float)M->t), c2 = 1.f - powf(b2, (float)M->t);
        hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, M->stream, M->params, M->m, M->v,
                           M->grad, lr, b1, b2, eps, c1, c2);
        M->off = (M->off + (int64_t)nb * 64) % M->n;
    }
    HIP_TRY_M(hipGetLastError());
    if (last_loss) {
        float lv = 0.f;
        HIP_TRY_M(hipMemcpyAsync(&lv, M->grad + MLP_NPARAM, sizeof(float), hipMemcpyDeviceToHost, M->stream));
        HIP_TRY_M(hipStreamSynchronize(M->stream));
        *last_loss = lv;
    }
    return LDPM_OK;
}

ldpm_status ldpm_mlp_forward(ldpm_mlp* M, const float* x, int64_t n, float* y)
{
    if (!M || !x || !y || n <= 0) return ldpm_fail(LDPM_ERR_ARG, "mlp: bad forward request");
    float *dx = nullptr, *dy = nullptr;
    if (hipMalloc(&dx, n * MLP_IN * sizeof(float)) != hipSuccess || hipMalloc(&dy, n * MLP_OUT * sizeof(float)) != hipSuccess) {
        (void)hipFree(dx);
        return ldpm_fail(LDPM_ERR_ALLOC, "mlp: forward allocation failed");
    }
    hipError_t e = hipMemcpyAsync(dx, x, n * MLP_IN * sizeof(float), hipMemcpyHostToDevice, M->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, M->stream, M->params, dx,
                           n, dy);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(y, dy, n * MLP_OUT * sizeof(float), hipMemcpyDeviceToHost, M->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(M->stream);
    (void)hipFree(dx);
    (void)hipFree(dy);
    if (e != hipSuccess) return ldpm_fail(LDPM_ERR_DEVICE, "mlp forward failed: %s", hipGetErrorString(e));
    return LDPM_OK;
}

ldpm_status ldpm_mlp_get_params(ldpm_mlp* M, float* params)
{
    if (!M || !params) return ldpm_fail(LDPM_ERR_ARG, "null argument");
    HIP_TRY_M(hipMemcpyAsync(params, M->params, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost, M->stream));
    HIP_TRY_M(hipStreamSynchronize(M->stream));
    return LDPM_OK;
}

int32_t ldpm_mlp_num_params(void) { return MLP_NPARAM; }

void ldpm_mlp_free(ldpm_mlp* M)
{
    if (!M) return;
    (void)hipStreamSynchronize(M->stream);
    for (float* p : {M->params, M->m, M->v, M->grad, M->partial, M->X, M->Y}) (void)hipFree(p);
    delete M;
}

}  // extern "C"
