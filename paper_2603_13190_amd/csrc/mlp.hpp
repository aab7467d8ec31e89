// Small MLP (9 -> 64 -> 64 -> 64 -> 3, tanh) on CDNA4 matrix cores:
// BF16 operands, FP32 accumulation, v_mfma_f32_16x16x32_bf16 tiles, one
// wave per 64 rows.  Shared by the surrogate facet kernel (inference) and
// the training kernels.
//
// Parameters (flat FP32 vector, 9155 values, weights stored [out][in]):
//   W1[64][9] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3]
//
// Fragment layout of the 16x16x32 MFMA used here: lane l supplies row
// (l % 16) of A and column (l % 16) of B, each with the 8 K-values
// 8*(l/16) .. 8*(l/16)+7 (A and B use the same K slots, so the dot product
// does not depend on the hardware's K order); the result lane l holds rows
// 4*(l/16)+i (i = 0..3) of column l % 16.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ldpm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MLP_IN = 9, MLP_H = 64, MLP_OUT = 3;
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + 2 * (MLP_H * MLP_H + MLP_H) + MLP_OUT * MLP_H + MLP_OUT;
// offsets in the flat parameter vector
constexpr int P_W1 = 0, P_B1 = P_W1 + MLP_H * MLP_IN, P_W2 = P_B1 + MLP_H, P_B2 = P_W2 + MLP_H * MLP_H,
              P_W3 = P_B2 + MLP_H, P_B3 = P_W3 + MLP_H * MLP_H, P_W4 = P_B3 + MLP_H,
              P_B4 = P_W4 + MLP_OUT * MLP_H;
static_assert(P_B4 + MLP_OUT == MLP_NPARAM, "parameter layout");

// padded LDS shapes (bf16 elements)
constexpr int K1 = 32;          // input features padded to one K step
constexpr int PA1 = K1 + 8;     // row pitch of 32-wide tiles
constexpr int PA = MLP_H + 8;   // row pitch of 64-wide tiles
constexpr int N4 = 16;          // output layer padded to one N tile

// BF16 weights of one network in LDS / global (row-major [out][in], padded)
struct MlpBf16 {
    __bf16 w1[MLP_H * PA1];  // [64][40]  (in 9 of 32 used)
    __bf16 w2[MLP_H * PA];   // [64][72]
    __bf16 w3[MLP_H * PA];   // [64][72]
    __bf16 w4[N4 * PA];      // [16][72]  (out 3 of 16 used)
    float b1[MLP_H], b2[MLP_H], b3[MLP_H], b4[N4];
};

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }
__device__ __forceinline__ float from_bf16(__bf16 x) { return (float)x; }

// tanh x = 1 - 2 / (2^(2 x log2 e) + 1) on the transcendental unit (exp2 and
// reciprocal, each about 1 ulp): absolute error ~1e-7, below the BF16
// rounding the activations then undergo; saturates to +-1 through exp2's
// overflow to +inf and underflow to 0.  Training and inference share it.
__device__ __forceinline__ float act_tanh(float x)
{
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);
    return 1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f);
}

// C[64 x 16*NT] tile loop for one wave: A rows from A (pitch pa), B given
// transposed as Bt (row n holds column n of B, pitch pb), KT steps of 32.
// epi(m, n, value) receives every result element.
template <int KT, int NT, typename Epi>
__device__ __forceinline__ void wave_gemm64(const __bf16* __restrict__ A, int pa, const __bf16* __restrict__ Bt,
                                            int pb, Epi epi)
{
    const int l = threadIdx.x & 63;
    const int r = l & 15, g = l >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        bf16x8 a[KT];
#pragma unroll
        for (int kt = 0; kt < KT; kt++) a[kt] = *(const bf16x8*)(A + (mt * 16 + r) * pa + kt * 32 + 8 * g);
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < KT; kt++) {
                const bf16x8 b = *(const bf16x8*)(Bt + (nt * 16 + r) * pb + kt * 32 + 8 * g);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kt], b, c, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; i++) epi(mt * 16 + 4 * g + i, nt * 16 + r, c[i]);
        }
    }
}

// Forward pass of one wave's 64 rows, in place: buf holds the input rows
// (64 x PA pitch, first 32 columns = padded features) and receives each
// layer's activations; out[m*4 + j] receives the 3 outputs of row m.
// Every A fragment of an M tile is read into registers before that tile's
// rows are overwritten, and a wave's LDS accesses complete in order.
__device__ __forceinline__ void mlp_forward_wave(const MlpBf16& W, __bf16* buf, float* out)
{
    wave_gemm64<1, 4>(buf, PA, W.w1, PA1, [&](int m, int n, float v) {
        buf[m * PA + n] = to_bf16(act_tanh(v + W.b1[n]));
    });
    __builtin_amdgcn_wave_barrier();
    wave_gemm64<2, 4>(buf, PA, W.w2, PA, [&](int m, int n, float v) {
        buf[m * PA + n] = to_bf16(act_tanh(v + W.b2[n]));
    });
    __builtin_amdgcn_wave_barrier();
    wave_gemm64<2, 4>(buf, PA, W.w3, PA, [&](int m, int n, float v) {
        buf[m * PA + n] = to_bf16(act_tanh(v + W.b3[n]));
    });
    __builtin_amdgcn_wave_barrier();
    wave_gemm64<2, 1>(buf, PA, W.w4, PA, [&](int m, int n, float v) {
        if (n < MLP_OUT) out[m * 4 + n] = v + W.b4[n];
    });
    __builtin_amdgcn_wave_barrier();
}

// Fill an MlpBf16 (LDS or global) from the flat FP32 parameters, block-wide.
__device__ __forceinline__ void mlp_load_bf16(const float* __restrict__ p, MlpBf16& W, int tid, int nth)
{
    for (int i = tid; i < MLP_H * PA1; i += nth) {
        const int o = i / PA1, k = i % PA1;
        W.w1[i] = to_bf16(k < MLP_IN ? p[P_W1 + o * MLP_IN + k] : 0.f);
    }
    for (int i = tid; i < MLP_H * PA; i += nth) {
        const int o = i / PA, k = i % PA;
        W.w2[i] = to_bf16(k < MLP_H ? p[P_W2 + o * MLP_H + k] : 0.f);
        W.w3[i] = to_bf16(k < MLP_H ? p[P_W3 + o * MLP_H + k] : 0.f);
    }
    for (int i = tid; i < N4 * PA; i += nth) {
        const int o = i / PA, k = i % PA;
        W.w4[i] = to_bf16((o < MLP_OUT && k < MLP_H) ? p[P_W4 + o * MLP_H + k] : 0.f);
    }
    for (int i = tid; i < MLP_H; i += nth) {
        W.b1[i] = p[P_B1 + i];
        W.b2[i] = p[P_B2 + i];
        W.b3[i] = p[P_B3 + i];
    }
    for (int i = tid; i < N4; i += nth) W.b4[i] = i < MLP_OUT ? p[P_B4 + i] : 0.f;
}

// ---------------------------------------------------------------------------
// Surrogate features of a facet in a frame aligned with its trial shear
// traction t*_T = t_old,T + alpha E0 de_T (tangent-frame invariant):
//   x = [de_N, de_par, de_perp, e_N, e_par, e_perp, t_N, t_par, t_perp]_old
// u = unit(t*_T) (or (1, 0) when t*_T vanishes); the output is the traction
// residual over the elastic predictor t_old + E de in the same frame.
// ---------------------------------------------------------------------------
struct AlignedFrame {
    float uM, uL;
};

__device__ __forceinline__ AlignedFrame shear_frame(float tM, float tL)
{
    const float n2 = tM * tM + tL * tL;
    AlignedFrame f{1.f, 0.f};
    if (n2 > 1e-30f) {
        const float in = 1.f / sqrtf(n2);
        f.uM = tM * in;
        f.uL = tL * in;
    }
    return f;
}

__device__ __forceinline__ void to_frame(const AlignedFrame& f, float aM, float aL, float& par, float& perp)
{
    par = aM * f.uM + aL * f.uL;
    perp = -aM * f.uL + aL * f.uM;
}

__device__ __forceinline__ void from_frame(const AlignedFrame& f, float par, float perp, float& aM, float& aL)
{
    aM = par * f.uM - perp * f.uL;
    aL = par * f.uL + perp * f.uM;
}

}  // namespace ldpm
