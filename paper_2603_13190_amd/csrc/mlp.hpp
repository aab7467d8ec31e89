// Small MLP (9 -> 64 -> 64 -> 64 -> 3, tanh) on CDNA4 matrix cores:
// BF16 operands, FP32 accumulation, v_mfma_f32_16x16x32_bf16 tiles, one
// wave per 64 rows.  Inference (the surrogate facet kernel and
// k_mlp_forward) keeps the activations in registers (mlp_infer_wave); the
// training kernels stage them in LDS (wave_gemm64, MlpBf16).
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
// Inference with the activations in registers.  Each layer is computed
// transposed, D = W H^T (A operand: weight rows n, B operand: activation
// rows m), so that after a layer lane (r, g) = (l % 16, l / 16) of a 16-row
// tile holds the outputs n = 16 nt + 4 g + i (nt, i = 0..3) of row r: 16
// values, which it passes on as the next layer's B operand.  The dot product
// does not depend on which K slot carries which k (A and B share the
// slots), so the next layer's K slots follow what the lane holds: slot j of
// K step kt in lane group g carries k = 16 (2 kt + j / 4) + 4 g + j % 4.
// The weights are stored in LDS with that assignment, fragment by fragment
// ([tile][step][lane] of 8 values: one conflict-free 16-byte read per lane
// and MFMA).  Layer 1 has one K step: lane group 0 carries features 0..7,
// group 1 feature 8, groups 2 and 3 zeros.  The output layer uses rows 0..2
// of one 16-row tile (rows 3..15 zero).  Rounding points are those of the
// LDS-staged form: BF16 inputs, weights and activations, FP32 sums.
// ---------------------------------------------------------------------------
struct MlpFrag {
    bf16x8 w1[4][64];     // [n tile][lane]
    bf16x8 w2[4][2][64];  // [n tile][K step][lane]
    bf16x8 w3[4][2][64];
    bf16x8 w4[2][64];     // [K step][lane]
    float b1[MLP_H], b2[MLP_H], b3[MLP_H], b4[N4];
};

// k carried by slot j of K step kt in lane group g (hidden layers)
__host__ __device__ __forceinline__ int frag_k(int kt, int g, int j) { return (2 * kt + (j >> 2)) * 16 + 4 * g + (j & 3); }

// Fill an MlpFrag (LDS) from the flat FP32 parameters, block-wide.
__device__ __forceinline__ void mlp_load_frag(const float* __restrict__ p, MlpFrag& W, int tid, int nth)
{
    __bf16* w1 = (__bf16*)W.w1;
    for (int i = tid; i < 4 * 64 * 8; i += nth) {
        const int j = i & 7, lane = (i >> 3) & 63, nt = i >> 9;
        const int n = nt * 16 + (lane & 15), g = lane >> 4;
        const int k = g == 0 ? j : ((g == 1 && j == 0) ? 8 : -1);
        w1[i] = to_bf16(k >= 0 ? p[P_W1 + n * MLP_IN + k] : 0.f);
    }
    __bf16 *w2 = (__bf16*)W.w2, *w3 = (__bf16*)W.w3;
    for (int i = tid; i < 4 * 2 * 64 * 8; i += nth) {
        const int j = i & 7, lane = (i >> 3) & 63, kt = (i >> 9) & 1, nt = i >> 10;
        const int n = nt * 16 + (lane & 15), k = frag_k(kt, lane >> 4, j);
        w2[i] = to_bf16(p[P_W2 + n * MLP_H + k]);
        w3[i] = to_bf16(p[P_W3 + n * MLP_H + k]);
    }
    __bf16* w4 = (__bf16*)W.w4;
    for (int i = tid; i < 2 * 64 * 8; i += nth) {
        const int j = i & 7, lane = (i >> 3) & 63, kt = i >> 9;
        const int n = lane & 15, k = frag_k(kt, lane >> 4, j);
        w4[i] = to_bf16(n < MLP_OUT ? p[P_W4 + n * MLP_H + k] : 0.f);
    }
    for (int i = tid; i < MLP_H; i += nth) {
        W.b1[i] = p[P_B1 + i];
        W.b2[i] = p[P_B2 + i];
        W.b3[i] = p[P_B3 + i];
    }
    for (int i = tid; i < N4; i += nth) W.b4[i] = i < MLP_OUT ? p[P_B4 + i] : 0.f;
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned pack_bf16(float a, float b)
{
    const bf16x2 v = {to_bf16(a), to_bf16(b)};
    return __builtin_bit_cast(unsigned, v);
}

// tanh of the biased results of the four n tiles, packed as the next
// layer's two K steps (tile 2 kt + t fills slots 4 t .. 4 t + 3 of step kt)
__device__ __forceinline__ void act_pack(const f32x4 (&c)[4], const float* bias, int g, bf16x8 (&h)[2])
{
    u32x4 q[2];
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
        const float* b = bias + nt * 16 + 4 * g;
        const unsigned lo = pack_bf16(act_tanh(c[nt][0] + b[0]), act_tanh(c[nt][1] + b[1]));
        const unsigned hi = pack_bf16(act_tanh(c[nt][2] + b[2]), act_tanh(c[nt][3] + b[3]));
        if (nt & 1) {
            q[nt >> 1][2] = lo;
            q[nt >> 1][3] = hi;
        } else {
            q[nt >> 1][0] = lo;
            q[nt >> 1][1] = hi;
        }
    }
    h[0] = __builtin_bit_cast(bf16x8, q[0]);
    h[1] = __builtin_bit_cast(bf16x8, q[1]);
}

// one hidden layer on MT 16-row tiles: h (two K steps per tile) -> h; each
// weight fragment read from LDS serves the MT tiles
template <int MT>
__device__ __forceinline__ void hidden_layer(const bf16x8 (&w)[4][2][64], const float* bias, int l,
                                             bf16x8 (&h)[MT][2])
{
    f32x4 c[MT][4];
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
        const bf16x8 w0 = w[nt][0][l], w1 = w[nt][1][l];
#pragma unroll
        for (int t = 0; t < MT; t++) {
            c[t][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0, h[t][0], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            c[t][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, h[t][1], c[t][nt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < MT; t++) act_pack(c[t], bias, l >> 4, h[t]);
}

// Forward pass of one wave: lane l passes its row's (normalised) features
// x and receives that row's outputs y.  Every lane of the wave must take
// part (wave-uniform call).  The four 16-row tiles are taken MT at a time.
template <int MT = 2>
__device__ __forceinline__ void mlp_infer_wave(const MlpFrag& W, const float (&x)[MLP_IN], float (&y)[MLP_OUT])
{
    const int l = threadIdx.x & 63, g = l >> 4;
    const int P0 = (int)pack_bf16(x[0], x[1]), P1 = (int)pack_bf16(x[2], x[3]);
    const int P2 = (int)pack_bf16(x[4], x[5]), P3 = (int)pack_bf16(x[6], x[7]);
    const int P4 = (int)pack_bf16(x[8], 0.f);
#pragma unroll
    for (int k = 0; k < MLP_OUT; k++) y[k] = 0.f;
#pragma unroll 1
    for (int m0 = 0; m0 < 4; m0 += MT) {
        // the weight fragments are re-read from LDS for every group of row
        // tiles rather than held in registers across groups (88 VGPRs)
        __asm__ volatile("" ::: "memory");
        bf16x8 h[MT][2];
        {
            // layer-1 operand: the features of row 16 mt + r, from that row's lane
            bf16x8 xin[MT];
#pragma unroll
            for (int t = 0; t < MT; t++) {
                const int src = ((m0 + t) * 16 + (l & 15)) * 4;
                const unsigned q0 = (unsigned)__builtin_amdgcn_ds_bpermute(src, P0);
                const unsigned q1 = (unsigned)__builtin_amdgcn_ds_bpermute(src, P1);
                const unsigned q2 = (unsigned)__builtin_amdgcn_ds_bpermute(src, P2);
                const unsigned q3 = (unsigned)__builtin_amdgcn_ds_bpermute(src, P3);
                const unsigned q4 = (unsigned)__builtin_amdgcn_ds_bpermute(src, P4);
                const u32x4 in = g == 0 ? u32x4{q0, q1, q2, q3} : (g == 1 ? u32x4{q4, 0u, 0u, 0u} : u32x4{0u, 0u, 0u, 0u});
                xin[t] = __builtin_bit_cast(bf16x8, in);
            }
            f32x4 c[MT][4];
#pragma unroll
            for (int nt = 0; nt < 4; nt++) {
                const bf16x8 w = W.w1[nt][l];
#pragma unroll
                for (int t = 0; t < MT; t++)
                    c[t][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, xin[t], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < MT; t++) act_pack(c[t], W.b1, g, h[t]);
        }
        hidden_layer<MT>(W.w2, W.b2, l, h);
        hidden_layer<MT>(W.w3, W.b3, l, h);
        f32x4 o[MT];
        {
            const bf16x8 w0 = W.w4[0][l], w1 = W.w4[1][l];
#pragma unroll
            for (int t = 0; t < MT; t++) {
                o[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0, h[t][0], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                o[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, h[t][1], o[t], 0, 0, 0);
            }
        }
        // lane (r, 0) holds outputs 0..3 of row 16 mt + r; that row's lane takes them
#pragma unroll
        for (int t = 0; t < MT; t++) {
#pragma unroll
            for (int k = 0; k < MLP_OUT; k++) {
                const float v = __builtin_bit_cast(
                    float, __builtin_amdgcn_ds_bpermute((l & 15) * 4, __builtin_bit_cast(int, o[t][k] + W.b4[k])));
                if ((l >> 4) == m0 + t) y[k] = v;
            }
        }
    }
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
