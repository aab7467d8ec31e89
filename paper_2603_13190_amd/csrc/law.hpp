// Facet constitutive update of LDPM on the device (paper, appendix:
// fracturing, compressive and frictional behaviour), templated on the
// arithmetic type R (double for the FP64 path, float for the mixed path).
//
// The history of a facet is its traction vector t = (t_N, t_M, t_L) and the
// maximum effective strain e_max.  The strain increment de is supplied by the
// caller (from the FP64 particle velocities), so the previous strain is
// e - de and never stored.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ldpm {

// FP64: correctly rounded square root and division.  FP32 (the mixed path,
// held to a stated tolerance, not to ulps): the hardware square root and
// reciprocal, about 1 ulp each.
__device__ __forceinline__ double d_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float d_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double d_div(double a, double b) { return a / b; }
__device__ __forceinline__ float d_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double d_exp(double x) { return exp(x); }
__device__ __forceinline__ double d_log(double x) { return log(x); }
// FP32: exp x = 2^(x log2 e) and log x = log2(x) ln 2 on the transcendental
// unit (a few ulp; overflow to +inf and log 0 = -inf are kept)
__device__ __forceinline__ float d_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ float d_log(float x) { return __builtin_amdgcn_logf(x) * 0.6931471805599453f; }
__device__ __forceinline__ double d_atan2(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float d_atan2(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double d_pow(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float d_pow(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double d_frexp(double x, int* e) { return frexp(x, e); }
__device__ __forceinline__ float d_frexp(float x, int* e) { return frexpf(x, e); }
__device__ __forceinline__ double d_ldexp(double x, int e) { return ldexp(x, e); }
__device__ __forceinline__ float d_ldexp(float x, int e) { return ldexpf(x, e); }
__device__ __forceinline__ double d_abs(double x) { return fabs(x); }
__device__ __forceinline__ double d_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float d_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ float d_abs(float x) { return fabsf(x); }

// |(a, b, c)| weighted as sqrt(a^2 + w (b^2 + c^2)), returned as the scaled
// value sv, its square sv2 and the exponent ex with value = sv * 2^ex.  The
// power-of-two rescaling is exact, so in the normal range the result equals
// the plain formula bit for bit; it only prevents squares of tiny strains
// from underflowing in FP32 (e = 0 while e_N > 0).  In FP64 the squares of
// any strain above 1e-150 are normal, so the plain formula is used (ex = 0).
template <typename R>
__device__ __forceinline__ void scaled_norm(R a, R b, R c, R w, R& sa, R& sbc2, R& sv, R& sv2, int& ex)
{
    if constexpr (sizeof(R) == 8) {
        ex = 0;
        sa = a;
        sbc2 = b * b + c * c;
        sv2 = a * a + w * sbc2;
        sv = d_sqrt(sv2);
        return;
    }
    R mx = d_abs(a);
    mx = d_abs(b) > mx ? d_abs(b) : mx;
    mx = d_abs(c) > mx ? d_abs(c) : mx;
    (void)d_frexp(mx, &ex);
    sa = d_ldexp(a, -ex);
    const R sb = d_ldexp(b, -ex), sc = d_ldexp(c, -ex);
    sbc2 = sb * sb + sc * sc;
    sv2 = sa * sa + w * sbc2;
    sv = d_sqrt(sv2);
}

// Material constants in the facet precision, derived once on the host.
template <typename R>
struct MatDev {
    R E0, alpha, aE0, inv_alpha, inv_E0;
    R sigma_t, l_t, c4;          // c4 = 4 alpha / r_st^2
    R n_t, Hs_over_alpha, k_t;
    R sigma_c0, Hc0, Hc1, kc1, kc2, eV0, ec0, ec1, Ed, beta;
    R sigma_s, sigma_s2, dmu_sN0, mu_inf, inv_sigma_N0;
    R two_over_pi;
};

// Update one facet.  e: current strain; de: increment since the previous
// step; eV: volumetric strain of the facet's tetrahedron; len: edge length.
// t: in = previous traction, out = new traction; emax: in/out.
template <typename R, int LAW>
__device__ __forceinline__ void facet_law(const MatDev<R>& p, R len, const R e[3], const R de[3],
                                          R eV, R t[3], R& emax)
{
    if (LAW == 0) {  // elastic: t = E0 diag(1, alpha, alpha) e
        t[0] = p.E0 * e[0];
        t[1] = p.aE0 * e[1];
        t[2] = p.aE0 * e[2];
        return;
    }
    const R eN = e[0], eM = e[1], eL = e[2];
    if (eN > R(0)) {
        // ---- fracturing behaviour ----
        const R al = p.alpha;
        R sN, sT2, seff, seff2;
        int ex;
        scaled_norm(eN, eM, eL, al, sN, sT2, seff, seff2, ex);
        const R eff = d_ldexp(seff, ex);
        const R o0 = eN - de[0], o1 = eM - de[1], o2 = eL - de[2];
        R so0, soT2, seffo, seffo2;
        int exo;
        scaled_norm(o0, o1, o2, al, so0, soT2, seffo, seffo2, exo);
        const R effo = d_ldexp(seffo, exo);
        // effective-strain increment without cancellation:
        // e^2 - e_old^2 = sum w_i de_i (e_i + e_old_i)
        const R num = de[0] * (eN + o0) + al * (de[1] * (eM + o1) + de[2] * (eL + o2));
        const R den = eff + effo;
        const R deff = den > R(0) ? d_div(num, den) : R(0);
        const R teo = d_sqrt(t[0] * t[0] + (t[1] * t[1] + t[2] * t[2]) * p.inv_alpha);
        const R inv = d_div(R(1), seff);
        const R sn = sN * inv;
        const R cs2 = al * sT2 * (inv * inv);
        const R sigma0 = d_div(R(2) * p.sigma_t, sn + d_sqrt(sn * sn + p.c4 * cs2));
        const R e0 = sigma0 * p.inv_E0;
        const R em = emax > eff ? emax : eff;
        const R over = em - e0;
        R sbt = sigma0;
        if (over > R(0)) {  // softening started: exp(-H0 <e_max - e0> / sigma0)
            const R omega = d_atan2(sN, d_sqrt(al * sT2));
            const R Ht = d_div(R(2) * p.E0, d_div(p.l_t, len) - R(1));
            // (2 omega / pi)^n_t for a base in [0, 1] (0 -> exp(-inf) = 0)
            const R H0 = p.Hs_over_alpha + (Ht - p.Hs_over_alpha) * d_exp(p.n_t * d_log(p.two_over_pi * omega));
            sbt = sigma0 * d_exp(d_div(-H0 * over, sigma0));
        }
        const R etr = p.k_t * (em - sbt * p.inv_E0);
        R ttr;
        if (teo > R(0)) {
            ttr = teo + p.E0 * deff;
        } else if (eff > etr) {
            const R base = etr > effo ? etr : effo;
            const R x = eff - base;
            ttr = x > R(0) ? p.E0 * x : R(0);
        } else {
            ttr = R(0);
        }
        R te = ttr < R(0) ? R(0) : ttr;
        te = te > sbt ? sbt : te;
        const R r = d_ldexp(te * inv, -ex);  // te / eff
        t[0] = r * eN;
        t[1] = al * r * eM;
        t[2] = al * r * eL;
        emax = em;
        return;
    }
    // ---- compressive behaviour ----
    const R eD = eN - eV;
    const R eDV = eV + p.beta * eD;
    R sbc = p.sigma_c0;
    if (-eDV > p.ec0) {  // beyond the onset of pore collapse
        const R aD = eD < R(0) ? -eD : eD;
        const R rDV = (eV <= R(0)) ? d_div(-aD, eV - p.eV0) : d_div(aD, p.eV0);
        const R xr = rDV - p.kc1;
        const R Hc = d_div(p.Hc0 - p.Hc1, R(1) + p.kc2 * (xr > R(0) ? xr : R(0))) + p.Hc1;
        if (-eDV <= p.ec1) {
            sbc = p.sigma_c0 + (-eDV - p.ec0) * Hc;
        } else {
            const R sc1 = p.sigma_c0 + (p.ec1 - p.ec0) * Hc;
            sbc = sc1 * d_exp(d_div((-eDV - p.ec1) * Hc, sc1));
        }
    }
    const R ENc = (-t[0] <= p.sigma_c0) ? p.E0 : p.Ed;
    R tN = t[0] + ENc * de[0];
    tN = tN < -sbc ? -sbc : tN;
    tN = tN > R(0) ? R(0) : tN;
    // ---- frictional behaviour: radial return onto sigma_bs(t_N) ----
    R tM = t[1] + p.aE0 * de[1];
    R tL = t[2] + p.aE0 * de[2];
    const R n2 = tM * tM + tL * tL;
    if (n2 > p.sigma_s2) {  // sigma_bs >= sigma_s for t_N <= 0
        const R sbs = p.sigma_s + p.dmu_sN0 - p.mu_inf * tN - p.dmu_sN0 * d_exp(tN * p.inv_sigma_N0);
        const R nrm = d_sqrt(n2);
        if (nrm > sbs) {
            const R f = d_div(sbs, nrm);
            tM *= f;
            tL *= f;
        }
    }
    t[0] = tN;
    t[1] = tM;
    t[2] = tL;
}

}  // namespace ldpm
