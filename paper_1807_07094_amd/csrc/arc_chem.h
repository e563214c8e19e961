// arc_chem.h -- rate coefficients and cooling of the chemistry step (section 2.8), shared
// by the plain solver and the learned step's gate. Hui & Gnedin (1997) appendix fits with
// lambda = 2 T_i / T; coefficients in FP32, products with densities in FP64.
#pragma once

#include <hip/hip_runtime.h>

namespace arc {

namespace chem {

constexpr float kTHI = 157807.0f, kTHeI = 285335.0f, kTHeII = 631515.0f;
constexpr double kKB = 1.380649e-16;
constexpr double kEV = 1.602176634e-12;

// e^x and 2^x from the hardware base-2 exponential (relative error ~1e-6 here, far below
// the accuracy of the fits they serve).
__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }

// The fits are products of powers of lambda = 2 T_i / T and of T. Every factor is evaluated
// as a power of two, so that one hardware log2 of T serves all of them and the quotients
// of the fits become differences of exponents (no divisions):
//   lambda^p = 2^(p L),  (1 + (lambda / c)^p)^q = 2^(q log2(1 + 2^(p (L - log2 c)))),
// with L = log2 lambda = log2(2 T_i) - log2 T.
struct Lam {
    float lt;                 // log2 T
    float hi, hei, heii;      // lambda_HI, lambda_HeI, lambda_HeII
    float lhi, lhei, lheii;   // their base-2 logarithms
};

__device__ __forceinline__ Lam lambdas(float T)
{
    Lam l;
    l.lt = __builtin_amdgcn_logf(T);
    const float it = __builtin_amdgcn_rcpf(T);
    l.hi = 2.0f * kTHI * it;
    l.hei = 2.0f * kTHeI * it;
    l.heii = 2.0f * kTHeII * it;
    l.lhi = 18.267801676247630f - l.lt;    // log2(2 T_HI)
    l.lhei = 19.122297197274480f - l.lt;   // log2(2 T_HeI)
    l.lheii = 20.268457476333417f - l.lt;  // log2(2 T_HeII)
    return l;
}

// q log2(1 + (lambda / c)^p) from L = log2 lambda and c2 = log2 c.
__device__ __forceinline__ float log2_den(float L, float c2, float p, float q)
{
    return q * __builtin_amdgcn_logf(1.0f + fexp2(p * (L - c2)));
}

constexpr float kL2_2740 = 1.4541758931858022f;   // log2 2.740
constexpr float kL2_0354 = -1.4981787345790898f;  // log2 0.354
constexpr float kL2_0416 = -1.2653445665209950f;  // log2 0.416
constexpr float kL2_0553 = -0.8546486144273799f;  // log2 0.553
constexpr float kL2_2250 = 1.1699250014423124f;   // log2 2.250
constexpr float kLog2e = 1.4426950408889634f;

struct Coef {
    float a_hii, a_heii, a_heiii, k_hi, k_hei, k_heii;
};

// Dielectronic recombination of HeII: 1.90e-3 T^-1.5 e^(-0.75 lambda_HeII / 2) (1 + 0.3 e^(-0.15 lambda_HeII / 2)).
__device__ __forceinline__ float dielectronic(const Lam& l)
{
    return 1.90e-3f * fexp2(-1.5f * l.lt - 0.375f * kLog2e * l.heii) * (1.0f + 0.3f * fexp2(-0.075f * kLog2e * l.heii));
}

__device__ __forceinline__ Coef coefficients(const Lam& l)
{
    Coef c;
    // case-B recombination 2.753e-14 lambda^1.5 / (1 + (lambda / 2.740)^0.407)^2.242 (HeIII: twice, at lambda_HeII)
    c.a_hii = 2.753e-14f * fexp2(1.5f * l.lhi - log2_den(l.lhi, kL2_2740, 0.407f, 2.242f));
    c.a_heii = 1.26e-14f * fexp2(0.750f * l.lhei) + dielectronic(l);
    c.a_heiii = 2.0f * 2.753e-14f * fexp2(1.5f * l.lheii - log2_den(l.lheii, kL2_2740, 0.407f, 2.242f));
    // collisional ionisation A T^-1.5 e^(-lambda / 2) lambda^-p / (1 + (lambda / c)^r)^s
    c.k_hi = 21.11f * fexp2(-1.5f * l.lt - 0.5f * kLog2e * l.hi - 1.089f * l.lhi - log2_den(l.lhi, kL2_0354, 0.874f, 1.101f));
    c.k_hei =
        32.38f * fexp2(-1.5f * l.lt - 0.5f * kLog2e * l.hei - 1.146f * l.lhei - log2_den(l.lhei, kL2_0416, 0.987f, 1.056f));
    c.k_heii = 19.95f *
               fexp2(-1.5f * l.lt - 0.5f * kLog2e * l.heii - 1.089f * l.lheii - log2_den(l.lheii, kL2_0553, 0.735f, 1.275f));
    return c;
}

__device__ __forceinline__ Coef coefficients(float T) { return coefficients(lambdas(T)); }

// Cooling per volume [erg cm^-3 s^-1]: recombination, collisional ionisation,
// collisional excitation, bremsstrahlung. Rate coefficients in FP32, products in FP64.
__device__ __forceinline__ double cooling(float T, const Lam& l, const Coef& k, double ne, double nhi, double nhii,
                                          double nhei, double nheii, double nheiii, int collisional)
{
    // recombination cooling: 3.435e-30 T lambda^1.970 / (1 + (lambda / 2.250)^0.376)^3.720; HeIII is
    // hydrogenic (Z^3 times hydrogen at T / Z^2, Z = 2), i.e. the same fit at lambda_HeII times 2 (the fit
    // carries one explicit T); HeII: k_B T 1.26e-14 lambda_HeI^0.750
    const float rec_hii = 3.435e-30f * fexp2(l.lt + 1.970f * l.lhi - log2_den(l.lhi, kL2_2250, 0.376f, 3.720f));
    const float rec_heii = (1.380649e-16f * 1.26e-14f) * fexp2(l.lt + 0.750f * l.lhei);
    const float rec_heiii = 2.0f * 3.435e-30f * fexp2(l.lt + 1.970f * l.lheii - log2_den(l.lheii, kL2_2250, 0.376f, 3.720f));
    const double diel_cool = 0.75 * 54.418 * kEV * (double)dielectronic(l);
    double lam = ne * ((double)rec_hii * nhii + (double)rec_heii * nheii + (double)rec_heiii * nheiii + diel_cool * nheii);
    if (collisional)
        lam += ne * (13.598 * kEV * (double)k.k_hi * nhi + 24.587 * kEV * (double)k.k_hei * nhei +
                     54.418 * kEV * (double)k.k_heii * nheii);
    // collisional excitation, damped by 1 / (1 + (T / 1e5)^(1/2))
    const float idamp = __builtin_amdgcn_rcpf(1.0f + sqrtf(T * 1e-5f));
    lam += ne * nhi * (double)(7.5e-19f * fexp2(-0.375f * kLog2e * l.hi) * idamp);
    lam += ne * nheii * (double)(5.54e-17f * fexp2(-0.397f * l.lt - 0.375f * kLog2e * l.heii) * idamp);
    // bremsstrahlung with the Gaunt factor 1.1 + 0.34 e^(-(5.5 - log10 T)^2 / 3)
    const float lt10 = l.lt * 0.30102999566398120f;
    const float gff = 1.1f + 0.34f * fexp(-(5.5f - lt10) * (5.5f - lt10) * (1.0f / 3.0f));
    lam += (double)(1.42e-27f * gff * sqrtf(T)) * (nhii + nheii + 4.0 * nheiii) * ne;
    return lam;
}

}  // namespace chem

}  // namespace arc
