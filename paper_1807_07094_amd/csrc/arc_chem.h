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

// x^y for x > 0 and e^x from the hardware base-2 logarithm and exponential (relative error
// ~1e-6 here, far below the accuracy of the fits they serve).
__device__ __forceinline__ float fpow(float x, float y) { return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x)); }
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }

struct Coef {
    float a_hii, a_heii, a_heiii, k_hi, k_hei, k_heii;
};

__device__ __forceinline__ Coef coefficients(float T)
{
    const float lhi = 2.0f * kTHI / T, lhei = 2.0f * kTHeI / T, lheii = 2.0f * kTHeII / T;
    const float t15 = fpow(T, -1.5f);
    Coef c;
    c.a_hii = 2.753e-14f * fpow(lhi, 1.5f) / fpow(1.0f + fpow(lhi / 2.740f, 0.407f), 2.242f);
    const float diel = 1.90e-3f * t15 * fexp(-0.75f * lheii / 2.0f) * (1.0f + 0.3f * fexp(-0.15f * lheii / 2.0f));
    c.a_heii = 1.26e-14f * fpow(lhei, 0.750f) + diel;
    c.a_heiii = 2.0f * 2.753e-14f * fpow(lheii, 1.5f) / fpow(1.0f + fpow(lheii / 2.740f, 0.407f), 2.242f);
    c.k_hi = 21.11f * t15 * fexp(-lhi / 2.0f) * fpow(lhi, -1.089f) / fpow(1.0f + fpow(lhi / 0.354f, 0.874f), 1.101f);
    c.k_hei = 32.38f * t15 * fexp(-lhei / 2.0f) * fpow(lhei, -1.146f) / fpow(1.0f + fpow(lhei / 0.416f, 0.987f), 1.056f);
    c.k_heii = 19.95f * t15 * fexp(-lheii / 2.0f) * fpow(lheii, -1.089f) / fpow(1.0f + fpow(lheii / 0.553f, 0.735f), 1.275f);
    return c;
}

// Cooling per volume [erg cm^-3 s^-1]: recombination, collisional ionisation,
// collisional excitation, bremsstrahlung. Rate coefficients in FP32, products in FP64.
__device__ __forceinline__ double cooling(float T, const Coef& k, double ne, double nhi, double nhii, double nhei,
                                          double nheii, double nheiii, int collisional)
{
    const float lhi = 2.0f * kTHI / T, lhei = 2.0f * kTHeI / T, lheii = 2.0f * kTHeII / T;
    const float rec_hii = 3.435e-30f * T * fpow(lhi, 1.970f) / fpow(1.0f + fpow(lhi / 2.250f, 0.376f), 3.720f);
    const float rec_heii = 1.380649e-16f * T * 1.26e-14f * fpow(lhei, 0.750f);
    const float rec_heiii = 8.0f * 3.435e-30f * T * fpow(lheii, 1.970f) / fpow(1.0f + fpow(lheii / 2.250f, 0.376f), 3.720f);
    const float diel = 1.90e-3f * fpow(T, -1.5f) * fexp(-0.75f * lheii / 2.0f) * (1.0f + 0.3f * fexp(-0.15f * lheii / 2.0f));
    const double diel_cool = 0.75 * 54.418 * kEV * (double)diel;
    double lam = ne * ((double)rec_hii * nhii + (double)rec_heii * nheii + (double)rec_heiii * nheiii + diel_cool * nheii);
    if (collisional)
        lam += ne * (13.598 * kEV * (double)k.k_hi * nhi + 24.587 * kEV * (double)k.k_hei * nhei +
                     54.418 * kEV * (double)k.k_heii * nheii);
    const float damp = 1.0f + sqrtf(T / 1e5f);
    lam += ne * nhi * (double)(7.5e-19f * fexp(-0.75f * lhi / 2.0f) / damp);
    lam += ne * nheii * (double)(5.54e-17f * fpow(T, -0.397f) * fexp(-0.75f * lheii / 2.0f) / damp);
    const float lt = log10f(T);
    const float gff = 1.1f + 0.34f * fexp(-(5.5f - lt) * (5.5f - lt) / 3.0f);
    lam += (double)(1.42e-27f * gff * sqrtf(T)) * (nhii + nheii + 4.0 * nheiii) * ne;
    return lam;
}

}  // namespace chem

}  // namespace arc
