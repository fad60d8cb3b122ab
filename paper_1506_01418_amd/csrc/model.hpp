// The Tweedie likelihood's gradient factor on the device (Section 4):
//   d/dmu log TW(v; mu, phi, beta) = (v - mu) mu^(beta-2) / phi,
// with the mean floored at mu_floor when beta < 2.  mu^(beta-2) uses the
// hardware reciprocal / reciprocal square root (1 ulp) for the common
// powers, and the hardware exp2/log2 otherwise.
#pragma once
#include <hip/hip_runtime.h>

namespace psgld {

enum Lik : int { LIK_GAUSS = 0, LIK_POISSON = 1, LIK_HALF = 2, LIK_GAMMA = 3, LIK_GENERAL = 4 };

inline int lik_kind_of(double beta)
{
    if (beta == 2.0) return LIK_GAUSS;
    if (beta == 1.0) return LIK_POISSON;
    if (beta == 0.5) return LIK_HALF;
    if (beta == 0.0) return LIK_GAMMA;
    return LIK_GENERAL;
}

template <int LIK>
__device__ __forceinline__ float tweedie_residual(float v, float mu, float inv_phi, float beta, float mu_floor)
{
    if constexpr (LIK == LIK_GAUSS) {
        return (v - mu) * inv_phi;
    } else {
        const float m = fmaxf(mu, mu_floor);
        float w;
        if constexpr (LIK == LIK_POISSON) {
            w = __builtin_amdgcn_rcpf(m);                 // m^-1
        } else if constexpr (LIK == LIK_HALF) {
            const float r = __builtin_amdgcn_rsqf(m);     // m^-1.5
            w = r * r * r;
        } else if constexpr (LIK == LIK_GAMMA) {
            const float r = __builtin_amdgcn_rcpf(m);     // m^-2
            w = r * r;
        } else {
            w = __builtin_amdgcn_exp2f((beta - 2.0f) * __builtin_amdgcn_logf(m));
        }
        return (v - m) * w * inv_phi;
    }
}

}  // namespace psgld
