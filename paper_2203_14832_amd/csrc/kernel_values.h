// Kernel values K(r) of the apply passes, shared by the single- and
// multi-column kernels.  1/r and log r vanish at r = 0 in the near field; the
// Gaussian and exp(-r/h) are 1 there.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "nnca.h"

namespace nnca {
// Internal kind of the length-scale derivative of the Gaussian:
// D(r) = (r^2/h^2) exp(-r^2/h^2), so that dK/dh = (2/h) D(r).  It runs
// through the same interaction kernels as K; it is zero at r = 0.
constexpr int K_GAUSS_DH = 103;

// The parameter `prm` of the apply kernels, from the kernel's length scale:
// the Gaussian 1/h^2 (FP64) or log2(e)/h^2 (FP32), exp(-r/h) 1/h (FP64) or
// log2(e)/h (FP32), the regularised 1/r its a, the regularised log r
// 1/log(a^2); unused by the others.
inline double kernel_prm64(int kind, double hp)
{
    if (kind == NNCA_K_GAUSS || kind == K_GAUSS_DH) return 1.0 / (hp * hp);
    if (kind == NNCA_K_EXP_R) return 1.0 / hp;
    if (kind == NNCA_K_INV_REG) return hp;
    if (kind == NNCA_K_LOG_REG) return 1.0 / std::log(hp * hp);
    return 0.0;
}
inline float kernel_prm32(int kind, double hp)
{
    if (kind == NNCA_K_GAUSS || kind == K_GAUSS_DH) return (float)(1.4426950408889634 / (hp * hp));
    if (kind == NNCA_K_EXP_R) return (float)(1.4426950408889634 / hp);
    return (float)kernel_prm64(kind, hp);
}

template <int KIND>
__device__ inline float kv32(float d2, float prm)
{
    if (KIND == NNCA_K_INV_R) return __builtin_amdgcn_rsqf(d2);
    if (KIND == NNCA_K_LOG_R) return 0.5f * logf(d2);
    if (KIND == NNCA_K_INV_REG) {   // prm = a
        const float rs = __builtin_amdgcn_rsqf(d2);
        return d2 >= prm * prm ? prm * rs : (d2 * rs) / prm;
    }
    if (KIND == NNCA_K_LOG_REG) {   // prm = 1 / log(a^2)
        const float l = logf(d2), t = 1.0f / prm;
        if (l >= t) return l * prm;
        const float r = sqrtf(d2), a = expf(0.5f * t);
        return (r * (0.5f * l - 1.0f)) / (a * (0.5f * t - 1.0f));
    }
    if (KIND == NNCA_K_EXP_R) return __builtin_amdgcn_exp2f(-sqrtf(d2) * prm);   // prm = log2(e) / h
    if (KIND == K_GAUSS_DH) {
        float t = d2 * prm;   // log2(e) r^2 / h^2
        return (t * 0.693147180559945309f) * __builtin_amdgcn_exp2f(-t);
    }
    return __builtin_amdgcn_exp2f(-d2 * prm);  // prm = log2(e) / h^2
}
template <int KIND>
__device__ inline double kv64(double d2, double prm)
{
    if (KIND == NNCA_K_INV_R) return 1.0 / sqrt(d2);
    if (KIND == NNCA_K_LOG_R) return 0.5 * log(d2);
    if (KIND == NNCA_K_INV_REG) return d2 >= prm * prm ? prm / sqrt(d2) : sqrt(d2) / prm;   // prm = a
    if (KIND == NNCA_K_LOG_REG) {   // prm = 1 / log(a^2)
        const double l = log(d2), t = 1.0 / prm;
        if (l >= t) return l * prm;
        const double r = sqrt(d2), a = exp(0.5 * t);
        return (r * (0.5 * l - 1.0)) / (a * (0.5 * t - 1.0));
    }
    if (KIND == NNCA_K_EXP_R) return exp(-sqrt(d2) * prm);   // prm = 1 / h
    if (KIND == K_GAUSS_DH) {
        double t = d2 * prm;  // r^2 / h^2
        return t * exp(-t);
    }
    return exp(-d2 * prm);  // prm = 1 / h^2
}
template <int KIND, typename T>
__device__ inline T kv(T d2, T prm)
{
    if constexpr (sizeof(T) == 4) return kv32<KIND>(d2, prm);
    else return kv64<KIND>(d2, prm);
}
// near field: 1/r and log r vanish at r = 0, the Gaussian and exp(-r/h) are 1 there
template <int KIND, typename T>
__device__ inline T kv_self(T d2, T prm)
{
    T v = kv<KIND, T>(d2, prm);
    if (KIND == NNCA_K_GAUSS || KIND == NNCA_K_EXP_R) return v;
    return d2 > T(0) ? v : T(0);
}

// 1/r from an FP32 reciprocal-square-root seed and one FP64 Newton step
// (relative error ~1e-14); the other kernels in FP64.
template <int KIND, int MODE = 0>
__device__ inline double kv_refined(double d2, double prm)
{
    if (KIND == NNCA_K_INV_R) {
        double y = (double)__builtin_amdgcn_rsqf((float)d2);
        return y * (1.5 - 0.5 * d2 * y * y);
    }
    return kv64<KIND>(d2, prm);
}


}  // namespace nnca
