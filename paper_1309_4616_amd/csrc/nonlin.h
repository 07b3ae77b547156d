// Pointwise nonlinearities g of u' = A u + g(u) (device code).
//
//   EXPI_G_CUBIC           g(u) = u - u^3 (the reaction-diffusion workload)
//   EXPI_G_COMBUSTION      g(u) = (2 - u)/4 exp(20 (1 - 1/u)), the combustion
//                          model of Sec. III-C, eq. (4)-(5), in the precision
//                          of the evaluation type: IEEE division and the
//                          library exp of that type
//   EXPI_G_COMBUSTION_FAST the same with the hardware approximations of
//                          Table III's "fast math" column: the reciprocal and
//                          the exponential are the FP32 hardware instructions
//                          (v_rcp_f32, 1 ulp; v_exp_f32, base 2), the factor
//                          (2 - u)/4 stays in the evaluation type (relative
//                          error about 1e-6 over u in [0.5, 2])
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/expi.h"

namespace expi {

// 20 / ln 2: exp(20 q) = 2^(q * 20/ln 2)
constexpr float kTwentyOverLn2 = 28.853900817779268f;

__device__ __forceinline__ double g_combustion(double u) {
    return 0.25 * (2.0 - u) * exp(20.0 * (1.0 - 1.0 / u));
}
__device__ __forceinline__ float g_combustion(float u) {
    return 0.25f * (2.0f - u) * expf(20.0f * (1.0f - 1.0f / u));
}
// exp(20 (1 - 1/u)) from the FP32 hardware reciprocal and base-2 exponential
__device__ __forceinline__ float combustion_exp_fast(float u) {
    const float q = 1.0f - __builtin_amdgcn_rcpf(u);
    return __builtin_amdgcn_exp2f(kTwentyOverLn2 * q);
}

// g of `kind` (uniform over the launch) at u, in T.
template <class T>
__device__ __forceinline__ T g_eval(int kind, T u) {
    if (kind == EXPI_G_COMBUSTION) return g_combustion(u);
    if (kind == EXPI_G_COMBUSTION_FAST) return (T)0.25 * ((T)2 - u) * (T)combustion_exp_fast((float)u);
    return u - u * u * u;
}

}  // namespace expi
