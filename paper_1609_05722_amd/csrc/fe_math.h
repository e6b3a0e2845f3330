// Pointwise arithmetic of the denoiser, shared by the FP32 kernels.
#pragma once

#include <hip/hip_runtime.h>

#define FE_DATA_QUADRATIC_ 1
#define FE_DATA_IDIV_ 2

namespace fe {

// eq. 2.3
__device__ __forceinline__ float anscombe(float y) { return 2.0f * sqrtf(y + 0.375f); }

// Explicit part of the iPiano step (eq. 2.8): u - tau g + gamma (u - u_prev).
__device__ __forceinline__ float inertial_step(float u, float u_prev, float g,
                                               float tau, float gamma)
{
    return fmaf(-tau, g, u) + gamma * (u - u_prev);
}

// Proximal map of tau G (eq. 2.9).  tl = tau * lambda, q1 = 1 / (1 + tl).
//  quadratic (eq. 3.5):   (u~ + tl v) / (1 + tl)
//  I-divergence (eq. 3.3 with y -> v, eq. 3.6):
//     (a + sqrt(a^2 + 4 tl v)) / 2,  a = u~ - tl;
//  for a < 0 the algebraically equal 2 tl v / (sqrt(a^2 + 4 tl v) - a)
//  avoids the cancellation of a + sqrt(...).
// The hardware square root and reciprocal (about 1 ulp each) stand in for
// the correctly rounded sequences.
__device__ __forceinline__ float prox_fast(float ut, float v, float tl, float q1, int data_term)
{
    if (data_term == FE_DATA_QUADRATIC_) return fmaf(tl, v, ut) * q1;
    const float a = ut - tl;
    const float s = __builtin_amdgcn_sqrtf(fmaf(a, a, 4.0f * tl * v));
    return a >= 0.0f ? 0.5f * (a + s) : (2.0f * tl * v) * __builtin_amdgcn_rcpf(s - a);
}

// eq. 2.3 with the hardware square root (about 1 ulp).
__device__ __forceinline__ float anscombe_fast(float y)
{
    return 2.0f * __builtin_amdgcn_sqrtf(y + 0.375f);
}

// Student-t potential rho(z) = log(1 + z^2) (eq. 2.6).  With x = z^2:
// below 1/16 the series x - x^2/2 + ... + x^5/5 - x^6/6 (truncation below
// x^7/7, a relative 1e-8), so that small responses keep their relative
// accuracy; above, ln 2 * log2(1 + x) on the hardware logarithm, whose
// result is then at least 0.087 and whose rounding of 1 + x costs at most
// 2^-24 relative.  Branch-free.
__device__ __forceinline__ float student_t_rho(float z)
{
    const float x = z * z;
    float s = fmaf(x, -1.0f / 6.0f, 0.2f);
    s = fmaf(x, s, -0.25f);
    s = fmaf(x, s, 1.0f / 3.0f);
    s = fmaf(x, s, -0.5f);
    s = fmaf(x, s, 1.0f);
    const float series = x * s;
    const float lg = 0.693147181f * __builtin_amdgcn_logf(1.0f + x);
    return x < 0.0625f ? series : lg;
}

// Data-term energy per pixel without the lambda factor:
//  quadratic 1/2 (u - v)^2; I-divergence u - v log u (+inf for u <= 0).
__device__ __forceinline__ float data_energy(float u, float v, int data_term)
{
    if (data_term == FE_DATA_QUADRATIC_) {
        const float d = u - v;
        return 0.5f * d * d;
    }
    return u > 0.0f ? u - v * logf(u) : __builtin_inff();
}

// Gradient of the data term without the lambda factor, with the hardware
// reciprocal (about 1 ulp) for the I-divergence's v / u.
__device__ __forceinline__ float data_gradient_fast(float u, float v, int data_term)
{
    return data_term == FE_DATA_QUADRATIC_ ? u - v : fmaf(-v, __builtin_amdgcn_rcpf(u), 1.0f);
}

// Gradient of the data term without the lambda factor.
__device__ __forceinline__ float data_gradient(float u, float v, int data_term)
{
    return data_term == FE_DATA_QUADRATIC_ ? u - v : 1.0f - v / u;
}

}  // namespace fe
