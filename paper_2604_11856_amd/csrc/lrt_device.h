// Device helpers shared by the accumulation and march translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lrt_internal.h"

namespace lrt {

constexpr double kLog2e = 1.4426950408889634;
// XCDs of the chip: workgroup ids go round-robin over them, each has its own L2.
constexpr int kXCDs = 8;

__device__ __forceinline__ int32_t uniform_i(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Blackbody intensity B(nu, T) in W cm^-2 sr^-1 per cm^-1 (CGS x 1e-7).
static __device__ __forceinline__ double planck_f64(double nu, double T)
{
    return 1e-7 * 2.0 * kPlanck * kLight * kLight * nu * nu * nu / expm1(kC2 * nu / T);
}

// F(t) = (1 - e^-t)/t from e = e^-t; Taylor for |t| < 0.1 avoids the
// cancellation in 1 - e (relative error of the direct form ~ 6e-8 / |t|).
static __device__ __forceinline__ float fexp_f32(float t, float e)
{
    const float poly = fmaf(t, fmaf(t, fmaf(t, fmaf(t, fmaf(t, -1.0f / 720.0f, 1.0f / 120.0f),
                                                   -1.0f / 24.0f), 1.0f / 6.0f), -0.5f), 1.0f);
    const float direct = (1.0f - e) * __builtin_amdgcn_rcpf(t);
    return fabsf(t) < 0.1f ? poly : direct;
}

// One cell-constant segment on scaled single-precision coefficients:
// tau = kappa ds; returns e^-tau (as the attenuation factor) and the emitted
// term eta ds F(tau) in double precision.  dsk = ds 2^esk (as float),
// dse = ds 2^ese.
static __device__ __forceinline__ void segment_f32(float eta_s, float kap_s, float dsk, double dse,
                                            double &atten, double &emit)
{
    const float tau = kap_s * dsk;
    const float e = __builtin_amdgcn_exp2f(tau * (float)(-kLog2e));
    const float F = fexp_f32(tau, e);
    atten = (double)e;
    emit = (double)(eta_s * F) * dse;
}

// Weights per unit length of the two nodes of a linear-j segment (Sec. 2.2.3:
// kappa from the far node, j linear between the nodes) at optical thickness
// t with e = e^-t: W_near = (1 - f)/t, W_far = (f - e)/t, f = (1 - e)/t, which
// integrate the transfer equation over the segment.  (The pairing follows the
// scheme's derivation; as t grows only the node next to the target counts.)
// For |t| < 0.1 both differences cancel; there the weights come from their
// Taylor series, W_near = sum (-t)^n/(n+2)!, W_far = sum (-1)^n (n+1) t^n/(n+2)!,
// whose first omitted terms are below 3e-11.
static __device__ __forceinline__ void linear_j_weights_f32(float t, float e, float &wf, float &wn)
{
    const float sn = fmaf(t, fmaf(t, fmaf(t, fmaf(t, fmaf(t, -1.0f / 5040.0f, 1.0f / 720.0f),
                                                   -1.0f / 120.0f), 1.0f / 24.0f), -1.0f / 6.0f), 0.5f);
    const float sf = fmaf(t, fmaf(t, fmaf(t, fmaf(t, fmaf(t, -1.0f / 840.0f, 1.0f / 144.0f),
                                                   -1.0f / 30.0f), 1.0f / 8.0f), -1.0f / 3.0f), 0.5f);
    const float r = __builtin_amdgcn_rcpf(t);
    const float f = (1.0f - e) * r;
    const bool thin = fabsf(t) < 0.1f;
    wn = thin ? sn : (1.0f - f) * r;
    wf = thin ? sf : (f - e) * r;
}

}  // namespace lrt
