// Device helpers shared by the accumulation and march translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lrt_internal.h"

namespace lrt {

constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;
// XCDs of the chip: workgroup ids go round-robin over them, each has its own L2.
constexpr int kXCDs = 8;

__device__ __forceinline__ int32_t uniform_i(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Blackbody intensity B(nu, T) in W cm^-2 sr^-1 per cm^-1 (CGS x 1e-7).
static __device__ __forceinline__ double planck_f64(double nu, double T)
{
    return 1e-7 * 2.0 * kPlanck * kLight * kLight * nu * nu * nu / expm1(kC2 * nu / T);
}

// F(t) = (1 - e^-t)/t of a segment, evaluated as H = F ln2 in u = t log2(e)
// (so e^-t = 2^-u is one hardware exponential, and the caller's emission
// factor carries the 1/ln2): the direct form (1 - e)/u, or for |t| < 0.1,
// where 1 - e cancels (relative error ~6e-8/|t|), the Taylor series
// F = sum_n (-t)^n/(n+1)! through t^4 (first omitted term below 1.4e-8
// relative) rewritten in u: H = sum_n (-1)^n ln2^(n+1) u^n/(n+1)!.
static __device__ __forceinline__ float fexp_u_f32(float u, float e)
{
    constexpr double l = kLn2, l2 = l * l, l3 = l2 * l;
    const float poly = fmaf(u, fmaf(u, fmaf(u, fmaf(u, (float)(l3 * l2 / 120.0), (float)(-l2 * l2 / 24.0)),
                                            (float)(l3 / 6.0)), (float)(-l2 / 2.0)), (float)l);
    const float direct = (1.0f - e) * __builtin_amdgcn_rcpf(u);
    return fabsf(u) < (float)(0.1 * kLog2e) ? poly : direct;
}

// One cell-constant segment on scaled single-precision coefficients:
// tau = kappa ds; returns e^-tau (as the attenuation factor) and the emitted
// term eta ds F(tau) in double precision.  dsu = ds log2(e) 2^esk (as float,
// so u = kappa dsu = tau log2(e)), dsl = ds log2(e) 2^ese.
static __device__ __forceinline__ void segment_f32(float eta_s, float kap_s, float dsu, double dsl,
                                            double &atten, double &emit)
{
    const float u = kap_s * dsu;
    const float e = __builtin_amdgcn_exp2f(-u);
    const float H = fexp_u_f32(u, e);
    atten = (double)e;
    emit = (double)(eta_s * H) * dsl;
}

// The per-segment factors of segment_f32 from ds and the cell's scales (dsu
// clamped below float overflow, so that kappa = 0 gives u = 0).
static __device__ __forceinline__ void segment_scales(double ds, int32_t ese, int32_t esk, float &dsu,
                                               double &dsl)
{
    const double d = ds * kLog2e;
    dsu = (float)fmin(ldexp(d, esk), 3.0e38);
    dsl = ldexp(d, ese);
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
