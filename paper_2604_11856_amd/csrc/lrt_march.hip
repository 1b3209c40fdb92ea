// gfx950 kernels of the ray march (arXiv 2604.11856, Sec. 2.2.3): per (ray,
// spectral chunk) the RTE march far -> target with the spectral trapezoid
// fused in, in the cell-constant or the linear-j segment scheme, and the
// deterministic sums of per-block partials and of ray fluxes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "lrt_device.h"
#include "lrt_internal.h"

namespace lrt {

namespace {

__device__ __forceinline__ void linear_j_weights_f64(double t, double &e, double &wf, double &wn)
{
    e = exp(-t);
    if (fabs(t) >= 0.05) {
        const double f = -expm1(-t) / t;
        wn = (1.0 - f) / t;
        wf = (f - e) / t;
        return;
    }
    // Horner over n = 17..0 of c_n t^n with c_n = (-1)^n/(n+2)! and (n+1) c_n
    double inv_fact[18];
    double fct = 2.0;
    for (int n = 0; n < 18; ++n) {
        inv_fact[n] = 1.0 / fct;
        fct *= (double)(n + 3);
    }
    double a = 0.0, b = 0.0;
    for (int n = 17; n >= 0; --n) {
        const double c = (n & 1) ? -inv_fact[n] : inv_fact[n];
        a = fma(a, t, c);
        b = fma(b, t, (double)(n + 1) * c);
    }
    wn = a;
    wf = b;
}

// One row (the PPT consecutive points kb.. of a lane) of eta and kappa, from
// the row bases of the segment's cell (the same for the whole wave, so the
// loads take a scalar base and the lane's 32-bit byte offset ob = kb sizeof(T)).
template <int PPT, typename T>
__device__ __forceinline__ void load_row(const T *erow, const T *krow, uint32_t kb, uint32_t ob, int32_t n_band,
                                         bool vec, T (&ev)[PPT], T (&kv)[PPT])
{
    if constexpr (sizeof(T) == 4) {
        if (vec) {   // one vector load per array and lane
            typedef float VecF __attribute__((ext_vector_type(PPT)));
            const VecF a = *(const VecF *)((const char *)erow + ob);
            const VecF b = *(const VecF *)((const char *)krow + ob);
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                ev[j] = a[j];
                kv[j] = b[j];
            }
            return;
        }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const bool ok = (int32_t)kb + j < n_band;
        ev[j] = ok ? erow[kb + j] : (T)0;
        kv[j] = ok ? krow[kb + j] : (T)0;
    }
}

// March of one (ray, chunk of 64 x PPT points), far -> target.
//   LINEAR = false: cell-constant segments, I <- I e^-tau + eta ds F(tau).
//   LINEAR = true: linear-j segments between LOS nodes at the far end of the
//     ray, the midpoint of every cell segment and the target; a node takes its
//     cell's state, so the node spacings are ds_0/2, (ds_m-1 + ds_m)/2, ...,
//     ds_M-1/2, and each segment uses the far node's kappa.
// T_far (NULL: all free) gives per ray the temperature of a solid far
// boundary (0: free), whose blackbody intensity starts the march.
// The (ray, chunk) of wave `wave` of workgroup b (b: index in the whole grid,
// launch offset b0 + blockIdx.x): the workgroup owns RAYS rays x (4 / RAYS)
// consecutive chunks, one (ray, chunk) per wave.  Workgroups go round-robin to
// the 8 XCDs (b % 8), each with its own L2.  With one ray per workgroup (few
// segments per cell) XCD x takes a contiguous range of the chunk-major items,
// so every ray of a spectral chunk runs on one XCD and the rows the rays share
// come from that XCD's L2.  With four rays per workgroup (many segments per
// cell) the items are taken in their own chunk-major order, so all XCDs work on
// the same chunk and its rows, read by every XCD, stay in the chip-wide last-
// level cache (measured on 131,072 rays over 131,072 cells: 544 against 560 ms
// per step; on the stagnation line and the 256 x 128 case, with one ray per
// workgroup, that order took 12.7 against 7.8 ms and 97.8 against 82.9 ms per
// launch).  When every wall point has
// the same rays (per_wall > 0) a chunk's rays are taken direction-major: the
// rays an XCD runs together are then nearly parallel lines from neighbouring
// wall points, which cross nearly the same cells.  (Measured against
// ray-fastest items with a contiguous ray range per XCD: 8.6 vs 11.2 ms on the
// 17 slab rays of the stagnation line, 100.6 vs 107.5 ms on 8192 axisymmetric
// rays.)  A bijection onto [0, n_rays) x [0, n_chunks) for any sizes (ray = -1
// for the waves past the last ray or chunk).
template <int RAYS>
__device__ __forceinline__ void march_item(uint32_t b, int32_t wave, const DevRays &rays, int32_t n_chunks,
                                           int &ray, int &chunk)
{
    constexpr int CHUNKS = kMarchThreads / 64 / RAYS;
    const uint32_t n_groups = ((uint32_t)rays.n_rays + RAYS - 1) / RAYS;
    const uint32_t n_cgroups = ((uint32_t)n_chunks + CHUNKS - 1) / CHUNKS;
    const uint32_t n = n_groups * n_cgroups, x = b % kXCDs, i = b / kXCDs;
    const uint32_t per = n / kXCDs, rem = n % kXCDs;
    const uint32_t gi = RAYS > 1 ? b : x * per + min(x, rem) + i;
    chunk = (int)(gi / n_groups) * CHUNKS + wave / RAYS;
    const int32_t q = (int32_t)(gi % n_groups) * RAYS + wave % RAYS;
    if (q >= rays.n_rays || chunk >= n_chunks) {
        ray = -1;   // past the last ray or chunk: this wave has nothing to do
    } else if (rays.per_wall > 0) {
        const int32_t n_wall = rays.n_rays / rays.per_wall;
        ray = (q % n_wall) * rays.per_wall + q / n_wall;   // direction-major
    } else {
        ray = q;
    }
}

template <bool FP32, bool LINEAR, int PPT, int RAYS>
__global__ __launch_bounds__(kMarchThreads) void march_kernel(
    DevRays rays, DevGrid g, int32_t k_first, int32_t n_band, const void *eta_v,
    const void *kappa_v, const int32_t *escale, const double *T_far, double *I_out,
    double *partials, int32_t n_chunks, int32_t aligned16, uint32_t b0)
{
    const int lane = threadIdx.x & 63, wave = uniform_i(threadIdx.x >> 6);
    int ray, chunk;
    march_item<RAYS>(b0 + blockIdx.x, wave, rays, n_chunks, ray, chunk);
    if (ray < 0) return;
    const int32_t kb = chunk * (64 * PPT) + lane * PPT;   // band-relative
    const int64_t m0 = rays.off[ray], m1 = rays.off[ray + 1];
    double I[PPT];
    const double Tw = T_far ? T_far[ray] : 0.0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        I[j] = 0.0;
        if (Tw > 0.0 && kb + j < n_band) I[j] = planck_f64(g.nu_min + (double)(k_first + kb + j) * g.h, Tw);
    }
    // vector loads only when every row start is aligned to PPT floats
    // (16-byte aligned bases, n_band a multiple of PPT) and the wave's
    // points are all inside the band (a wave-uniform choice)
    const bool vec = aligned16 && (int64_t)(chunk + 1) * (64 * PPT) <= n_band && (n_band % PPT) == 0;
    using T = std::conditional_t<FP32, float, double>;
    const T *eta = (const T *)eta_v;
    const T *kap = (const T *)kappa_v;
    const uint32_t ob = (uint32_t)kb * (uint32_t)sizeof(T);   // byte offset of the lane's points in a row

    if constexpr (!LINEAR) {
        // the segment loop, with vector or guarded row loads chosen once
        // outside it; a 32-bit trip count keeps the loop test on the scalar unit
        const int32_t *cell_m = rays.cell + m0;
        const double *ds_m = rays.ds + m0;
        const int32_t n_seg = (int32_t)(m1 - m0);
        auto cell_march = [&](auto vec_c) {
#pragma unroll 2
            for (int32_t i = 0; i < n_seg; ++i) {
                const int32_t c = cell_m[i];
                const double ds = ds_m[i];
                const int64_t row = (int64_t)c * n_band;
                T ev[PPT], kv[PPT];
                load_row<PPT, T>(eta + row, kap + row, (uint32_t)kb, ob, n_band, decltype(vec_c)::value, ev, kv);
                if constexpr (FP32) {
                    float dsu;
                    double dsl;
                    segment_scales(ds, escale[2 * c + 0], escale[2 * c + 1], dsu, dsl);
#pragma unroll
                    for (int j = 0; j < PPT; ++j) {
                        double at, em;
                        segment_f32(ev[j], kv[j], dsu, dsl, at, em);
                        I[j] = fma(I[j], at, em);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < PPT; ++j) {
                        if (kb + j < n_band) {
                            const double tau = kv[j] * ds;
                            const double em = expm1(-tau);
                            const double F = (tau == 0.0) ? 1.0 : -em / tau;
                            I[j] = I[j] * (1.0 + em) + ev[j] * ds * F;
                        }
                    }
                }
            }
        };
        if (vec)
            cell_march(std::true_type{});
        else
            cell_march(std::false_type{});
    } else {
        // previous node (the far node of the next segment)
        T pe[PPT], pk[PPT];
        int32_t pee = 0, pek = 0;
        double pds = 0.0;
        // one linear-j segment of length L from node (fe, fk) to node (ne_)
        auto segment = [&](const T (&fe)[PPT], const T (&fk)[PPT], int32_t fee,
                           int32_t fek, const T (&ne_)[PPT], int32_t nee, double L) {
            if constexpr (FP32) {
                const double Lf = ldexp(L, fee), Ln = ldexp(L, nee);
                const float Lk = (float)fmin(ldexp(L, fek), 3.0e38);
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    const float t = fk[j] * Lk;
                    const float e = __builtin_amdgcn_exp2f(t * (float)(-kLog2e));
                    float wf, wn;
                    linear_j_weights_f32(t, e, wf, wn);
                    I[j] = fma(I[j], (double)e, (double)(wf * fe[j]) * Lf + (double)(wn * ne_[j]) * Ln);
                }
            } else {
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    if (kb + j < n_band) {
                        double e, wf, wn;
                        linear_j_weights_f64(fk[j] * L, e, wf, wn);
                        I[j] = I[j] * e + L * (wf * fe[j] + wn * ne_[j]);
                    }
                }
            }
        };
        for (int64_t m = m0; m < m1; ++m) {
            const int32_t c = rays.cell[m];
            const double ds = rays.ds[m];
            T ev[PPT], kv[PPT];
            load_row<PPT, T>(eta + (int64_t)c * n_band, kap + (int64_t)c * n_band, (uint32_t)kb, ob, n_band, vec,
                             ev, kv);
            const int32_t ee = FP32 ? escale[2 * c + 0] : 0, ek = FP32 ? escale[2 * c + 1] : 0;
            if (m == m0)
                segment(ev, kv, ee, ek, ev, ee, 0.5 * ds);             // far end -> first midpoint
            else
                segment(pe, pk, pee, pek, ev, ee, 0.5 * (pds + ds));   // midpoint -> midpoint
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                pe[j] = ev[j];
                pk[j] = kv[j];
            }
            pee = ee;
            pek = ek;
            pds = ds;
        }
        if (m1 > m0) segment(pe, pk, pee, pek, pe, pee, 0.5 * pds);     // last midpoint -> target
    }
    // outputs: I and the trapezoid partial with global-index weights
    double part = 0.0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int32_t kl = kb + j;
        if (kl < n_band) {
            const int32_t kg = k_first + kl;
            const double w = (kg == 0 || kg == g.n_points - 1) ? 0.5 * g.h : g.h;
            part += w * I[j];
            if (I_out) I_out[(int64_t)ray * n_band + kl] = I[j];
        }
    }
    // the wave's sum in a fixed order (xor-shuffles)
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (lane == 0) partials[(int64_t)ray * n_chunks + chunk] = part;
}

__global__ void reduce_rows_kernel(const double *p, int32_t n_rows, int32_t n_cols, double *out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    double s = 0.0;
    for (int j = 0; j < n_cols; ++j) s += p[(int64_t)r * n_cols + j];
    out[r] = s;
}

__global__ void wall_sum_kernel(const double *I_int, const double *weight, const int64_t *wall_off,
                                int32_t n_wall, double *q)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_wall) return;
    double s = 0.0;
    for (int64_t r = wall_off[w]; r < wall_off[w + 1]; ++r) s += weight[r] * I_int[r];
    q[w] = s;
}

__global__ void add_kernel(double *acc, const double *x, int32_t n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) acc[t] += x[t];
}

}  // namespace

hipError_t launch_march(bool fp32, bool linear, int32_t ppt, const DevRays &rays, const DevGrid &g,
                        int32_t k_first, int32_t n_band, const void *eta, const void *kappa,
                        const int32_t *escale, const double *T_far, double *I_out,
                        double *partials, int32_t n_chunks, hipStream_t st)
{
    if (rays.n_rays == 0) return hipSuccess;
    if (ppt != 2 && ppt != 4) return hipErrorInvalidValue;
    // 128-point chunks: 4 rays per workgroup; 256-point chunks: 4 chunks of one ray
    const int64_t waves = kMarchThreads / 64, n_rays = rays.n_rays;
    const int64_t n_blocks = ppt == 2 ? (n_rays + waves - 1) / waves * n_chunks
                                      : n_rays * ((n_chunks + waves - 1) / waves);
    if (n_blocks > (int64_t)UINT32_MAX) return hipErrorInvalidConfiguration;
    const int32_t al = ((((uintptr_t)eta) | ((uintptr_t)kappa)) & 15) == 0;
    for (int64_t b0 = 0; b0 < n_blocks; b0 += kMaxLaunchBlocks) {
        const dim3 grid((unsigned)std::min(kMaxLaunchBlocks, n_blocks - b0));
#define LRT_MARCH(F, LIN, P, R)                                                                          \
    hipLaunchKernelGGL((march_kernel<F, LIN, P, R>), grid, dim3(kMarchThreads), 0, st, rays, g, k_first, \
                       n_band, eta, kappa, escale, T_far, I_out, partials, n_chunks, al, (uint32_t)b0)
#define LRT_MARCH_P(F, LIN) \
    if (ppt == 2) LRT_MARCH(F, LIN, 2, 4); else LRT_MARCH(F, LIN, 4, 1)
        if (fp32) {
            if (linear) LRT_MARCH_P(true, true); else LRT_MARCH_P(true, false);
        } else {
            if (linear) LRT_MARCH_P(false, true); else LRT_MARCH_P(false, false);
        }
#undef LRT_MARCH_P
#undef LRT_MARCH
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_reduce_rows(const double *partials, int32_t n_rows, int32_t n_cols, double *out,
                              hipStream_t st)
{
    if (n_rows == 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(blocks_for(n_rows, 64)), dim3(64), 0, st, partials,
                       n_rows, n_cols, out);
    return hipGetLastError();
}

hipError_t launch_wall_sum(const double *I_int, const double *weight, const int64_t *wall_off,
                           int32_t n_wall, double *q, hipStream_t st)
{
    if (n_wall == 0) return hipSuccess;
    hipLaunchKernelGGL(wall_sum_kernel, dim3(blocks_for(n_wall, 64)), dim3(64), 0, st, I_int,
                       weight, wall_off, n_wall, q);
    return hipGetLastError();
}

hipError_t launch_add(double *acc, const double *x, int32_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(add_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, acc, x, n);
    return hipGetLastError();
}

}  // namespace lrt
