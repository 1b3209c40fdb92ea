// gfx950 generation of the rovibronic line list of diatomic band systems
// (arXiv 2604.11856, Sec. 2.2.2): per candidate (system, V_u, V_l,
// rotational index, branch) one thread forms the two state energies from the
// vibrational term, the rotational constants of its level and the rotational
// term of the coupling case, the line centre, the Hoenl-London factor of the
// branch and the molecular Einstein coefficient, in double precision.  Two
// passes give the lines in candidate order without atomics: the first counts
// the lines of each workgroup, the host scans the counts, the second writes
// every line at its rank.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/lrt.h"
#include "lrt_ctx.h"
#include "lrt_device.h"
#include "lrt_internal.h"

namespace lrt {

namespace {

constexpr int kGenThreads = 256;

struct DevBand {
    int32_t species, hund, lam_u, lam_l;
    int32_t nv_u, nv_l, J_max, slots;   // slots: candidates per (V_u, V_l) band
    int64_t cand0;                      // first candidate of the system
    int64_t re2_off;                    // its Re'^2 table in the concatenated array
    double Te_u, Te_l, g_u, g_l;
    double we_u, wexe_u, weye_u, Be_u, ae_u, De_u, be_u, gamma_u;
    double we_l, wexe_l, weye_l, Be_l, ae_l, De_l, be_l, gamma_l;
};

struct GenLine {
    double nu0, A, Eu_ev, Eu_rot, El_ev, El_rot, gu, gl;
    int32_t species;
};

// 64 pi^4 (e a0)^2 / (3 h) in CGS: e in statcoulomb (its exact SI value times
// c/10), a0 as the paper prints it, h exact.
constexpr double kEsu = 1.602176634e-19 * 2.99792458e10 / 10.0;
constexpr double kA0 = 5.291772083e-9;

__device__ __forceinline__ double vib_term(double we, double wexe, double weye, double x)
{
    return we * x - wexe * x * x + weye * x * x * x;
}

// Hoenl-London factor, Hund's case (a) table (by J_u; br 0 P, 1 Q, 2 R).
__device__ __forceinline__ double hl_case_a(int br, double J, int lu, int ll)
{
    const double L = (double)lu;
    if (lu == 0 && ll == 0) return br == 0 ? J + 1.0 : (br == 1 ? 0.0 : J);
    if (lu == ll) {
        if (br == 0) return (J + 1.0 + L) * (J + 1.0 - L) / (J + 1.0);
        if (br == 1) return (2.0 * J + 1.0) * L * L / (J * (J + 1.0));
        return (J + L) * (J - L) / J;
    }
    const double sg = (lu - ll == 1) ? 1.0 : -1.0;   // upper sign of the table for dLambda = +1
    if (br == 0) return (J + 1.0 - sg * L) * (J + 2.0 - sg * L) / (2.0 * (J + 1.0));
    if (br == 1) return (J + sg * L) * (J + 1.0 - sg * L) * (2.0 * J + 1.0) / (2.0 * J * (J + 1.0));
    return (J + sg * L) * (J - 1.0 + sg * L) / (2.0 * J);
}

// Hoenl-London factor, Hund's case (b) table (by J_l).
__device__ __forceinline__ double hl_case_b(int br, double J)
{
    if (br == 0) return (J * J - 0.25) / J;
    if (br == 1) return (2.0 * J + 1.0) / (4.0 * J * (J + 1.0));
    return ((J + 1.0) * (J + 1.0) - 0.25) / (J + 1.0);
}

// Candidate t of the whole list; false if it is not a line in [nu_lo, nu_hi].
__device__ bool gen_candidate(const DevBand *sys, int n_sys, const double *re2, int64_t t, double nu_lo,
                              double nu_hi, GenLine &o)
{
    int k = 0;
    while (k + 1 < n_sys && sys[k + 1].cand0 <= t) ++k;
    const DevBand &s = sys[k];
    const int64_t loc = t - s.cand0;
    const int64_t band = loc / s.slots;
    const int32_t r = (int32_t)(loc % s.slots);
    const int32_t vu = (int32_t)(band / s.nv_l), vl = (int32_t)(band % s.nv_l);
    const double xu = vu + 0.5, xl = vl + 0.5;
    const double Bu = s.Be_u - s.ae_u * xu, Du = s.De_u + s.be_u * xu;
    const double Bl = s.Be_l - s.ae_l * xl, Dl = s.De_l + s.be_l * xl;
    double Ju, Jl, S, Eur, Elr;
    int br;
    if (s.hund == LRT_HUND_A) {
        br = r % 3;
        Ju = (double)(r / 3);
        Jl = Ju + (br == 0 ? 1.0 : (br == 1 ? 0.0 : -1.0));
        if (Ju < s.lam_u || Jl < s.lam_l || Jl < 0.0) return false;
        S = hl_case_a(br, Ju, s.lam_u, s.lam_l);
        Eur = Bu * Ju * (Ju + 1.0) - Du * Ju * Ju * (Ju + 1.0) * (Ju + 1.0);
        Elr = Bl * Jl * (Jl + 1.0) - Dl * Jl * Jl * (Jl + 1.0) * (Jl + 1.0);
    } else {
        const int32_t q = r % 6;
        br = q % 3;
        const double Sl = q < 3 ? 0.5 : -0.5;
        const double Nl = (double)(r / 6);
        Jl = Nl + Sl;
        Ju = Jl + (br == 0 ? -1.0 : (br == 1 ? 0.0 : 1.0));
        const double Su = br == 1 ? -Sl : Sl;
        const double Nu = Ju - Su;
        if (Jl < 0.5 || Nu < 0.0 || Ju < 0.5) return false;
        S = hl_case_b(br, Jl);
        Eur = Bu * Nu * (Nu + 1.0) - Du * Nu * Nu * (Nu + 1.0) * (Nu + 1.0) + Su * s.gamma_u * (Nu + 0.5 - Su);
        Elr = Bl * Nl * (Nl + 1.0) - Dl * Nl * Nl * (Nl + 1.0) * (Nl + 1.0) + Sl * s.gamma_l * (Nl + 0.5 - Sl);
    }
    if (!(S > 0.0)) return false;
    const double Eue = s.Te_u + vib_term(s.we_u, s.wexe_u, s.weye_u, xu);
    const double Ele = s.Te_l + vib_term(s.we_l, s.wexe_l, s.weye_l, xl);
    const double nu = (Eue + Eur) - (Ele + Elr);
    if (!(nu >= nu_lo && nu <= nu_hi)) return false;
    constexpr double kPi4 = kPi * kPi * kPi * kPi;
    const double Re2 = re2[s.re2_off + (int64_t)vu * s.nv_l + vl];
    o.nu0 = nu;
    o.A = 64.0 * kPi4 * nu * nu * nu * (kEsu * kA0) * (kEsu * kA0) * Re2 * S / (3.0 * kPlanck * (2.0 * Ju + 1.0));
    o.Eu_ev = Eue;
    o.Eu_rot = Eur;
    o.El_ev = Ele;
    o.El_rot = Elr;
    o.gu = s.g_u * (2.0 * Ju + 1.0);
    o.gl = s.g_l * (2.0 * Jl + 1.0);
    o.species = s.species;
    return true;
}

// Rank of a valid candidate inside its workgroup (candidate order), and the
// workgroup's count (thread 0 of the result).
__device__ __forceinline__ int32_t block_rank(bool ok, int32_t *s_wave, int32_t &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t m = __ballot(ok);
    if (lane == 0) s_wave[wave] = __popcll(m);
    __syncthreads();
    int32_t before = 0;
    total = 0;
    for (int w = 0; w < kGenThreads / 64; ++w) {
        if (w < wave) before += s_wave[w];
        total += s_wave[w];
    }
    return before + __popcll(m & ((1ull << lane) - 1ull));
}

__global__ __launch_bounds__(kGenThreads) void gen_count_kernel(const DevBand *sys, int n_sys, const double *re2,
                                                                 int64_t n_cand, double nu_lo, double nu_hi,
                                                                 int32_t *counts)
{
    __shared__ int32_t s_wave[kGenThreads / 64];
    const int64_t t = (int64_t)blockIdx.x * kGenThreads + threadIdx.x;
    GenLine o;
    const bool ok = t < n_cand && gen_candidate(sys, n_sys, re2, t, nu_lo, nu_hi, o);
    int32_t total;
    (void)block_rank(ok, s_wave, total);
    if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

__global__ __launch_bounds__(kGenThreads) void gen_write_kernel(const DevBand *sys, int n_sys, const double *re2,
                                                                 int64_t n_cand, double nu_lo, double nu_hi,
                                                                 const int64_t *offsets, lrt_line_buffers out)
{
    __shared__ int32_t s_wave[kGenThreads / 64];
    const int64_t t = (int64_t)blockIdx.x * kGenThreads + threadIdx.x;
    GenLine o;
    const bool ok = t < n_cand && gen_candidate(sys, n_sys, re2, t, nu_lo, nu_hi, o);
    int32_t total;
    const int32_t rank = block_rank(ok, s_wave, total);
    if (!ok) return;
    const int64_t i = offsets[blockIdx.x] + rank;
    out.nu0[i] = o.nu0;
    out.A[i] = o.A;
    out.Eu_ev[i] = o.Eu_ev;
    out.Eu_rot[i] = o.Eu_rot;
    out.El_ev[i] = o.El_ev;
    out.El_rot[i] = o.El_rot;
    out.gu[i] = o.gu;
    out.gl[i] = o.gl;
    out.species[i] = o.species;
}

bool finite_nonneg(double v) { return v >= 0.0 && std::isfinite(v); }

}  // namespace
}  // namespace lrt

using namespace lrt;

extern "C" lrt_status lrt_gen_rovib_lines(lrt_ctx *c, int n, const lrt_band_system *sys, double nu_min,
                                          double nu_max, int64_t cap, const lrt_line_buffers *out,
                                          int64_t *n_out, void *stream)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (c->n_species < 1) return fail(c, LRT_E_STATE, "set species before generating lines");
    if (n < 1 || !sys || !n_out) return fail(c, LRT_E_ARG, "need at least one band system and n_out");
    if (!(nu_min < nu_max) || !std::isfinite(nu_min) || !std::isfinite(nu_max))
        return fail(c, LRT_E_ARG, "nu_min < nu_max required");
    if (cap < 0 || (cap > 0 && (!out || !out->nu0 || !out->A || !out->Eu_ev || !out->Eu_rot || !out->El_ev ||
                                !out->El_rot || !out->gu || !out->gl || !out->species)))
        return fail(c, LRT_E_ARG, "output arrays must be non-NULL when cap > 0");
    std::vector<DevBand> h(n);
    std::vector<double> re2;
    int64_t n_cand = 0;
    for (int k = 0; k < n; ++k) {
        const lrt_band_system &s = sys[k];
        if (s.species < 0 || s.species >= c->n_species || c->sp_kind[s.species] != LRT_KIND_MOLECULE)
            return fail(c, LRT_E_ARG, "system %d: species %d is not a molecule", k, s.species);
        if (s.nv_u < 1 || s.nv_l < 1 || s.J_max < 0 || s.J_max > 100000 || !s.Re2)
            return fail(c, LRT_E_ARG, "system %d: needs nv >= 1, 0 <= J_max and Re2", k);
        if (s.hund != LRT_HUND_A && s.hund != LRT_HUND_B)
            return fail(c, LRT_E_ARG, "system %d: unknown coupling case %d", k, s.hund);
        if (s.Lambda_u < 0 || s.Lambda_l < 0 || (s.hund == LRT_HUND_A && std::abs(s.Lambda_u - s.Lambda_l) > 1) ||
            (s.hund == LRT_HUND_B && (s.Lambda_u != 0 || s.Lambda_l != 0)))
            return fail(c, LRT_E_ARG, "system %d: Lambda outside the tables", k);
        if (!(s.g_u >= 1.0) || !(s.g_l >= 1.0) || !std::isfinite(s.g_u) || !std::isfinite(s.g_l))
            return fail(c, LRT_E_ARG, "system %d: degeneracy factors must be >= 1", k);
        const double *cs[18] = {&s.Te_u, &s.Te_l, &s.we_u, &s.wexe_u, &s.weye_u, &s.Be_u, &s.ae_u, &s.De_u,
                                &s.be_u, &s.gamma_u, &s.we_l, &s.wexe_l, &s.weye_l, &s.Be_l, &s.ae_l,
                                &s.De_l, &s.be_l, &s.gamma_l};
        for (const double *p : cs)
            if (!std::isfinite(*p)) return fail(c, LRT_E_ARG, "system %d: non-finite constant", k);
        const int64_t nb = (int64_t)s.nv_u * s.nv_l;
        for (int64_t b = 0; b < nb; ++b)
            if (!finite_nonneg(s.Re2[b])) return fail(c, LRT_E_ARG, "system %d: Re2 must be >= 0 and finite", k);
        DevBand &d = h[k];
        d.species = s.species;
        d.hund = s.hund;
        d.lam_u = s.Lambda_u;
        d.lam_l = s.Lambda_l;
        d.nv_u = s.nv_u;
        d.nv_l = s.nv_l;
        d.J_max = s.J_max;
        d.slots = (s.hund == LRT_HUND_A ? 3 : 6) * (s.J_max + 1);
        d.cand0 = n_cand;
        d.re2_off = (int64_t)re2.size();
        d.Te_u = s.Te_u; d.Te_l = s.Te_l; d.g_u = s.g_u; d.g_l = s.g_l;
        d.we_u = s.we_u; d.wexe_u = s.wexe_u; d.weye_u = s.weye_u; d.Be_u = s.Be_u; d.ae_u = s.ae_u;
        d.De_u = s.De_u; d.be_u = s.be_u; d.gamma_u = s.gamma_u;
        d.we_l = s.we_l; d.wexe_l = s.wexe_l; d.weye_l = s.weye_l; d.Be_l = s.Be_l; d.ae_l = s.ae_l;
        d.De_l = s.De_l; d.be_l = s.be_l; d.gamma_l = s.gamma_l;
        re2.insert(re2.end(), s.Re2, s.Re2 + nb);
        n_cand += nb * d.slots;
    }
    if (n_cand >= ((int64_t)1 << 31)) return fail(c, LRT_E_ARG, "too many candidate lines (%lld)", (long long)n_cand);
    hipStream_t st = (hipStream_t)stream;
    const int64_t n_blocks = (n_cand + kGenThreads - 1) / kGenThreads;
    lrt_status r;
    if ((r = ensure(c, c->w_gen_sys, h.size() * sizeof(DevBand))) || (r = ensure(c, c->w_gen_re2, re2.size() * 8)) ||
        (r = ensure(c, c->w_gen_cnt, (size_t)n_blocks * sizeof(int32_t))) ||
        (r = ensure(c, c->w_gen_off, (size_t)n_blocks * sizeof(int64_t))))
        return r;
    LRT_HIP(c, hipMemcpyAsync(c->w_gen_sys.p, h.data(), h.size() * sizeof(DevBand), hipMemcpyHostToDevice, st));
    LRT_HIP(c, hipMemcpyAsync(c->w_gen_re2.p, re2.data(), re2.size() * 8, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(gen_count_kernel, dim3((unsigned)n_blocks), dim3(kGenThreads), 0, st,
                       c->w_gen_sys.as<DevBand>(), n, c->w_gen_re2.as<double>(), n_cand, nu_min, nu_max,
                       c->w_gen_cnt.as<int32_t>());
    LRT_HIP(c, hipGetLastError());
    std::vector<int32_t> cnt((size_t)n_blocks);
    LRT_HIP(c, hipMemcpyAsync(cnt.data(), c->w_gen_cnt.p, cnt.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    LRT_HIP(c, hipStreamSynchronize(st));
    std::vector<int64_t> off((size_t)n_blocks);
    int64_t tot = 0;
    for (int64_t b = 0; b < n_blocks; ++b) {
        off[b] = tot;
        tot += cnt[b];
    }
    *n_out = tot;
    if (cap == 0) return LRT_OK;
    if (cap < tot) return fail(c, LRT_E_ARG, "capacity %lld below the %lld lines", (long long)cap, (long long)tot);
    LRT_HIP(c, hipMemcpyAsync(c->w_gen_off.p, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(gen_write_kernel, dim3((unsigned)n_blocks), dim3(kGenThreads), 0, st,
                       c->w_gen_sys.as<DevBand>(), n, c->w_gen_re2.as<double>(), n_cand, nu_min, nu_max,
                       c->w_gen_off.as<int64_t>(), *out);
    LRT_HIP(c, hipGetLastError());
    LRT_HIP(c, hipStreamSynchronize(st));
    return LRT_OK;
}
