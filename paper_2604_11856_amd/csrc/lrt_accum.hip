// gfx950 kernels of the line-by-line path (arXiv 2604.11856): populations,
// line setups and the line-to-grid accumulation.
//
//   thermo      per (cell, species): atomic partition function, ln(N/Q),
//               Doppler coefficient; per cell: beta's, Lorentz HWHM, line-skip
//               bound (Sec. 2.1 Boltzmann populations, Sec. 2.2.1 widths);
//               molq: ln(N/Q) of the molecules, one wave per (cell, species); the
//               QSS-CR populations of selected atoms come from lrt_cr.hip
//               and enter the line setup as departures from Boltzmann
//   ranges      per (cell, tile): index range of the nu0-sorted lines that
//               can reach the tile
//   scale       per cell: power-of-two scale of the single-precision eta/kappa
//   accum_*     per (cell, tile): stage per-(cell, line) setups in LDS (FP64),
//               then every lane accumulates the Whiting-Voigt profile of each
//               staged line at its own grid points (Sec. 2.2.1)
//   count       per (cell, candidate line): in-window and core term counts
//   serve       serving kernel: profiles + march of request chunks, one
//               workgroup per item, and the composition of finished tiles
// The march of the path and its reductions live in lrt_march.hip.
//
// Everything is output-stationary: each output element has one owner, so no
// atomics touch eta, kappa, I or the flux; sums run in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <climits>
#include <cstdint>
#include <cmath>
#include <type_traits>

#include "lrt_device.h"
#include "lrt_internal.h"

namespace lrt {

namespace {


// ---------------------------------------------------------------------------
// a1: partition functions and per-cell constants (FP64)
// ---------------------------------------------------------------------------

// van der Waals HWHM (cm^-1) of the lines of atom s in cell c: the printed
// lambda^2 [6.65e-29 N_s (2T/M_s)^0.5 + 2.925e-29 N_o (2T/M_o)^0.5] nm times
// 1e7/lambda^2; N_o, M_o over the other species but electrons (M < 0.01).
__device__ double vdw_width(const DevSpecies &sp, const DevCells &cells, int c, int s)
{
    const int S = cells.n_species;
    const double Ttr = cells.T_tr[c];
    double No = 0.0, NMo = 0.0;
    for (int t = 0; t < S; ++t) {
        if (t == s || sp.mass[t] < 0.01) continue;
        const double n = cells.N[(int64_t)c * S + t];
        No += n;
        NMo += n * sp.mass[t];
    }
    double w = 6.65e-29 * cells.N[(int64_t)c * S + s] * sqrt(2.0 * Ttr / sp.mass[s]);
    if (No > 0.0) w += 2.925e-29 * No * sqrt(2.0 * Ttr / (NMo / No));
    return 1e7 * w;
}

__global__ void thermo_kernel(DevSpecies sp, DevCells cells, DevWidths wd, double M_min,
                              uint64_t mask, CellConst *cc, CellSpecies *cs)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int S = cells.n_species;
    if (t >= (int64_t)cells.n_cells * S) return;
    const int c = (int)(t / S), s = (int)(t % S);
    const double Tv = cells.T_v[c], Ttr = cells.T_tr[c];
    const double bv = kC2 / Tv, br = kC2 / Ttr;
    const int kind = sp.kind[s];
    double Q = 0.0;
    if (kind == 1) {
        for (int64_t j = sp.lev_off[s]; j < sp.lev_off[s + 1]; ++j)
            Q += sp.lev_g[j] * exp(-bv * sp.lev_E[j]);
    }
    const double N = cells.N[(int64_t)c * S + s];
    CellSpecies o;
    // species outside a non-zero mask carry no lines (bit s of mask); a
    // molecule's ln(N/Q) comes from molq_kernel, launched next
    const bool on = species_on(mask, s);
    o.lnNQ = (on && kind == 1 && N > 0.0 && Q > 0.0) ? log(N) - log(Q) : -INFINITY;
    o.dop = 7.16233e-7 / 2.0 * sqrt(Ttr / sp.mass[s]);
    o.gW = (wd.E_ion && kind == 1 && wd.E_ion[s] > 0.0) ? vdw_width(sp, cells, c, s) : 0.0;
    cs[t] = o;
    if (s == 0) {
        CellConst k;
        k.beta_v = bv;
        k.beta_tr = br;
        k.gL = 1e-16 * cells.n_e[c] * pow(Tv / 1e4, 0.33);
        // Voigt HWHM <= gL + gG, gG = dop(M) nu0 <= dop(M_min) nu0; widened.
        // gL of any line <= gN_max + gS_max gL(c) + the largest van der Waals width.
        double gWmax = 0.0;
        if (wd.E_ion)
            for (int s2 = 0; s2 < S; ++s2)
                if (sp.kind[s2] == 1 && wd.E_ion[s2] > 0.0) gWmax = fmax(gWmax, vdw_width(sp, cells, c, s2));
        k.cand_G = 100.0 * (wd.gN_max + wd.gS_max * k.gL + gWmax) * (1.0 + 1e-6);
        k.cand_A = 100.0 * (7.16233e-7 / 2.0) * sqrt(Ttr / M_min) * (1.0 + 1e-6);
        cc[c] = k;
    }
}

// ln(N/Q) of a molecule (Sec. 2.1 molecular Boltzmann relation), one wave per
// (cell, species): Q = sum_e g_e e^{-beta_v T_e} sum_v e^{-beta_v G_v}
// sum_J (2J+1) e^{-beta_tr (B_v J(J+1) - D_v J^2(J+1)^2)}, lane l taking the
// J = l (mod 64) terms of every (e, v), then the lanes summed in a fixed
// butterfly order.  Waves of other species leave at once.
__global__ __launch_bounds__(64) void molq_kernel(DevSpecies sp, DevCells cells, uint64_t mask, CellSpecies *cs)
{
    const int S = cells.n_species;
    const int64_t t = blockIdx.x;
    const int c = (int)(t / S), s = (int)(t % S);
    if (sp.kind[s] != 2) return;
    const int lane = threadIdx.x;
    const double bv = kC2 / cells.T_v[c], br = kC2 / cells.T_tr[c];
    double Q = 0.0;
    for (int64_t e = sp.el_off[s]; e < sp.el_off[s + 1]; ++e) {
        double qvr = 0.0;
        const int Jmax = sp.el_Jmax[e];
        for (int64_t v = sp.vib_off[e]; v < sp.vib_off[e + 1]; ++v) {
            const double B = sp.vib_B[v], D = sp.vib_D[v];
            double qr = 0.0;
            for (int J = lane; J <= Jmax; J += 64) {
                const double jj = (double)J * (J + 1.0);
                qr += (2.0 * J + 1.0) * exp(-br * (B * jj - D * jj * jj));
            }
            qvr += exp(-bv * sp.vib_G[v]) * qr;
        }
        Q += sp.el_g[e] * exp(-bv * sp.el_T[e]) * qvr;
    }
    for (int o = 32; o > 0; o >>= 1) Q += __shfl_xor(Q, o);
    if (lane == 0) {
        const double N = cells.N[(int64_t)c * S + s];
        cs[t].lnNQ = (species_on(mask, s) && N > 0.0 && Q > 0.0) ? log(N) - log(Q) : -INFINITY;
    }
}

// ---------------------------------------------------------------------------
// a2: one (cell, line) pair in FP64
// ---------------------------------------------------------------------------

struct PairF64 {
    double se, sk;        // eta and kappa per unit profile shape (strength * norm)
    double inv2g, r;      // 1 / (2 gamma_V), gamma_L / gamma_V
    int32_t klo, khi;     // inclusive window, klo > khi when empty
    int32_t kclo, kchi;   // core: points with |nu_k - nu0| <= kCoreHalfWidth gamma_V
};

// Half-width of the single-precision core in units of gamma_V, where the
// profile's two exponential terms are evaluated.  Beyond it x = |dnu|/(2
// gamma_V) > 6, and with the staged normalisation s = max(r, 2^-40) the
// exponential part (1-r)/s e^{-2.772 x^2} + 0.016 r(1-r)/s e^{-0.4 x^2.25}
// is below 5.1e-32 + 2.7e-12, while the rational part 1/(1+4x^2) -
// 0.016(1-r)/(1+0.1 x^2.25) is at least 4.48e-3 (both ratios fall with x):
// the omitted part is below 2^-30 of the term, under a quarter of the
// single-precision rounding of the term itself.  (At 25 gamma_V both
// exponentials are exactly zero in single precision; the narrower core
// halves the terms that evaluate them.)
constexpr double kCoreHalfWidth = 12.0;

// The cell's row of ln departures from Boltzmann (QSS-CR populations), or
// NULL when no line has levels.
__device__ __forceinline__ const double *cr_row(const DevLines &L, int c)
{
    return L.lev ? L.lnd + (int64_t)c * L.lnd_stride : nullptr;
}

__device__ __forceinline__ bool pair_setup(const DevLines &L, const DevGrid &g, const CellConst &k,
                                           const CellSpecies *csc, const double *lnd_c, int64_t i,
                                           PairF64 &p)
{
    const int s = L.species[i];
    const CellSpecies q = csc[s];
    if (!(q.lnNQ > -INFINITY)) {
        p.klo = p.kclo = 1;
        p.khi = p.kchi = 0;
        p.se = p.sk = p.inv2g = p.r = 0.0;
        return false;
    }
    const double nu0 = L.nu0[i];
    const double Eu_ev = L.Eu_ev[i], Eu_rot = L.Eu_rot[i];
    const double El_ev = L.El_ev[i], El_rot = L.El_rot[i];
    const double base = q.lnNQ + L.lngu[i];
    // N_u = N g_u e^{-E_u}/Q, and N_l g_u/g_l = N_u e^{x} with x the line's
    // reduced energy, so N_l (g_u/g_l)(1 - e^{-x}) = N_u (e^{x} - 1)
    const double lnNu = base - k.beta_v * Eu_ev - k.beta_tr * Eu_rot;
    const double x = k.beta_v * (Eu_ev - El_ev) + k.beta_tr * (Eu_rot - El_rot);
    const int32_t lv = lnd_c ? L.lev[i] : -1;
    double Nu, Nlx;
    if (lv < 0) {
        Nu = exp(lnNu);
        // (the two-factor form only while N_u e^{x} stays representable)
        Nlx = (lnNu > -700.0 && x < 700.0) ? Nu * expm1(x) : exp(lnNu + x) * (-expm1(-x));
    } else {
        // QSS-CR populations: both levels carry their departure from
        // Boltzmann, N_u = e^{lu}, N_l g_u/g_l = e^{ll}, and the absorption
        // takes N_l g_u/g_l - N_u (negative for an inverted pair)
        const double lu = lnNu + lnd_c[lv & 0xffff];
        const double ll = lnNu + x + lnd_c[lv >> 16];
        Nu = exp(lu);
        Nlx = (ll >= lu) ? (ll > -INFINITY ? exp(ll) * -expm1(lu - ll) : 0.0) : -(Nu * -expm1(ll - lu));
    }
    const double Seta = L.seta0[i] * Nu;
    const double Skap = L.skap0[i] * Nlx;
    // widths (Sec. 2.2.1): Doppler, Lorentz, Voigt (Olivero fit)
    const double gG = q.dop * nu0;
    const double gL = L.gN[i] + L.gS[i] * k.gL + q.gW;
    const double sum = gL + gG;
    const double d = (gL - gG) / sum;
    const double gV = (1.0 - 0.18121 * (1.0 - d * d)
                       - (0.023665 * exp(0.6 * d) + 0.00418 * exp(-1.9 * d)) * sinpi(d)) * sum;
    const double inv_gV = 1.0 / gV;
    const double r = gL * inv_gV;
    const double norm = (0.5 * inv_gV) / (1.065 + 0.447 * r + 0.058 * r * r);
    // window |nu_k - nu0| <= 100 gamma_V; rounding-exact operation order
    const double W = __dmul_rn(100.0, gV);
    double lo = ceil(__ddiv_rn(__dsub_rn(__dsub_rn(nu0, W), g.nu_min), g.h));
    double hi = floor(__ddiv_rn(__dsub_rn(__dadd_rn(nu0, W), g.nu_min), g.h));
    lo = fmax(lo, 0.0);
    hi = fmin(hi, (double)(g.n_points - 1));
    if (lo > hi) {
        p.klo = 1;
        p.khi = 0;
    } else {
        p.klo = (int32_t)lo;
        p.khi = (int32_t)hi;
    }
    {
        // core: a superset of the points within 25 gamma_V (one point of
        // margin on each side covers the rounding of the product by 1/h)
        const double Wc = kCoreHalfWidth * gV;
        double clo = fmax(ceil((nu0 - Wc - g.nu_min) * g.inv_h) - 1.0, lo);
        double chi = fmin(floor((nu0 + Wc - g.nu_min) * g.inv_h) + 1.0, hi);
        if (clo > chi) {
            p.kclo = 1;
            p.kchi = 0;
        } else {
            p.kclo = (int32_t)clo;
            p.kchi = (int32_t)chi;
        }
    }
    p.se = Seta * norm;
    p.sk = Skap * norm;
    p.inv2g = 0.5 * inv_gV;
    p.r = r;
    return p.klo <= p.khi;
}

// ---------------------------------------------------------------------------
// atomic continuum (Sec. 2.2.1 bound-free and free-free)
// ---------------------------------------------------------------------------

constexpr double kElectronMass = 9.1093837015e-28;   // g

// Per cell: prefix sums over the sorted thresholds of the bound-free
// absorption and emission weights (times nu_thr^3), the two free-free
// coefficients, and ln upper bounds of eta_c and kappa_c over [nu_lo, nu_hi]
// for the power-of-two scale.
__global__ void cont_cells_kernel(const ContThr *thr, int32_t n_thr, const ContRec *rec,
                                  int32_t n_rec, DevCells cells, const CellSpecies *cs, DevCR cr,
                                  uint64_t species_mask, double nu_lo, double nu_hi, double *cum,
                                  double *ff, double *lnb)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells.n_cells) return;
    const int ns = cells.n_species;
    const double T = cells.T_v[c], ne = cells.n_e[c];
    // Saha-Boltzmann volume (h^2 / (2 pi m_e k T))^{3/2}
    const double V = pow(kPlanck * kPlanck / (2.0 * kPi * kElectronMass * kBoltz * T), 1.5);
    double *cA = cum + (int64_t)c * 2 * (n_thr + 1), *cB = cA + (n_thr + 1);
    double a = 0.0, b = 0.0, ka = 0.0, eb = 0.0;
    cA[0] = cB[0] = 0.0;
    const double twohc2 = 1e-7 * 2.0 * kPlanck * kLight * kLight;
    for (int j = 0; j < n_thr; ++j) {
        const ContThr t = thr[j];
        const ContRec r = rec[t.rec];
        if (!species_on(species_mask, r.species)) {   // a species outside the mask radiates nothing
            cA[j + 1] = a;
            cB[j + 1] = b;
            continue;
        }
        const double Np = cells.N[(int64_t)c * ns + r.ion];
        const int slot = cr.n > 0 ? cr.slot[r.species] : -1;
        // absorption from the level: its QSS-CR population, else Boltzmann
        const double aj = slot >= 0 ? cr.pop[((int64_t)c * cr.n + slot) * cr.LS + t.lev] * t.s3
                                    : exp(cs[(int64_t)c * ns + r.species].lnNQ) * t.g * exp(-kC2 * t.E / T) * t.s3;
        const double bj = Np * ne * V * t.g / (2.0 * r.Q_ion) * t.s3;   // without e^{c2 nu_j / T}
        a += aj;
        b += bj * exp(kC2 * t.nu / T);
        cA[j + 1] = a;
        cB[j + 1] = b;
        // bounds: at nu >= max(nu_j, nu_lo), aj / nu^3 <= aj / max(nu_j, nu_lo)^3 and
        // B(nu) bj e^{c2 nu_j/T} / nu^3 <= 2hc^2 bj / (1 - e^{-c2 max(nu_j, nu_lo)/T})
        const double nm = fmax(t.nu, nu_lo);
        ka += aj / (nm * nm * nm);
        eb += twohc2 * bj / -expm1(-kC2 * nm / T);
    }
    double f0 = 0.0, f1 = 0.0;
    for (int q = 0; q < n_rec; ++q) {
        const ContRec r = rec[q];
        if (!species_on(species_mask, r.species)) continue;
        const double w = cells.N[(int64_t)c * ns + r.ion] * ne * 1e-40 * r.z4inv;
        f0 += w * (r.peach[0] + r.peach[1] * exp(-r.peach[2] * T));
        f1 += w * (r.peach[3] + r.peach[4] * exp(-r.peach[5] * T) + r.peach[6] * exp(-r.peach[7] * T));
    }
    ff[2 * c + 0] = f0;
    ff[2 * c + 1] = f1;
    // free-free falls with nu on the grid; its emission carries the Planck
    // factor, whose maximum over [nu_lo, nu_hi] is at nu_p = 2.8214 T / c2 or
    // the nearer end
    const double inv3 = 1.0 / (nu_lo * nu_lo * nu_lo);
    const double kff = (fabs(f0) * kNuH / nu_lo + fabs(f1)) * kNuH * kNuH * kNuH * inv3;
    const double nu_p = fmin(fmax(2.8214393721220787 * T / kC2, nu_lo), nu_hi);
    const double km = ka + kff, em = eb + planck_f64(nu_p, T) * kff;
    lnb[2 * c + 0] = em > 0.0 ? log(em) : -INFINITY;
    lnb[2 * c + 1] = km > 0.0 ? log(km) : -INFINITY;
}

// Continuum eta and kappa of cell c at nu (double precision).
__device__ __forceinline__ void continuum_point(const DevCont &ct, int c, double nu, double &eta,
                                                double &kap)
{
    int lo = 0, hi = ct.n_thr;   // m = number of thresholds <= nu
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ct.thr[mid].nu <= nu) lo = mid + 1; else hi = mid;
    }
    const double *cA = ct.cum + (int64_t)c * 2 * (ct.n_thr + 1);
    const double inv3 = 1.0 / (nu * nu * nu);
    const double kff = (ct.ff[2 * c] * (kNuH / nu) + ct.ff[2 * c + 1]) * (kNuH * kNuH * kNuH) * inv3;
    kap = cA[lo] * inv3 + kff;
    eta = planck_f64(nu, ct.T_v[c]) * (cA[ct.n_thr + 1 + lo] * inv3 + kff);
}

// ---------------------------------------------------------------------------
// candidate line ranges per (cell, tile)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int64_t lower_bound_dev(const double *a, int64_t n, double v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t m = lo + ((hi - lo) >> 1);
        if (a[m] < v) lo = m + 1; else hi = m;
    }
    return lo;
}

__global__ void ranges_kernel(DevLines L, DevGrid g, const CellConst *cc, int32_t n_cells,
                              int32_t k_first, int32_t n_band, int32_t tile_points,
                              int32_t n_tiles, int2 *ranges)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_cells * n_tiles) return;
    const int c = (int)(t / n_tiles), tile = (int)(t % n_tiles);
    const CellConst k = cc[c];
    const int32_t ka = k_first + tile * tile_points;
    const int32_t kb = min(k_first + n_band, ka + tile_points) - 1;
    const double nu_a = g.nu_min + (double)ka * g.h - g.h;
    const double nu_b = g.nu_min + (double)kb * g.h + g.h;
    const double lo = (nu_a - k.cand_G) / (1.0 + k.cand_A);
    const double hi = (nu_b + k.cand_G) / (1.0 - k.cand_A);
    int2 r;
    r.x = (int)lower_bound_dev(L.nu0, L.n, lo);
    r.y = (int)lower_bound_dev(L.nu0, L.n, hi);
    ranges[t] = r;
}

// ---------------------------------------------------------------------------
// per-cell power-of-two scale for the single-precision form
// ---------------------------------------------------------------------------

__global__ void scale_kernel(DevLines L, int64_t i0, int64_t i1, DevGrid g, const CellConst *cc,
                             const CellSpecies *cs, int32_t n_cells, int32_t n_species,
                             int32_t *emax)
{
    const int64_t i = i0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int c = blockIdx.y; c < n_cells; c += gridDim.y) {
        int ee = INT_MIN, ek = INT_MIN;
        if (i < i1) {
            PairF64 p;
            if (pair_setup(L, g, cc[c], cs + (int64_t)c * n_species, cr_row(L, c), i, p)) {
                if (p.se != 0.0) ee = ilogb(p.se) + 1;
                if (p.sk != 0.0) ek = ilogb(fabs(p.sk)) + 1;
            }
        }
        // wave max, then one atomic per wave (max is order independent)
        for (int o = 32; o > 0; o >>= 1) {
            ee = max(ee, __shfl_xor(ee, o));
            ek = max(ek, __shfl_xor(ek, o));
        }
        if ((threadIdx.x & 63) == 0) {
            if (ee != INT_MIN) atomicMax(&emax[2 * c + 0], ee);
            if (ek != INT_MIN) atomicMax(&emax[2 * c + 1], ek);
        }
    }
}

// Per-cell scale from the level-energy bins: one wave per cell takes the
// largest upper bound of ln(eta peak) and ln(|kappa peak|) over the bins.
// Peak of line i: strength * norm with norm = 1/(2 gV (1.065 + ...)) and
// gV >= 0.9 gG (the Voigt width is at least the Doppler one; 0.9 leaves room
// for the fit), gG = dop_s nu0; |kappa| <= skap0 max(N_u, N_l g_u/g_l).  The
// bound exceeds the true peak by a modest factor (bin width, Lorentz part of
// the width), which the power-of-two scale absorbs.
__global__ void scale_bound_kernel(DevBins B, const CellConst *cc, const CellSpecies *cs,
                                   const double *cont_lnb, int32_t n_cells, int32_t n_species,
                                   int32_t *escale)
{
    const int c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= n_cells) return;
    const CellConst k = cc[c];
    const double ln_norm = -log(2.0 * 1.065 * 0.9);
    double ve = -INFINITY, vk = -INFINITY;
    const double *lnd_c = B.lev_off ? B.lnd + (int64_t)c * B.lnd_stride : nullptr;
    // a spectral window: line centres that can reach it (as ranges_kernel)
    double ca = -INFINITY, cb = INFINITY;
    if (B.nu_lo) {
        ca = (B.win_a - k.cand_G) / (1.0 + k.cand_A);
        cb = (B.win_b + k.cand_G) / (1.0 - k.cand_A);
    }
    for (int b = lane; b < B.n; b += 64) {
        if (B.nu_lo && (B.nu_hi[b] < ca || B.nu_lo[b] > cb)) continue;
        const CellSpecies q = cs[(int64_t)c * n_species + B.species[b]];
        if (!(q.lnNQ > -INFINITY)) continue;
        double v = q.lnNQ + ln_norm - log(q.dop) - k.beta_v * B.Ev[b] - k.beta_tr * B.Er[b];
        if (lnd_c) {
            // QSS-CR: the largest departure from Boltzmann among the bin's levels
            double d = -INFINITY;
            for (int32_t j = B.lev_off[b]; j < B.lev_off[b + 1]; ++j) {
                const int32_t o = B.lev[j];
                d = fmax(d, o < 0 ? 0.0 : lnd_c[o]);
            }
            v += d;
        }
        ve = fmax(ve, B.a_eta[b] + v);
        vk = fmax(vk, B.a_kap[b] + v);
    }
    for (int o = 32; o > 0; o >>= 1) {
        ve = fmax(ve, __shfl_xor(ve, o));
        vk = fmax(vk, __shfl_xor(vk, o));
    }
    if (cont_lnb) {   // the atomic continuum's own bound
        ve = fmax(ve, cont_lnb[2 * c + 0]);
        vk = fmax(vk, cont_lnb[2 * c + 1]);
    }
    if (lane == 0) {
        // peak < 2^e; stay unscaled while e is within 2^+-60
        const double v2[2] = {ve, vk};
        for (int j = 0; j < 2; ++j) {
            int e = 0;
            if (v2[j] > -INFINITY) {
                const double t = ceil(v2[j] * kLog2e) + 1.0;
                e = (int)fmax(-2000.0, fmin(2000.0, t));
                if (e >= -60 && e <= 60) e = 0;
            }
            escale[2 * c + j] = e;
        }
    }
}

__global__ void scale_finish_kernel(const int32_t *emax, const double *cont_lnb, int32_t n, int32_t *escale)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int e = emax[t];
    if (cont_lnb && cont_lnb[t] > -INFINITY)   // the atomic continuum's own bound: peak < 2^e
        e = max(e, (int)fmax(-2000.0, fmin(2000.0, ceil(cont_lnb[t] * kLog2e) + 1.0)));
    // keep values unscaled while the largest line peak stays within 2^+-60
    escale[t] = (e == INT_MIN || (e >= -60 && e <= 60)) ? 0 : e;
}

// ---------------------------------------------------------------------------
// a3: line-to-grid accumulation
// ---------------------------------------------------------------------------

// Single-precision line record staged in LDS.  Grid indices inside the
// kernel are relative to the tile start, so every float index is a small
// exact integer whatever the grid size.
//
// `mode` holds three masks over the tile's 64-point slices (slice s = points
// 64s..64s+63, bit s of each byte): bits 0-7 "window reaches the slice",
// bits 8-15 "window edge inside the slice (mask lanes)", bits 16-23 "core
// window reaches the slice (exponential terms)".  Decided once at staging; a
// wave turns the bits of its own slices, over a block of lines, into scalar
// bit masks and needs no vector work for control flow.
constexpr int kSlices = kTilePoints / 64;
struct __align__(16) RecF32 {
    float k0f, hg, fg, qw;          // centre index (tile-relative), h/gV, frac0/gV, 0.016 r (1-r) / s
    float qg, pad0, se, sk;         // (1-r) / s, -, strengths times s and the cell's scale
    float klo, khi;                 // window, tile-relative, clamped to [-1, tile] (edge masks)
    uint32_t mode, pad;
};
static_assert(kSlices <= 8 && kPPL <= 2, "mode masks hold at most 8 slices per tile");

// Slices of the tile overlapped by [lo, hi] (tile-relative, possibly beyond
// the tile): a contiguous run of bits.
__device__ __forceinline__ uint32_t slice_run(int32_t lo, int32_t hi)
{
    if (lo > hi || hi < 0 || lo > kTilePoints - 1) return 0u;
    const int32_t a = max(lo, 0) >> 6, b = min(hi, kTilePoints - 1) >> 6;
    return (2u << b) - (1u << a);
}

// Mode masks of a window [klo, khi] with core window [kclo, kchi] (tile-relative).
__device__ __forceinline__ uint32_t slice_modes(int32_t klo, int32_t khi, int32_t kclo, int32_t kchi)
{
    const uint32_t in = slice_run(klo, khi);
    // a slice holds a window edge when the window starts or ends strictly inside it
    uint32_t edge = 0u;
    if (klo >= 0 && (klo & 63) != 0) edge |= 1u << min(klo >> 6, 31);
    if (khi < kTilePoints && (khi & 63) != 63 && khi >= 0) edge |= 1u << min(khi >> 6, 31);
    const uint32_t core = slice_run(max(kclo, klo), min(kchi, khi));
    return in | ((edge & in) << 8) | ((core & in) << 16);
}

struct __align__(16) RecF64 {
    int32_t klo, khi, k0;
    uint32_t mode;          // slice masks: in, edge, x^2.25 window, Gaussian window
    double frac0, inv2g, r, se, sk, pad2;
};

// The Whiting profile is evaluated in y = (nu_k - nu0) / gamma_V = +-2x, so that
// 1 + 4x^2 = 1 + y^2 is one FMA and x^2.25 = 2^-2.25 |y|^2.25.
constexpr double kTwoM225 = 0.21022410381342863;   // 2^-2.25

// Constants of the single-precision profile.  The kernels set them once,
// outside their loops, and an empty asm keeps them in scalar registers: VOP3
// instructions take no literal on this chip, so a constant rebuilt inside
// the loop costs a vector move per use.
struct ShapeConsts {
    float c225;   // 2.25 (the exponent of |y|)
    float cw;     // 0.1 * 2^-2.25 (0.1 x^2.25 from |y|^2.25)
    float cg;     // -2.772/4 log2(e) (the Gaussian exponent from 1 + y^2)
    float ce;     // -0.4 * 2^-2.25 log2(e) (the other exponent)
};

__device__ __forceinline__ ShapeConsts shape_consts()
{
    ShapeConsts K{2.25f, (float)(0.1 * kTwoM225), (float)(-2.772 / 4.0 * kLog2e),
                  (float)(-0.4 * kTwoM225 * kLog2e)};
    asm volatile("" : "+s"(K.c225), "+s"(K.cw), "+s"(K.cg), "+s"(K.ce));
    return K;
}

// The profile divided by s = r = gL/gV (the staged strengths carry the
// factor s back): rational part [1/(1+4x^2) - 0.016 (1-r)/(1+0.1 x^2.25)]
// over one reciprocal, whose numerator (1+0.1 x^2.25) - 0.016 (1-r)(1+4x^2)
// is one FMA; also returns 1 + y^2 and |y|^2.25 for the exponential part.
// A line with r below kRScaleMin is staged with s = kRScaleMin instead, which
// adds a Lorentzian of at most kRScaleMin of the line's own peak.  (Two
// reciprocals save instructions but measured 4 % slower: the transcendental
// pipe, not the instruction count, then sets the pace.)
__device__ __forceinline__ float shape_rational_f32(float kf, const RecF32 &q, const ShapeConsts &K, float &d1,
                                                    float &p)
{
    const float y = fmaf(kf - q.k0f, q.hg, -q.fg);
    d1 = fmaf(y, y, 1.0f);
    p = __builtin_amdgcn_exp2f(K.c225 * __builtin_amdgcn_logf(fabsf(y)));
    const float d2 = fmaf(p, K.cw, 1.0f);
    const float num = fmaf(-q.qw, d1, d2);
    return num * __builtin_amdgcn_rcpf(d1 * d2);
}

// Smallest normalisation s of the staged profile (2^-40).
constexpr double kRScaleMin = 9.094947017729282e-13;

// Exponential part [(1-r) e^{-2.772 x^2} + 0.016 r(1-r) e^{-0.4 x^2.25}] / s
// added to P, with x^2 = (d1 - 1)/4 folded into the exponent's FMA.
__device__ __forceinline__ float shape_exp_f32(const RecF32 &q, const ShapeConsts &K, float d1, float p, float P)
{
    const float gs = __builtin_amdgcn_exp2f(fmaf(d1, K.cg, -K.cg));
    const float e = __builtin_amdgcn_exp2f(p * K.ce);
    return fmaf(q.qg, gs, fmaf(q.qw, e, P));
}

// Block -> (tile, cell) order of the accumulation grid: groups of 8 tiles x
// all cells; within a group XCD x (workgroups go round-robin over the 8 XCDs,
// each with its own L2) takes tile 8g + x for every cell, so the cells of one
// tile share their candidate lines in one L2 while tiles stay interleaved
// across XCDs.  (Measured against tile-fastest order: 3 % faster; against a
// contiguous range of tiles per XCD: 37 % faster, the per-XCD work being
// uneven because line density varies along nu.)
__device__ __forceinline__ void block_tile_cell(uint32_t b, int32_t n_cells, int32_t n_tiles, int &tile,
                                                int &cell)
{
    const uint32_t gsz = (uint32_t)kXCDs * (uint32_t)n_cells;
    const uint32_t g = b / gsz, r = b % gsz;
    const uint32_t full = (uint32_t)n_tiles / kXCDs;
    if (g < full) {
        tile = (int)(g * kXCDs + r % kXCDs);
        cell = (int)(r / kXCDs);
    } else {   // last partial group of tiles
        tile = (int)(g * kXCDs + r / (uint32_t)n_cells);
        cell = (int)(r % (uint32_t)n_cells);
    }
}

// Compensated (Kahan) addition of a block partial v into (s, c).
__device__ __forceinline__ void kahan_add(float &s, float &c, float v)
{
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Square root of x > 0 from the hardware reciprocal square root (about 5e-8
// relative) and one Newton step on y^2 = x.  Measured on the chip, the fourth
// root as two such steps stays within 4.2e-15 relative of x^(1/4) over
// [1e-20, 1e4], against 38 instructions for two correctly rounded roots.
__device__ __forceinline__ double sqrt_newton(double x)
{
    const double r = __builtin_amdgcn_rsq(x);
    const double y = x * r;
    return fma(fma(-y, y, x), 0.5 * r, y);
}

// Lines per compensated block: partials of at most kBlock terms are added
// plainly, blocks are merged with Kahan's compensation (64-line blocks
// measured 1 % faster than 32-line ones).  A block is one ballot mask: one bit
// per line.
constexpr int kBlock = 64;
using BlockMask = uint64_t;

// The terms of one staged line (bit t of the block masks) on this wave's
// slices, added to the block partials.
template <typename Mask>
__device__ __forceinline__ void line_terms(const RecF32 &qr, int t, const float (&kf)[kPPL], const ShapeConsts &K,
                                           const Mask (&m_in)[kPPL], const Mask (&m_core)[kPPL],
                                           const Mask (&m_edge)[kPPL], float (&ae)[kPPL], float (&ak)[kPPL])
{
    const RecF32 q = qr;
#pragma unroll
    for (int j = 0; j < kPPL; ++j) {
        if (!((m_in[j] >> t) & 1u)) continue;      // slice outside the window
        float d1, pw;
        float P = shape_rational_f32(kf[j], q, K, d1, pw);
        // Within kCoreHalfWidth gamma_V of the centre the exponentials
        // contribute; beyond it they are below 2^-30 of the term.  Both
        // conditions are wave-uniform; the empty asm keeps them real
        // scalar branches instead of computing both sides and selecting.
        if ((m_core[j] >> t) & 1u) {
            asm volatile("");
            P = shape_exp_f32(q, K, d1, pw, P);
        }
        // slice crossing a window edge: mask the lanes outside
        if ((m_edge[j] >> t) & 1u) {
            asm volatile("");
            P = (kf[j] >= q.klo && kf[j] <= q.khi) ? P : 0.0f;
        }
        ae[j] = fmaf(P, q.se, ae[j]);
        ak[j] = fmaf(P, q.sk, ak[j]);
    }
}

// eta and kappa of one cell on one tile (kTilePoints points starting at the
// global index kt) in single precision: every round stages kStage candidate
// lines (one FP64 setup per thread) into `rec`, then each wave evaluates the
// staged lines on its kPPL slices of 64 points.  Lanes hold the compensated sums;
// the function returns eta[j], kappa[j] of point kt + kw + 64 j + lane (scaled
// by 2^-ese, 2^-esk).  Must be called by the whole workgroup.
__device__ __forceinline__ void accum_cell_tile_f32(RecF32 *rec, const DevLines &L, const DevGrid &g,
                                                    const CellConst &k, const CellSpecies *csc,
                                                    const double *lnd_c, int ese, int esk, int2 rg, int32_t kt,
                                                    int32_t kw, int lane, float (&eta)[kPPL],
                                                    float (&kap)[kPPL])
{
    // first slice of this wave (kw = wave * 64 * kPPL)
    const uint32_t wshift = (uint32_t)(kw / 64);
    const ShapeConsts K = shape_consts();
    float kf[kPPL];
    float se[kPPL], ce[kPPL], sk[kPPL], ck[kPPL], ae[kPPL], ak[kPPL];
#pragma unroll
    for (int j = 0; j < kPPL; ++j) {
        kf[j] = (float)(kw + 64 * j + lane);
        asm volatile("" : "+v"(kf[j]));   // keep the float index in a register
        se[j] = ce[j] = sk[j] = ck[j] = ae[j] = ak[j] = 0.0f;
    }

    for (int base = rg.x; base < rg.y; base += kStage) {
        // stage: one (cell, line) setup per thread, in double precision
        const int64_t i = (int64_t)base + threadIdx.x;
        RecF32 rr;
        rr.mode = 0;
        rr.klo = 1.0f;
        rr.khi = 0.0f;
        rr.k0f = rr.hg = rr.fg = rr.qw = rr.qg = rr.pad0 = rr.se = rr.sk = 0.0f;
        rr.pad = 0;
        if (i < rg.y) {
            PairF64 p;
            if (pair_setup(L, g, k, csc, lnd_c, i, p)) {
                const int32_t lo = p.klo - kt, hi = p.khi - kt;
                rr.mode = slice_modes(lo, hi, p.kclo - kt, p.kchi - kt);
                // small exact integers in float: the lanes compare their float index
                rr.klo = (float)max(lo, -1);
                rr.khi = (float)min(hi, kTilePoints);
                rr.k0f = (float)(L.k0[i] - kt);
                rr.hg = (float)(2.0 * g.h * p.inv2g);
                rr.fg = (float)(2.0 * L.frac0[i] * p.inv2g);
                // profile divided by s = r, strengths times s
                const double sc = fmax(p.r, kRScaleMin), isc = 1.0 / sc;
                rr.qw = (float)(0.016 * p.r * (1.0 - p.r) * isc);
                rr.qg = (float)((1.0 - p.r) * isc);
                rr.se = (float)ldexp(p.se * sc, -ese);
                rr.sk = (float)ldexp(p.sk * sc, -esk);
            }
        }
        rec[threadIdx.x] = rr;
        __syncthreads();
        const int n = min(kStage, rg.y - base);
        for (int l0 = 0; l0 < n; l0 += kBlock) {
            // Control of the block's lines on this wave, as bit masks over the
            // block in scalar registers: lane t < kBlock reads line l0 + t's
            // mode byte, one ballot per (slice, flag).  The loop then visits
            // only the lines that reach this wave, in line order.
            uint32_t mb = 0;
            if (lane < kBlock && l0 + lane < n) mb = rec[l0 + lane].mode >> wshift;
            BlockMask todo = (BlockMask)__ballot((mb & ((1u << kPPL) - 1u)) != 0);
            BlockMask m_in[kPPL], m_edge[kPPL], m_core[kPPL];
#pragma unroll
            for (int j = 0; j < kPPL; ++j) {
                m_in[j] = (BlockMask)__ballot(mb & (1u << j));
                m_edge[j] = (BlockMask)__ballot(mb & (1u << (8 + j)));
                m_core[j] = (BlockMask)__ballot(mb & (1u << (16 + j)));
            }
            // groups of 8 lines: within a group the LDS offsets are constants
            // from one base address held in a vector register, and the block
            // masks, shifted once per group, are tested at constant bits; a
            // group that no line of it reaches is skipped whole
            for (int g8 = 0; g8 < kBlock; g8 += 8) {
                const uint32_t gt = (uint32_t)(todo >> g8) & 0xffu;
                if (gt == 0) continue;
                uint32_t gi[kPPL], gc[kPPL], ge[kPPL];
#pragma unroll
                for (int j = 0; j < kPPL; ++j) {
                    gi[j] = (uint32_t)(m_in[j] >> g8);
                    gc[j] = (uint32_t)(m_core[j] >> g8);
                    ge[j] = (uint32_t)(m_edge[j] >> g8);
                }
                // one LDS base per group (a byte offset in a vector register),
                // not one per line
                uint32_t off = (uint32_t)((l0 + g8) * (int)sizeof(RecF32));
                asm volatile("" : "+v"(off));
                const RecF32 *rg8 = (const RecF32 *)((const char *)rec + off);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if ((gt >> u) & 1u) line_terms(rg8[u], u, kf, K, gi, gc, ge, ae, ak);
            }
#pragma unroll
            for (int j = 0; j < kPPL; ++j) {
                kahan_add(se[j], ce[j], ae[j]);
                kahan_add(sk[j], ck[j], ak[j]);
                ae[j] = ak[j] = 0.0f;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < kPPL; ++j) {
        eta[j] = se[j] - ce[j];
        kap[j] = sk[j] - ck[j];
    }
}

__global__ __launch_bounds__(kAccumThreads) __attribute__((amdgpu_waves_per_eu(LRT_ACCUM_WAVES)))
void accum_f32_kernel(
    DevLines L, DevGrid g, const CellConst *cc, const CellSpecies *cs, const int32_t *escale,
    const int2 *ranges, int32_t n_cells, int32_t n_species, int32_t k_first, int32_t n_band,
    int32_t n_tiles, uint32_t b0, DevCont ct, float *eta, float *kappa)
{
    __shared__ RecF32 rec[kStage];
    int tile, c;
    block_tile_cell(b0 + blockIdx.x, n_cells, n_tiles, tile, c);
    // the wave index is uniform across the wave: keep it (and every bound
    // derived from it) in scalar registers so slice tests are scalar branches
    const int lane = threadIdx.x & 63, wave = uniform_i(threadIdx.x >> 6);
    const int32_t kt = k_first + tile * kTilePoints;   // first (global) point of the tile
    const int32_t kw = wave * 64 * kPPL;               // first point of the wave, tile-relative
    const int32_t kend = k_first + n_band;             // exclusive, global
    float e[kPPL], kp[kPPL];
    accum_cell_tile_f32(rec, L, g, cc[c], cs + (int64_t)c * n_species, cr_row(L, c), escale[2 * c + 0],
                        escale[2 * c + 1], ranges[(int64_t)c * n_tiles + tile], kt, kw, lane, e, kp);
#pragma unroll
    for (int j = 0; j < kPPL; ++j) {
        const int32_t kk = kt + kw + 64 * j + lane;
        if (kk < kend) {
            const int64_t o = (int64_t)c * n_band + (kk - k_first);
            if (ct.n_thr >= 0) {
                // atomic continuum, added in double precision and rounded once
                double ce, ck;
                continuum_point(ct, c, g.nu_min + (double)kk * g.h, ce, ck);
                e[j] = (float)((double)e[j] + ldexp(ce, -escale[2 * c + 0]));
                kp[j] = (float)((double)kp[j] + ldexp(ck, -escale[2 * c + 1]));
            }
            eta[o] = e[j];
            kappa[o] = kp[j];
        }
    }
}

// Whiting profile in double precision.  The two rational terms share one
// division.  An exponential whose argument is below -745.6 underflows to
// exactly zero (e^-745.14 is under half the smallest subnormal), so the
// windows of the two exponentials, in units of gamma_V, stop where that
// happens: beyond |dnu| = 33 gamma_V (x = 16.5) e^{-2.772 x^2} is exactly
// zero in double precision, beyond 57 gamma_V (x = 28.5) so is
// e^{-0.4 x^2.25}, while the line windows reach x = 50; the point windows
// carry one point of margin on each side, and a lane inside a window slice
// but beyond its exponential's bound adds an exact zero.
constexpr double kF64GaussHalfWidth = 33.0;
constexpr double kF64WexpHalfWidth = 57.0;

// The terms of one staged line (bit t of the block masks) on this wave's
// slices of points kk[j], added to the sums.
template <typename Mask>
__device__ __forceinline__ void line_terms_f64(const RecF64 &qr, int t, const int32_t (&kk)[kPPL], double h,
                                               const Mask (&m_in)[kPPL], const Mask (&m_w)[kPPL],
                                               const Mask (&m_g)[kPPL], const Mask (&m_edge)[kPPL],
                                               double (&se)[kPPL], double (&sk)[kPPL])
{
    const RecF64 q = qr;
#pragma unroll
    for (int j = 0; j < kPPL; ++j) {
        if (!((m_in[j] >> t) & 1u)) continue;
        const double x = fabs(fma((double)(kk[j] - q.k0), h, -q.frac0)) * q.inv2g;
        const double u = x * x;
        const double p = u * (x > 0.0 ? sqrt_newton(sqrt_newton(x)) : 0.0);
        const double d1 = 1.0 + 4.0 * u, d2 = 1.0 + 0.1 * p;
        const double w = 0.016 * q.r * (1.0 - q.r);
        double P = (q.r * d2 - w * d1) / (d1 * d2);
        // exponentials by slice window (a lane beyond its term's bound adds an
        // exact zero, as the lane-wise form skips it)
        if ((m_g[j] >> t) & 1u) {
            asm volatile("");
            P += (1.0 - q.r) * exp(-2.772 * u);
        }
        if ((m_w[j] >> t) & 1u) {
            asm volatile("");
            P += w * exp(-0.4 * p);
        }
        if ((m_edge[j] >> t) & 1u) {
            asm volatile("");
            P = (kk[j] >= q.klo && kk[j] <= q.khi) ? P : 0.0;
        }
        se[j] += q.se * P;
        sk[j] += q.sk * P;
    }
}

// Waves per SIMD the double-precision kernel is compiled for (its register
// budget 512 / waves per lane): measured on the stagnation line, 4 (no limit,
// 120 registers) 4.88 s, 6 4.65 s, 8 4.79 s per launch.
#ifndef LRT_F64_WAVES
#define LRT_F64_WAVES 6
#endif
__global__ __launch_bounds__(kAccumThreads) __attribute__((amdgpu_waves_per_eu(LRT_F64_WAVES))) void accum_f64_kernel(
    DevLines L, DevGrid g, const CellConst *cc, const CellSpecies *cs, const int2 *ranges,
    int32_t n_cells, int32_t n_species, int32_t k_first, int32_t n_band, int32_t n_tiles,
    uint32_t b0, DevCont ct, double *eta, double *kappa)
{
    __shared__ RecF64 rec[kStage];
    int tile, c;
    block_tile_cell(b0 + blockIdx.x, n_cells, n_tiles, tile, c);
    const int lane = threadIdx.x & 63, wave = uniform_i(threadIdx.x >> 6);
    const int32_t kt = k_first + tile * kTilePoints;
    const int32_t kw = kt + wave * 64 * kPPL;
    const int32_t kend = k_first + n_band;
    const CellConst k = cc[c];
    const CellSpecies *csc = cs + (int64_t)c * n_species;
    const double *lnd_c = cr_row(L, c);
    const int2 rg = ranges[(int64_t)c * n_tiles + tile];

    double se[kPPL], sk[kPPL];
#pragma unroll
    for (int j = 0; j < kPPL; ++j) se[j] = sk[j] = 0.0;
    const uint32_t wshift = (uint32_t)(wave * kPPL);
    int32_t kk[kPPL];
#pragma unroll
    for (int j = 0; j < kPPL; ++j) kk[j] = kw + 64 * j + lane;

    for (int base = rg.x; base < rg.y; base += kStage) {
        const int64_t i = (int64_t)base + threadIdx.x;
        RecF64 rr;
        rr.klo = 1;
        rr.khi = 0;
        rr.k0 = 0;
        rr.mode = 0;
        rr.frac0 = rr.inv2g = rr.r = rr.se = rr.sk = rr.pad2 = 0.0;
        if (i < rg.y) {
            PairF64 p;
            if (pair_setup(L, g, k, csc, lnd_c, i, p)) {
                rr.klo = p.klo;
                rr.khi = p.khi;
                rr.k0 = L.k0[i];
                rr.frac0 = L.frac0[i];
                rr.inv2g = p.inv2g;
                rr.r = p.r;
                rr.se = p.se;
                rr.sk = p.sk;
                // windows of the two exponentials, one point of margin each side
                const double nu0 = L.nu0[i], gV = 0.5 / p.inv2g;
                const double wg = kF64GaussHalfWidth * gV, ww = kF64WexpHalfWidth * gV;
                const int32_t glo = (int32_t)fmax(ceil((nu0 - wg - g.nu_min) * g.inv_h) - 1.0, (double)p.klo);
                const int32_t ghi = (int32_t)fmin(floor((nu0 + wg - g.nu_min) * g.inv_h) + 1.0, (double)p.khi);
                const int32_t wlo = (int32_t)fmax(ceil((nu0 - ww - g.nu_min) * g.inv_h) - 1.0, (double)p.klo);
                const int32_t whi = (int32_t)fmin(floor((nu0 + ww - g.nu_min) * g.inv_h) + 1.0, (double)p.khi);
                const uint32_t m = slice_modes(p.klo - kt, p.khi - kt, wlo - kt, whi - kt);
                const uint32_t gm = slice_run(max(glo, p.klo) - kt, min(ghi, p.khi) - kt) & m & 0xffu;
                rr.mode = m | (gm << 24);
            }
        }
        rec[threadIdx.x] = rr;
        __syncthreads();
        const int n = min(kStage, rg.y - base);
        for (int l0 = 0; l0 < n; l0 += kBlock) {
            uint32_t mb = 0;
            if (lane < kBlock && l0 + lane < n) mb = rec[l0 + lane].mode >> wshift;
            const BlockMask todo = (BlockMask)__ballot((mb & ((1u << kPPL) - 1u)) != 0);
            BlockMask m_in[kPPL], m_edge[kPPL], m_w[kPPL], m_g[kPPL];
#pragma unroll
            for (int j = 0; j < kPPL; ++j) {
                m_in[j] = (BlockMask)__ballot(mb & (1u << j));
                m_edge[j] = (BlockMask)__ballot(mb & (1u << (8 + j)));
                m_w[j] = (BlockMask)__ballot(mb & (1u << (16 + j)));
                m_g[j] = (BlockMask)__ballot(mb & (1u << (24 + j)));
            }
            for (int g8 = 0; g8 < kBlock; g8 += 8) {
                const uint32_t gt = (uint32_t)(todo >> g8) & 0xffu;
                if (gt == 0) continue;
                uint32_t gi[kPPL], gw[kPPL], gg[kPPL], ge[kPPL];
#pragma unroll
                for (int j = 0; j < kPPL; ++j) {
                    gi[j] = (uint32_t)(m_in[j] >> g8);
                    gw[j] = (uint32_t)(m_w[j] >> g8);
                    gg[j] = (uint32_t)(m_g[j] >> g8);
                    ge[j] = (uint32_t)(m_edge[j] >> g8);
                }
                uint32_t off = (uint32_t)((l0 + g8) * (int)sizeof(RecF64));
                asm volatile("" : "+v"(off));
                const RecF64 *rg8 = (const RecF64 *)((const char *)rec + off);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if ((gt >> u) & 1u) line_terms_f64(rg8[u], u, kk, g.h, gi, gw, gg, ge, se, sk);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < kPPL; ++j) {
        const int32_t kq = kw + 64 * j + lane;
        if (kq < kend) {
            const int64_t o = (int64_t)c * n_band + (kq - k_first);
            if (ct.n_thr >= 0) {   // atomic continuum
                double ce, ck;
                continuum_point(ct, c, g.nu_min + (double)kq * g.h, ce, ck);
                se[j] += ce;
                sk[j] += ck;
            }
            eta[o] = se[j];
            kappa[o] = sk[j];
        }
    }
}

// ---------------------------------------------------------------------------
// in-window term count (the evaluation count of the metric)
// ---------------------------------------------------------------------------

__global__ void count_kernel(DevLines L, DevGrid g, const CellConst *cc, const CellSpecies *cs,
                             const int2 *band_ranges, int32_t n_cells, int32_t n_species,
                             int32_t k_first, int32_t n_band, unsigned long long *count)
{
    // lines i in the cell's candidate range for the band, grid-stride in x
    unsigned long long n = 0, nc = 0;
    for (int c = blockIdx.y; c < n_cells; c += gridDim.y) {
        const int2 rg = band_ranges[c];
        for (int64_t i = (int64_t)rg.x + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rg.y;
             i += (int64_t)gridDim.x * blockDim.x) {
            PairF64 p;
            if (pair_setup(L, g, cc[c], cs + (int64_t)c * n_species, cr_row(L, c), i, p)) {
                const int32_t a = max(p.klo, k_first), b = min(p.khi, k_first + n_band - 1);
                if (b >= a) n += (unsigned long long)(b - a + 1);
                const int32_t ca = max(p.kclo, k_first), cb = min(p.kchi, k_first + n_band - 1);
                if (cb >= ca) nc += (unsigned long long)(cb - ca + 1);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        n += __shfl_xor(n, o);
        nc += __shfl_xor(nc, o);
    }
    if ((threadIdx.x & 63) == 0) {
        if (n) atomicAdd(&count[0], n);
        if (nc) atomicAdd(&count[1], nc);
    }
}

__global__ void fill_i32_kernel(int32_t *p, int32_t v, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

__global__ void check_cells_kernel(DevCells cells, int32_t *flags)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int S = cells.n_species;
    if (t >= (int64_t)cells.n_cells * (S + 1)) return;
    const int64_t c = t / (S + 1), s = t % (S + 1);
    if (s == S) {
        const double a = cells.T_tr[c], b = cells.T_v[c], e = cells.n_e[c];
        if (!(a > 0.0 && a <= DBL_MAX && b > 0.0 && b <= DBL_MAX)) atomicOr(&flags[0], 1);
        if (!(e >= 0.0 && e <= DBL_MAX)) atomicOr(&flags[1], 1);
    } else {
        const double n = cells.N[c * S + s];
        if (!(n >= 0.0 && n <= DBL_MAX)) atomicOr(&flags[1], 1);
    }
}

__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long v, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// ---------------------------------------------------------------------------
// a7: serving.  One workgroup per (request, tile, chunk) item of an epoch's
// list, so workgroups retire all through an epoch and work on other streams
// (admissions, result copies) finds free slots without waiting for the epoch.
// An item accumulates eta/kappa of each cell of its chunk on its tile (in LDS /
// registers, never stored) and marches through them at once, producing the
// chunk's transmittance T and source S per point: I_out = I_in T + S.  The
// workgroup that completes the last chunk of a tile composes the tile's chunks
// far -> observer, and the one that completes the last tile sums the tiles:
// every sum runs in a fixed order, so nothing depends on what else shares the
// epoch or on the order in which items finish.
// ---------------------------------------------------------------------------

// One linear-j segment of length Ls (cm) from far node (fe, fk) to near node
// ne (scaled single-precision coefficients with their power-of-two scales),
// composed into the chunk's transmittance and source at ts[loc],
// ts[kTilePoints + loc]: I <- I e^-t + Ls (wf fe + wn ne), t = fk Ls.
__device__ __forceinline__ void linear_j_step(const float (&fe)[kPPL], const float (&fk)[kPPL], int fee, int fek,
                                              const float (&ne)[kPPL], int nee, double Ls, double *ts,
                                              int32_t kw, int lane)
{
    const double Lf = ldexp(Ls, fee), Ln = ldexp(Ls, nee);
    const float Lk = (float)fmin(ldexp(Ls, fek), 3.0e38);
#pragma unroll
    for (int j = 0; j < kPPL; ++j) {
        int32_t loc = kw + 64 * j + lane;
        asm volatile("" : "+v"(loc));   // recomputed here, not held across the accumulation
        const float t = fk[j] * Lk;
        const float ex = __builtin_amdgcn_exp2f(t * (float)(-kLog2e));
        float wf, wn;
        linear_j_weights_f32(t, ex, wf, wn);
        ts[loc] *= (double)ex;
        ts[kTilePoints + loc] = fma(ts[kTilePoints + loc], (double)ex, (double)(wf * fe[j]) * Lf + (double)(wn * ne[j]) * Ln);
    }
}

// Compose the chunks of the tile's points far -> observer (I <- I T + S in
// chunk order, from the far boundary's blackbody intensity when there is
// one), write I and the tile's trapezoid sum (h/2 at both window ends) in a
// fixed order: each thread's points, the wave's lanes by xor-shuffles, then
// the waves in order.  Called by the whole workgroup.
__device__ __forceinline__ void serve_compose_tile(const ServeReq &R, const DevGrid &g, int32_t tile, int32_t kw,
                                                   int lane, double *s_part)
{
    double part = 0.0;
#pragma unroll
    for (int j = 0; j < kPPL; ++j) {
        const int32_t loc = kw + 64 * j + lane;
        const int32_t t = tile * kTilePoints + loc;
        if (t < R.n_window) {
            double I = R.T_far > 0.0 ? planck_f64(g.nu_min + (double)(R.k_first + t) * g.h, R.T_far) : 0.0;
            for (int32_t m = 0; m < R.n_chunks; ++m) {
                const double *ts = R.TS + ((int64_t)tile * R.n_chunks + m) * 2 * kTilePoints;
                I = fma(I, ts[loc], ts[kTilePoints + loc]);
            }
            R.I_out[t] = I;
            const double w = (t == 0 || t == R.n_window - 1) ? 0.5 * g.h : g.h;
            part = fma(w, I, part);
        }
    }
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    if (lane == 0) s_part[kw / (64 * kPPL)] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int wv = 0; wv < kAccumThreads / 64; ++wv) sum += s_part[wv];
        R.tile_part[tile] = sum;
    }
}

__global__ __launch_bounds__(kAccumThreads) __attribute__((amdgpu_waves_per_eu(LRT_SERVE_WAVES)))
void serve_kernel(DevLines L, DevGrid g, const ServeReq *reqs, const ServeItem *items, int32_t n_species)
{
    __shared__ RecF32 rec[kStage];
    __shared__ int32_t s_last;
    __shared__ double s_part[kAccumThreads / 64];
    const int lane = threadIdx.x & 63, wave = uniform_i(threadIdx.x >> 6);
    const int32_t kw = wave * 64 * kPPL;
    {
        const ServeItem w = items[blockIdx.x];
        // the request's fields are read where used: held in registers across
        // the cell loop they would crowd out the accumulation's
        const ServeReq &R = reqs[w.req];
        const int32_t kt = R.k_first + w.tile * kTilePoints;
        const int32_t c0 = w.chunk * R.chunk_cells;
        const int32_t c1 = min(R.n_cells, c0 + R.chunk_cells);
        // the chunk's transmittance T and source S per point live in its own
        // slice of the request's buffer (each lane owns its points), not in
        // registers across the cells
        double *ts = R.TS + ((int64_t)w.tile * R.n_chunks + w.chunk) * 2 * kTilePoints;
#pragma unroll
        for (int j = 0; j < kPPL; ++j) {
            const int32_t loc = kw + 64 * j + lane;
            ts[loc] = 1.0;
            ts[kTilePoints + loc] = 0.0;
        }
        // linear-j: the chunk owns the segments that end at its cells' midpoint
        // nodes (the first from the far end, the last chunk's also to the
        // observer), so it starts one cell early for its first far node
        float pe[kPPL], pk[kPPL];
        int pee = 0, pek = 0;
        double pds = 0.0;
        const bool linear = R.linear != 0;
        const int32_t cs0 = (linear && c0 > 0) ? c0 - 1 : c0;
        for (int32_t c = cs0; c < c1; ++c) {
            float e[kPPL], kp[kPPL];
            const int ese = R.escale[2 * c + 0], esk = R.escale[2 * c + 1];
            accum_cell_tile_f32(rec, L, g, R.cc[c], R.cs + (int64_t)c * n_species,
                                R.lnd ? R.lnd + (int64_t)c * R.lnd_stride : nullptr, ese, esk,
                                R.ranges[(int64_t)c * R.n_tiles + w.tile], kt, kw, lane, e, kp);
            if (R.ct.n_thr >= 0) {
                // atomic continuum, added in double precision and rounded once
#pragma unroll
                for (int j = 0; j < kPPL; ++j) {
                    // (recomputed per cell: the per-point parts hoisted out of
                    // the cell loop would be spilled across the accumulation)
                    int32_t kk = kt + kw + 64 * j + lane;
                    asm volatile("" : "+v"(kk));
                    const double nu = g.nu_min + (double)kk * g.h;
                    double ce, ck;
                    continuum_point(R.ct, c, nu, ce, ck);
                    e[j] = (float)((double)e[j] + ldexp(ce, -ese));
                    kp[j] = (float)((double)kp[j] + ldexp(ck, -esk));
                }
            }
            const double ds = R.ds[c];
            if (!linear) {
                float dsu;
                double dsl;
                segment_scales(ds, ese, esk, dsu, dsl);
#pragma unroll
                for (int j = 0; j < kPPL; ++j) {
                    int32_t loc = kw + 64 * j + lane;
                    asm volatile("" : "+v"(loc));
                    double at, em;
                    segment_f32(e[j], kp[j], dsu, dsl, at, em);
                    ts[loc] *= at;
                    ts[kTilePoints + loc] = fma(ts[kTilePoints + loc], at, em);
                }
                continue;
            }
            if (c >= c0) {
                if (c == 0)   // far end -> first midpoint, both nodes the first cell's state
                    linear_j_step(e, kp, ese, esk, e, ese, 0.5 * ds, ts, kw, lane);
                else          // midpoint -> midpoint, kappa from the far node
                    linear_j_step(pe, pk, pee, pek, e, ese, 0.5 * (pds + ds), ts, kw, lane);
            }
#pragma unroll
            for (int j = 0; j < kPPL; ++j) {
                pe[j] = e[j];
                pk[j] = kp[j];
            }
            pee = ese;
            pek = esk;
            pds = ds;
        }
        if (linear && c1 == R.n_cells)   // last midpoint -> observer
            linear_j_step(pe, pk, pee, pek, pe, pee, 0.5 * pds, ts, kw, lane);
        // publish this chunk's T and S; the workgroup that brings the tile's
        // count to n_chunks composes the tile (device-scope fences around the
        // counter: the chunks may have run on other XCDs)
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) s_last = atomicAdd(R.done + w.tile, 1) == R.n_chunks - 1;
        __syncthreads();
        if (!s_last) return;
        __threadfence();
        serve_compose_tile(R, g, w.tile, kw, lane, s_part);
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) s_last = atomicAdd(R.done + R.n_tiles, 1) == R.n_tiles - 1;
        __syncthreads();
        if (!s_last) return;
        __threadfence();
        if (threadIdx.x == 0) {
            double sum = 0.0;
            for (int32_t t = 0; t < R.n_tiles; ++t) sum += R.tile_part[t];
            *R.I_int = sum;
            *R.I_int_host = sum;
        }
    }
}




}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_thermo(const DevSpecies &sp, const DevCells &cells, const DevWidths &wd, double M_min,
                         uint64_t species_mask, CellConst *cc, CellSpecies *cs, hipStream_t st)
{
    const int64_t n = (int64_t)cells.n_cells * cells.n_species;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(thermo_kernel, dim3(blocks_for(n, 64)), dim3(64), 0, st, sp, cells, wd, M_min,
                       species_mask, cc, cs);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n > (int64_t)UINT32_MAX) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(molq_kernel, dim3((unsigned)n), dim3(64), 0, st, sp, cells, species_mask, cs);
    return hipGetLastError();
}

hipError_t launch_ranges(const DevLines &L, const DevGrid &g, const CellConst *cc, int32_t n_cells,
                         int32_t k_first, int32_t n_band, int32_t tile_points, int2 *ranges,
                         hipStream_t st)
{
    const int32_t n_tiles = (n_band + tile_points - 1) / tile_points;
    const int64_t n = (int64_t)n_cells * n_tiles;
    hipLaunchKernelGGL(ranges_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, L, g, cc,
                       n_cells, k_first, n_band, tile_points, n_tiles, ranges);
    return hipGetLastError();
}

hipError_t launch_scale_bound(const DevBins &B, const CellConst *cc, const CellSpecies *cs,
                              const double *cont_lnb, int32_t n_cells, int32_t n_species,
                              int32_t *escale, hipStream_t st)
{
    if (n_cells == 0) return hipSuccess;
    hipLaunchKernelGGL(scale_bound_kernel, dim3(blocks_for(n_cells, 4)), dim3(256), 0, st, B, cc, cs,
                       cont_lnb, n_cells, n_species, escale);
    return hipGetLastError();
}

hipError_t launch_cont_cells(const ContThr *thr, int32_t n_thr, const ContRec *rec, int32_t n_rec,
                             const DevCells &cells, const CellSpecies *cs, const DevCR &cr,
                             uint64_t species_mask, double nu_lo, double nu_hi, double *cum, double *ff,
                             double *lnb, hipStream_t st)
{
    if (cells.n_cells == 0) return hipSuccess;
    hipLaunchKernelGGL(cont_cells_kernel, dim3(blocks_for(cells.n_cells, 64)), dim3(64), 0, st, thr,
                       n_thr, rec, n_rec, cells, cs, cr, species_mask, nu_lo, nu_hi, cum, ff, lnb);
    return hipGetLastError();
}

hipError_t launch_scale(const DevLines &L, int64_t i0, int64_t i1, const DevGrid &g,
                        const CellConst *cc, const CellSpecies *cs, int32_t n_cells,
                        int32_t n_species, const double *cont_lnb, int32_t *emax, int32_t *escale,
                        hipStream_t st)
{
    // emax must hold INT_MIN on entry (set by a fill kernel of the caller);
    // lines i0 <= i < i1 are scanned
    if (i1 > i0) {
        hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(i1 - i0, 256), min(n_cells, 65535)),
                           dim3(256), 0, st, L, i0, i1, g, cc, cs, n_cells, n_species, emax);
    }
    hipLaunchKernelGGL(scale_finish_kernel, dim3(blocks_for(2 * n_cells, 256)), dim3(256), 0, st,
                       emax, cont_lnb, 2 * n_cells, escale);
    return hipGetLastError();
}

hipError_t launch_accum_f32(const DevLines &L, const DevGrid &g, const CellConst *cc,
                            const CellSpecies *cs, const int32_t *escale, const int2 *ranges,
                            int32_t n_cells, int32_t n_species, int32_t k_first, int32_t n_band,
                            const DevCont &ct, float *eta, float *kappa, hipStream_t st)
{
    const int32_t n_tiles = (n_band + kTilePoints - 1) / kTilePoints;
    const int64_t n_blocks = (int64_t)n_tiles * n_cells;
    if (n_blocks > (int64_t)UINT32_MAX) return hipErrorInvalidConfiguration;
    for (int64_t b0 = 0; b0 < n_blocks; b0 += kMaxLaunchBlocks) {
        hipLaunchKernelGGL(accum_f32_kernel, dim3((unsigned)std::min(kMaxLaunchBlocks, n_blocks - b0)),
                           dim3(kAccumThreads), 0, st, L, g, cc, cs, escale, ranges, n_cells, n_species,
                           k_first, n_band, n_tiles, (uint32_t)b0, ct, eta, kappa);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_accum_f64(const DevLines &L, const DevGrid &g, const CellConst *cc,
                            const CellSpecies *cs, const int2 *ranges, int32_t n_cells,
                            int32_t n_species, int32_t k_first, int32_t n_band, const DevCont &ct,
                            double *eta, double *kappa, hipStream_t st)
{
    const int32_t n_tiles = (n_band + kTilePoints - 1) / kTilePoints;
    const int64_t n_blocks = (int64_t)n_tiles * n_cells;
    if (n_blocks > (int64_t)UINT32_MAX) return hipErrorInvalidConfiguration;
    for (int64_t b0 = 0; b0 < n_blocks; b0 += kMaxLaunchBlocks) {
        hipLaunchKernelGGL(accum_f64_kernel, dim3((unsigned)std::min(kMaxLaunchBlocks, n_blocks - b0)),
                           dim3(kAccumThreads), 0, st, L, g, cc, cs, ranges, n_cells, n_species, k_first,
                           n_band, n_tiles, (uint32_t)b0, ct, eta, kappa);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_count(const DevLines &L, const DevGrid &g, const CellConst *cc,
                        const CellSpecies *cs, const int2 *band_ranges, int32_t n_cells,
                        int32_t n_species, int32_t k_first, int32_t n_band,
                        unsigned long long *count, hipStream_t st)
{
    if (L.n == 0) return hipSuccess;
    hipLaunchKernelGGL(count_kernel, dim3(64, min(n_cells, 65535)), dim3(256), 0, st, L, g, cc, cs,
                       band_ranges, n_cells, n_species, k_first, n_band, count);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t launch_check_cells(const DevCells &cells, int32_t *flags, hipStream_t st)
{
    const int64_t n = (int64_t)cells.n_cells * (cells.n_species + 1);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(check_cells_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, cells, flags);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}


hipError_t launch_serve(const DevLines &L, const DevGrid &g, const ServeReq *reqs,
                        const ServeItem *items, int32_t n_items, int32_t n_species, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(serve_kernel, dim3((unsigned)n_items), dim3(kAccumThreads), 0, st, L, g, reqs, items,
                       n_species);
    return hipGetLastError();
}

}  // namespace lrt
