// Internal declarations shared by the host side (lrt_host.cpp) and the
// gfx950 kernels (lrt_accum.hip, lrt_march.hip, lrt_cr.hip).  Not part of
// the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lrt {

// CODATA exact constants in CGS units.
constexpr double kPlanck = 6.62607015e-27;  // erg s
constexpr double kLight = 2.99792458e10;    // cm s^-1
constexpr double kBoltz = 1.380649e-16;     // erg K^-1
constexpr double kC2 = kPlanck * kLight / kBoltz;  // second radiation constant, cm K
constexpr double kPi = 3.14159265358979323846;

// Accumulation tile: 4 waves of 64 lanes, each lane owns kPPL grid points,
// one workgroup owns 256 * kPPL consecutive points of one cell.  The
// accumulation kernels are compiled for LRT_ACCUM_WAVES waves per SIMD
// (register budget 512 / waves per lane).  Measured on the 400-cell, 2.2M-line
// stagnation case: 2 points per lane at 8 waves per SIMD beats 4 points at 4
// waves by 22% (1385 ms vs 1785 ms per launch).  At 8 waves the FP64 staging
// code fits the 64-register budget only if the compiler's machine-level loop
// invariant motion is off (it hoists FP64 constants into registers that then
// spill); the build passes that option for the accumulation's unit.
#ifndef LRT_ACCUM_PPL
#define LRT_ACCUM_PPL 2
#endif
#ifndef LRT_ACCUM_WAVES
#define LRT_ACCUM_WAVES 8
#endif
#ifndef LRT_SERVE_WAVES
#define LRT_SERVE_WAVES 8
#endif
#ifndef LRT_ACCUM_THREADS
#define LRT_ACCUM_THREADS 256
#endif
constexpr int kAccumThreads = LRT_ACCUM_THREADS;
constexpr int kPPL = LRT_ACCUM_PPL;
constexpr int kTilePoints = kAccumThreads * kPPL;
// Line records staged in LDS per round: one per thread.
constexpr int kStage = kAccumThreads;

// March tile: one workgroup of 4 waves; each wave marches one ray over one
// chunk of 64 x PPT consecutive points, PPT per lane, and the waves share no
// state.  Smaller chunks keep more cell rows in L2 while a chunk's rays run
// (a row is 8 B per point), at more per-segment work per point, so the tile
// follows how often the rays cross a cell: from kMarchReuseNarrow segments per
// cell on, 128-point chunks (PPT 2) and 4 rays per workgroup; below, 256-point
// chunks (PPT 4) and 4 consecutive chunks of one ray per workgroup.  March time per step of the large
// axisymmetric slice (131,072 rays, 391 segments per cell), by chunk points /
// rays per workgroup: 1024 / 1 (4 points per lane): 826 ms; 256 / 1: 794;
// 256 / 2: 794; 256 / 4: 712; 256 / 8: 717; 128 / 4: 641-651; 128 / 8: 656;
// 64 / 4: 909; 64 / 8: 928.  On the 256 x 128-cell case (8,192 rays, few
// segments per cell), per band: 128 / 4: 97 ms; 256 / 4: 88 ms; 256-point
// chunks, 4 of one ray per workgroup: 84 ms.
constexpr int kMarchThreads = 256;
constexpr int64_t kMarchReuseNarrow = 128;

// Points per lane of the march for a ray set with n_seg segments over n_cells cells.
inline int32_t march_points_per_lane(int64_t n_seg, int64_t n_cells)
{
    return n_seg >= kMarchReuseNarrow * n_cells ? 2 : 4;
}

// Workgroups per launch of a kernel whose grid can be large (the accumulation
// over cells x tiles, the march over rays x chunks): a dispatch counts at most
// 2^32 - 1 work-items, so such grids go in launches of 2^23 workgroups of 256
// (a multiple of the 8 XCDs, so every launch starts on XCD 0 as one launch would).
constexpr int64_t kMaxLaunchBlocks = int64_t(1) << 23;

// Species level tables on the device (flattened).
struct DevSpecies {
    int n;
    const int32_t *kind;
    const double *mass;
    const int64_t *lev_off;   // [n+1]
    const double *lev_E, *lev_g;
    const int64_t *el_off;    // [n+1]
    const double *el_T, *el_g;
    const int32_t *el_Jmax;
    const int64_t *vib_off;   // [n_el_total+1]
    const double *vib_G, *vib_B, *vib_D;
};

// Line list on the device, sorted by nu0, structure of arrays.
struct DevLines {
    int64_t n;
    const double *nu0, *Eu_ev, *Eu_rot, *El_ev, *El_rot, *lngu;
    // cell-independent strength factors: seta0 = 1e-7 (hc/4pi) nu0 A (W cm),
    // skap0 = A / (8 pi c nu0^2) (cm^2 s^-1 ... per unit population)
    const double *seta0, *skap0;
    // Lorentz HWHM of line i in cell c: gN[i] + gS[i] gL(c) + gW(c, species),
    // gL(c) = 1e-16 n_e (T_v/1e4)^0.33 (gN = 0, gS = 1, gW = 0: that law)
    const double *gN, *gS;
    const int32_t *species;
    // grid-relative centre: nu0 = nu_min + k0 h + frac0 (frac0 exact to a
    // few units of its last place)
    const int32_t *k0;
    const double *frac0;
    // QSS-CR level populations (NULL: Boltzmann for every line): lev[i] = -1
    // for a line without levels, else the offsets of its upper (low 16 bits)
    // and lower (high 16 bits) level into a cell's row of lnd, the ln
    // departures from Boltzmann, lnd_stride entries per cell
    const int32_t *lev = nullptr;
    const double *lnd = nullptr;
    int32_t lnd_stride = 0;
};

// Atomic continuum.  A bound-free threshold (sorted by nu over all records)
// and its level; s3 = sigma0 nu_thr^3 (the cross section is s3 / nu^3 above).
struct ContThr {
    double nu, E, g, s3;
    int32_t rec, lev;   // record, level index in the atom's table
};
struct ContRec {
    int32_t species, ion;
    double E_ion, Q_ion, z4inv;   // z4inv = 1/z^4
    double peach[8];
};
// What the accumulation needs per cell: with m = number of thresholds <= nu,
//   kappa_c = cum[0][m] / nu^3 + kff(nu), eta_c = B(nu, T_v) (cum[1][m] / nu^3 + kff(nu)),
//   kff(nu) = (ff[0] nu_H / nu + ff[1]) nu_H^3 / nu^3.
struct DevCont {
    int32_t n_thr;          // < 0: no continuum
    const ContThr *thr;
    const double *cum;      // [n_cells][2][n_thr+1]
    const double *ff;       // [n_cells][2]
    const double *T_v;      // [n_cells]
};
constexpr double kNuH = 1e7 / 91.1267;   // hydrogen ground-state threshold, cm^-1

// QSS collisional-radiative species (Sec. 2.1 CR model): an atom's table
// levels or a diatomic molecule's electronic states.  States 0..n_model-1
// are solved for; states n_model..n_lev-1 stay in Boltzmann ratio
// (T_v, T_tr) with state n_model-1.  Rate tables are Arrhenius triples
// (C, n, E_a) of the forward processes: hpie/eie [l][l][3] at [lo][hi] for
// lo -> hi, A [l][l] at [hi][lo], eii/ce (atoms) and hpid/eid (molecules)
// [l][3] per state.  texp[2m], texp[2m+1]: forward / backward temperature
// T_tr^a T_v^(1-a) of mechanism m (HPIE, EIE, EII, CE, HPID, EID).
constexpr int kCRMaxLevels = 64;   // one lane per state
struct CRRec {
    int32_t species, ion, partner, partner_ion;
    int32_t n_model, n_lev, pn_lev, kind;   // kind: 1 atom, 2 molecule
    int32_t diss_x, diss_y;                 // molecule: products, -1 without dissociation
    int32_t nx_lev, ny_lev;                 // level counts of atomic products (0: constant Q)
    int64_t lev0, plev0;                    // atom: first level of the atom / its partner
    int64_t e0;                             // molecule: first electronic state
    int64_t x_lev0, y_lev0;                 // first levels of atomic products
    double E_ion, Q_ion, pE_ion, pQ_ion, nu_cut;
    double Q_x, Q_y, E_diss, mu;            // mu: reduced mass of the products, g
    double texp[12];
    const double *hpie, *eie, *A, *eii, *ce, *hpid, *eid;
};
struct DevCR {
    int32_t n;                 // atoms (0: off)
    int32_t LS;                // entries per (cell, atom) row of pop / lnd
    const CRRec *rec;
    const int32_t *slot;       // per species: its atom record, or -1
    const double *collider_w;  // per species: weight among the heavy colliders
    double *pop;               // [n_cells][n][LS] level populations, cm^-3
    double *lnd;               // [n_cells][n][LS] ln(population / Boltzmann population)
};

// Upper bounds of the line peaks for the per-cell scale, from level-energy
// bins of the line list (one entry per (species, E_ev bin, E_rot bin) of the
// upper levels and one per bin of the lower levels).  For every line i in a
// bin, with Ev <= E_ev,i and Er <= E_rot,i:
//   ln(seta0_i g_u,i / nu0_i) <= a_eta,  ln(skap0_i g_u,i / nu0_i) <= a_kap
// (a_eta = -inf for lower-level bins).  With QSS-CR populations the bound of
// bin b also takes the largest ln departure of the levels its lines belong to:
// offsets lev[lev_off[b] .. lev_off[b+1]-1] into the cell's row of lnd (-1: a
// line with Boltzmann populations); lev_off NULL: no departures.
struct DevBins {
    int32_t n;
    const int32_t *species;
    const double *Ev, *Er, *a_eta, *a_kap;
    const int32_t *lev_off = nullptr, *lev = nullptr;
    const double *lnd = nullptr;
    int32_t lnd_stride = 0;
    // optional window [win_a, win_b] (cm^-1, nu_lo non-NULL): only bins whose
    // line centres [nu_lo, nu_hi] meet the cell's candidate range of the
    // window count
    const double *nu_lo = nullptr, *nu_hi = nullptr;
    double win_a = 0.0, win_b = 0.0;
};

struct DevGrid {
    double nu_min, h;
    int32_t n_points;
    double inv_h;   // 1/h (approximate bounds only; exact windows divide by h)
};

struct DevCells {
    int32_t n_cells, n_species;
    const double *T_tr, *T_v, *N, *n_e;
};

// Per-cell constants written by the thermo kernel.
struct CellConst {
    double beta_v, beta_tr;  // c2 / T_v, c2 / T_tr
    double gL;               // Lorentz HWHM, cm^-1
    double cand_G, cand_A;   // line-skip bound: |nu - nu0| <= cand_G + cand_A nu0
};

// Whether species s radiates under a species mask (bit s; 0: every species).
__host__ __device__ inline bool species_on(uint64_t mask, int s)
{
    return mask == 0 || (s < 64 && ((mask >> s) & 1ull));
}

// Per (cell, species) constants written by the thermo kernel.
struct CellSpecies {
    double lnNQ;   // ln(N_s / Q_s), -inf when the species carries no population
    double dop;    // Doppler HWHM per unit nu0: (7.16233e-7/2) sqrt(T_tr / M_s)
    double gW;     // van der Waals HWHM of the species' lines, cm^-1 (0 unless full widths)
};

// Full Lorentz widths: per-species ionization energies (NULL: off) and the
// largest per-line natural width and Stark coefficient (for the skip bound).
struct DevWidths {
    const double *E_ion;
    double gN_max, gS_max;
};

// Rays on the device.
struct DevRays {
    int32_t n_rays;
    const int64_t *off;     // [n_rays+1] into cell / ds
    const int32_t *cell;
    const double *ds;
    // rays per wall point when every wall point has that many (wall-major
    // ray order), else 0: the march then visits the rays direction-major
    int32_t per_wall = 0;
};

// One admitted line-of-sight request as the serving kernels see it.
struct ServeReq {
    int32_t n_cells, k_first, n_window, n_tiles, n_chunks, chunk_cells;
    const CellConst *cc;
    const CellSpecies *cs;
    const int32_t *escale;   // [cell][2]
    const double *ds;        // [cell], far -> observer
    const int2 *ranges;      // [cell][tile]
    double *TS;              // [tile][chunk][2][kTilePoints]: transmittance, source
    double *I_out;           // [n_window]
    int32_t *done;           // [n_tiles + 1]: chunks composed per tile, then tiles composed
    double *tile_part;       // [n_tiles]: trapezoid sum of each tile's points
    double *I_int;           // [1]
    double *I_int_host;      // the request's slot in pinned host memory
    DevCont ct;              // the request's atomic continuum (n_thr < 0: none)
    double T_far;            // solid far boundary temperature (0: free)
    int32_t linear;          // segment scheme: 0 cell-constant, 1 linear-j
    int32_t lnd_stride;      // QSS-CR: entries per cell of lnd
    const double *lnd;       // QSS-CR: [cell][lnd_stride] ln departures, or NULL
};

// One unit of serving work: the cells of one chunk on one tile of a request.
struct ServeItem {
    int32_t req, tile, chunk;
};

// ---- kernel launchers (lrt_accum.hip, lrt_march.hip) ----
hipError_t launch_thermo(const DevSpecies &sp, const DevCells &cells, const DevWidths &wd, double M_min,
                         uint64_t species_mask, CellConst *cc, CellSpecies *cs, hipStream_t st);

hipError_t launch_ranges(const DevLines &L, const DevGrid &g, const CellConst *cc,
                         int32_t n_cells, int32_t k_first, int32_t n_band, int32_t tile_points,
                         int2 *ranges, hipStream_t st);

hipError_t launch_scale_bound(const DevBins &B, const CellConst *cc, const CellSpecies *cs,
                              const double *cont_lnb, int32_t n_cells, int32_t n_species,
                              int32_t *escale, hipStream_t st);
hipError_t launch_cont_cells(const ContThr *thr, int32_t n_thr, const ContRec *rec, int32_t n_rec,
                             const DevCells &cells, const CellSpecies *cs, const DevCR &cr,
                             uint64_t species_mask, double nu_lo, double nu_hi, double *cum, double *ff,
                             double *lnb, hipStream_t st);

// QSS-CR populations of every (cell, atom) (lrt_cr.hip); max_l / max_lev:
// largest n_model / n_lev over the records.
hipError_t launch_cr(const DevSpecies &sp, const DevCells &cells, const DevCR &cr, int32_t max_l,
                     int32_t max_lev, const CellSpecies *cs, hipStream_t st);
hipError_t launch_scale(const DevLines &L, int64_t i0, int64_t i1, const DevGrid &g,
                        const CellConst *cc, const CellSpecies *cs, int32_t n_cells,
                        int32_t n_species, const double *cont_lnb, int32_t *emax, int32_t *escale,
                        hipStream_t st);

hipError_t launch_accum_f32(const DevLines &L, const DevGrid &g, const CellConst *cc,
                            const CellSpecies *cs, const int32_t *escale, const int2 *ranges,
                            int32_t n_cells, int32_t n_species, int32_t k_first, int32_t n_band,
                            const DevCont &ct, float *eta, float *kappa, hipStream_t st);

hipError_t launch_accum_f64(const DevLines &L, const DevGrid &g, const CellConst *cc,
                            const CellSpecies *cs, const int2 *ranges, int32_t n_cells,
                            int32_t n_species, int32_t k_first, int32_t n_band, const DevCont &ct,
                            double *eta, double *kappa, hipStream_t st);

hipError_t launch_count(const DevLines &L, const DevGrid &g, const CellConst *cc,
                        const CellSpecies *cs, const int2 *band_ranges, int32_t n_cells,
                        int32_t n_species, int32_t k_first, int32_t n_band,
                        unsigned long long *count, hipStream_t st);

hipError_t launch_march(bool fp32, bool linear, int32_t ppt, const DevRays &rays, const DevGrid &g,
                        int32_t k_first, int32_t n_band, const void *eta, const void *kappa,
                        const int32_t *escale, const double *T_far, double *I_out,
                        double *partials, int32_t n_chunks, hipStream_t st);

hipError_t launch_reduce_rows(const double *partials, int32_t n_rows, int32_t n_cols,
                              double *out, hipStream_t st);

hipError_t launch_wall_sum(const double *I_int, const double *weight, const int64_t *wall_off,
                           int32_t n_wall, double *q, hipStream_t st);

hipError_t launch_add(double *acc, const double *x, int32_t n, hipStream_t st);

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);
// Cell-state validation on the device: flags[0] |= 1 for a temperature that is
// not positive and finite, flags[1] |= 1 for a density or n_e that is not
// finite and >= 0 (flags zeroed by the caller).
hipError_t launch_check_cells(const DevCells &cells, int32_t *flags, hipStream_t st);

hipError_t launch_serve(const DevLines &L, const DevGrid &g, const ServeReq *reqs,
                        const ServeItem *items, int32_t n_items, int32_t n_species, hipStream_t st);

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t st);

}  // namespace lrt
