// Host-side context of liblrt, shared by lrt_host.cpp and lrt_serve.cpp.
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/lrt.h"
#include "lrt_internal.h"

namespace lrt {

// Device buffer owned by the context (hipFree on release).
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

}  // namespace lrt

struct lrt_ctx {
    using DBuf = lrt::DBuf;
    using DevSpecies = lrt::DevSpecies;
    int device = 0;
    std::string err;

    // species
    int n_species = 0;
    std::vector<int32_t> sp_kind;
    std::vector<double> sp_mass;
    DBuf d_kind, d_mass, d_lev_off, d_lev_E, d_lev_g, d_el_off, d_el_T, d_el_g, d_el_J,
        d_vib_off, d_vib_G, d_vib_B, d_vib_D;
    DevSpecies sp{};
    double M_min = 0.0;
    std::vector<int64_t> h_el_off;       // host copy of the electronic-state offsets
    std::vector<int64_t> h_lev_off;      // host copies of the atomic level tables
    std::vector<double> h_lev_E, h_lev_g;

    // atomic continuum: thresholds sorted by nu, records, per-cell sums
    int n_cont_rec = 0, n_cont_thr = 0;
    DBuf d_cont_thr, d_cont_rec;         // ContThr[n_thr], ContRec[n_rec]
    DBuf d_cont_cum, d_cont_ff, d_cont_lnb;   // per cell: [2][n_thr+1], [2], [2]

    // QSS-CR atoms: records (device pointers into d_cr_tab), per-species
    // record index, collider weights, per-(cell, atom) populations and ln
    // departures ([n_cells][n_cr][cr_LS])
    int n_cr = 0, cr_LS = 0, cr_max_l = 0;
    std::vector<int32_t> h_cr_slot, h_cr_nlev;
    DBuf d_cr_rec, d_cr_tab, d_cr_slot, d_cr_w, d_cr_pop, d_cr_lnd;
    // per line (sorted order) its upper / lower level (-1: none), and the packed
    // offsets into a cell's departure row the line setup reads (built when both
    // the levels and the CR atoms are set)
    std::vector<int32_t> h_lev_u, h_lev_l;
    DBuf d_line_lev;
    // per scale bin the departure-row offsets of the levels of its lines
    // (CSR; -1 for lines with Boltzmann populations)
    DBuf d_bin_lev_off, d_bin_lev;
    bool line_lev_ready = false;

    // lines (sorted by nu0 on the host, resident on the device)
    int64_t n_lines = -1;
    std::vector<int64_t> h_line_order;   // sorted position -> caller's index
    std::vector<int32_t> h_bin_u, h_bin_l;   // scale bin of each line's upper / lower level
    std::vector<double> h_nu0;   // sorted centres, host copy for k0/frac0
    DBuf d_nu0, d_seta0, d_skap0, d_Eu_ev, d_Eu_rot, d_El_ev, d_El_rot, d_lngu, d_species, d_k0, d_frac0;
    std::vector<int32_t> h_spc;   // sorted order: species and upper-level energy
    std::vector<double> h_Eu;

    // Lorentz widths: per-species ionization energies (empty: uniform law),
    // per-line natural width and Stark coefficient
    std::vector<double> h_Eion;
    DBuf d_Eion, d_gN, d_gS;
    double gN_max = 0.0, gS_max = 1.0;
    bool lines_grid_ready = false;

    // grid
    bool have_grid = false;
    double nu_min = 0, nu_max = 0, h = 0;
    int64_t n_points = 0, band_points = 0;

    // cells
    int64_t n_cells = -1;
    DBuf d_T_tr, d_T_v, d_N, d_n_e;
    DBuf d_cc, d_cs;
    bool thermo_ready = false;
    DBuf d_emax, d_escale;
    DBuf d_bin_sp, d_bin_Ev, d_bin_Er, d_bin_aeta, d_bin_akap, d_bin_nlo, d_bin_nhi;
    int64_t n_bins = 0;
    bool scale_ready = false;

    // rays
    int64_t n_rays = -1, n_wall = 0;
    int64_t rays_cells = 0;   // number of cells the geometry expects
    std::vector<int64_t> h_off;
    std::vector<int32_t> h_cell;
    std::vector<double> h_ds, h_weight;
    std::vector<int64_t> h_wall_off, h_ray_wall;
    DBuf d_off, d_cell, d_ds, d_weight, d_wall_off;
    DBuf d_Tfar;              // per-ray far-boundary temperature (valid when have_Tfar)
    bool have_Tfar = false;
    int march_scheme = 0;     // lrt_march_scheme

    // workspace
    DBuf w_ranges, w_eta, w_kappa, w_partials, w_Iband, w_Itot, w_qband, w_count;
    DBuf w_gen_sys, w_gen_re2, w_gen_cnt, w_gen_off;   // rovibronic line generation

    // profiler: event pairs per kernel family
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[LRT_K_COUNT];

    void clear_events()
    {
        for (auto &v : ev) {
            for (auto &p : v) {
                (void)hipEventDestroy(p.first);
                (void)hipEventDestroy(p.second);
            }
            v.clear();
        }
    }
    ~lrt_ctx() { clear_events(); }
};

namespace lrt {

// Record the message and return the status (ctx == NULL: the thread's
// create-time message).
lrt_status fail(lrt_ctx *c, lrt_status s, const char *fmt, ...);
// Allocate (and fill from src, if not NULL) a device buffer.
lrt_status upload(lrt_ctx *c, DBuf &b, const void *src, size_t bytes);
// Grow-only workspace.
lrt_status ensure(lrt_ctx *c, DBuf &b, size_t bytes);
// Lines placed on the grid (k0, frac0).
lrt_status prepare_lines(lrt_ctx *c);
// Lines on the grid, per-cell constants (and scales when need_scale).
lrt_status prepare(lrt_ctx *c, hipStream_t st, bool need_scale, bool force = false);
DevLines dev_lines(const lrt_ctx *c);
// QSS-CR: device view, line-to-level packing, per-cell solve (after thermo).
DevCR dev_cr(const lrt_ctx *c);
lrt_status cr_build_line_levels(lrt_ctx *c);
lrt_status cr_run(lrt_ctx *c, const DevCells &cells, hipStream_t st);

// Launch `fn` (returning hipError_t) on stream st, bracketed by events when
// the context profiles.
template <class F>
hipError_t timed(lrt_ctx *c, int kernel, hipStream_t st, F fn)
{
    if (!c->prof) return fn();
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) {
        (void)hipEventDestroy(a);
        return e;
    }
    (void)hipEventRecord(a, st);
    e = fn();
    (void)hipEventRecord(b, st);
    c->ev[kernel].push_back({a, b});
    return e;
}
inline DevWidths dev_widths(const lrt_ctx *c)
{
    return DevWidths{c->h_Eion.empty() ? nullptr : c->d_Eion.as<double>(), c->gN_max, c->gS_max};
}
lrt_status line_widths(lrt_ctx *c);
lrt_status band_range(lrt_ctx *c, int64_t band, int32_t &k_first, int32_t &n_band);
lrt_status march_range(lrt_ctx *c, int32_t k_first, int32_t n_band, lrt_precision prec, const void *eta,
                       const void *kappa, const int32_t *escale, double *I_out, double *I_int_out,
                       hipStream_t st, double *partials, int64_t cap);
// Device address of the static scratch array on `device` (current device),
// looked up once per device; lrt_march_noalloc's buffer.
hipError_t noalloc_scratch_init(int device);
inline DevGrid dev_grid(const lrt_ctx *c)
{
    return DevGrid{c->nu_min, c->h, (int32_t)c->n_points, 1.0 / c->h};
}

}  // namespace lrt

#define LRT_HIP(ctx, call)                                                                     \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::lrt::fail((ctx), LRT_E_DEVICE, "%s: %s (%s:%d)", #call,                   \
                               hipGetErrorString(e_), __FILE__, __LINE__);                     \
    } while (0)
