// Host side of liblrt: context, validation, uploads, line preparation, ray
// geometry (Sec. 2.2.3) and the band loop that drives the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <numeric>
#include <unordered_map>
#include <string>
#include <vector>

#include "../../include/lrt.h"
#include "lrt_ctx.h"
#include "lrt_geom.h"
#include "lrt_internal.h"

using namespace lrt;




namespace lrt {

lrt_status fail(lrt_ctx *c, lrt_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf; else host_error() = buf;
    return s;
}



lrt_status upload(lrt_ctx *c, DBuf &b, const void *src, size_t bytes)
{
    b.release();
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        return fail(c, LRT_E_OOM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    b.bytes = bytes;
    if (src) {
        e = hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(c, LRT_E_DEVICE, "hipMemcpy: %s", hipGetErrorString(e));
    }
    return LRT_OK;
}

template <class T>
lrt_status upload_vec(lrt_ctx *c, DBuf &b, const std::vector<T> &v)
{
    return upload(c, b, v.empty() ? nullptr : v.data(), v.size() * sizeof(T));
}

// grow-only workspace
lrt_status ensure(lrt_ctx *c, DBuf &b, size_t bytes)
{
    if (b.bytes >= bytes && b.p) return LRT_OK;
    return upload(c, b, nullptr, bytes);
}

}  // namespace lrt

namespace {

bool finite_all(const double *p, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

// ===========================================================================
// public API
// ===========================================================================

extern "C" {

const char *lrt_version(void) { return "0.1.0"; }

const char *lrt_status_string(lrt_status s)
{
    switch (s) {
    case LRT_OK: return "ok";
    case LRT_E_ARG: return "invalid argument";
    case LRT_E_OOM: return "out of memory";
    case LRT_E_DEVICE: return "device error";
    case LRT_E_BUDGET: return "over budget";
    case LRT_E_NOT_READY: return "not ready";
    case LRT_E_STATE: return "invalid state";
    }
    return "unknown status";
}

lrt_status lrt_create(int device, lrt_ctx **out)
{
    if (!out) return fail(nullptr, LRT_E_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return fail(nullptr, LRT_E_DEVICE, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (device < 0 || device >= n) return fail(nullptr, LRT_E_ARG, "device %d out of range (%d devices)", device, n);
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, LRT_E_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
    // the static scratch of lrt_march_noalloc: its address on this device
    e = noalloc_scratch_init(device);
    if (e != hipSuccess) return fail(nullptr, LRT_E_DEVICE, "scratch address: %s", hipGetErrorString(e));
    lrt_ctx *c = new (std::nothrow) lrt_ctx();
    if (!c) return fail(nullptr, LRT_E_OOM, "context allocation failed");
    c->device = device;
    *out = c;
    return LRT_OK;
}

void lrt_destroy(lrt_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    delete ctx;
}

const char *lrt_last_error(const lrt_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : host_error().c_str();
}

lrt_status lrt_set_species(lrt_ctx *c, int n, const lrt_species *sp)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (n < 1 || !sp) return fail(c, LRT_E_ARG, "n_species must be >= 1 and species non-NULL");
    std::vector<int32_t> kind(n), el_J;
    std::vector<double> mass(n), lev_E, lev_g, el_T, el_g, vib_G, vib_B, vib_D;
    std::vector<int64_t> lev_off(1, 0), el_off(1, 0), vib_off(1, 0);
    double M_min = INFINITY;
    for (int s = 0; s < n; ++s) {
        const lrt_species &x = sp[s];
        if (x.kind != LRT_KIND_NONE && x.kind != LRT_KIND_ATOM && x.kind != LRT_KIND_MOLECULE)
            return fail(c, LRT_E_ARG, "species %d: unknown kind %d", s, x.kind);
        if (!(x.mass > 0.0) || !std::isfinite(x.mass))
            return fail(c, LRT_E_ARG, "species %d: mass must be positive", s);
        kind[s] = x.kind;
        mass[s] = x.mass;
        if (x.kind == LRT_KIND_ATOM) {
            if (x.n_levels < 1 || !x.level_E || !x.level_g)
                return fail(c, LRT_E_ARG, "species %d: atom needs levels", s);
            for (int j = 0; j < x.n_levels; ++j) {
                if (!std::isfinite(x.level_E[j]) || !(x.level_g[j] > 0.0) || !std::isfinite(x.level_g[j]))
                    return fail(c, LRT_E_ARG, "species %d level %d: bad energy or degeneracy", s, j);
                lev_E.push_back(x.level_E[j]);
                lev_g.push_back(x.level_g[j]);
            }
        }
        if (x.kind == LRT_KIND_MOLECULE) {
            if (x.n_el < 1 || !x.el_T || !x.el_g || !x.el_nv || !x.el_Jmax || !x.vib_G || !x.vib_B || !x.vib_D)
                return fail(c, LRT_E_ARG, "species %d: molecule needs electronic / vibrational tables", s);
            int64_t pos = 0;
            for (int e = 0; e < x.n_el; ++e) {
                if (x.el_nv[e] < 1 || x.el_Jmax[e] < 0 || !std::isfinite(x.el_T[e]) || !(x.el_g[e] > 0.0))
                    return fail(c, LRT_E_ARG, "species %d state %d: bad electronic entry", s, e);
                if ((int64_t)x.el_nv[e] * ((int64_t)x.el_Jmax[e] + 1) > (int64_t(1) << 30))
                    return fail(c, LRT_E_ARG, "species %d state %d: more than 2^30 (v, J) terms", s, e);
                el_T.push_back(x.el_T[e]);
                el_g.push_back(x.el_g[e]);
                el_J.push_back(x.el_Jmax[e]);
                for (int v = 0; v < x.el_nv[e]; ++v, ++pos) {
                    if (!std::isfinite(x.vib_G[pos]) || !std::isfinite(x.vib_B[pos]) || !std::isfinite(x.vib_D[pos]))
                        return fail(c, LRT_E_ARG, "species %d: non-finite vibrational entry", s);
                    vib_G.push_back(x.vib_G[pos]);
                    vib_B.push_back(x.vib_B[pos]);
                    vib_D.push_back(x.vib_D[pos]);
                }
                vib_off.push_back((int64_t)vib_G.size());
            }
        }
        lev_off.push_back((int64_t)lev_E.size());
        el_off.push_back((int64_t)el_T.size());
        if (x.kind != LRT_KIND_NONE) M_min = std::min(M_min, x.mass);
    }
    lrt_status st;
    if ((st = upload_vec(c, c->d_kind, kind)) || (st = upload_vec(c, c->d_mass, mass)) ||
        (st = upload_vec(c, c->d_lev_off, lev_off)) || (st = upload_vec(c, c->d_lev_E, lev_E)) ||
        (st = upload_vec(c, c->d_lev_g, lev_g)) || (st = upload_vec(c, c->d_el_off, el_off)) ||
        (st = upload_vec(c, c->d_el_T, el_T)) || (st = upload_vec(c, c->d_el_g, el_g)) ||
        (st = upload_vec(c, c->d_el_J, el_J)) || (st = upload_vec(c, c->d_vib_off, vib_off)) ||
        (st = upload_vec(c, c->d_vib_G, vib_G)) || (st = upload_vec(c, c->d_vib_B, vib_B)) ||
        (st = upload_vec(c, c->d_vib_D, vib_D)))
        return st;
    c->n_species = n;
    c->sp_kind = kind;
    c->sp_mass = mass;
    c->h_lev_off = lev_off;
    c->h_el_off = el_off;
    c->h_lev_E = lev_E;
    c->h_lev_g = lev_g;
    c->n_cont_rec = c->n_cont_thr = 0;   // continuum records refer to the old table
    c->h_Eion.clear();                   // so does the Lorentz model
    c->n_cr = 0;                         // and the QSS-CR atoms
    c->h_cr_slot.clear();
    c->h_cr_nlev.clear();
    c->h_lev_u.clear();
    c->h_lev_l.clear();
    c->line_lev_ready = false;
    c->M_min = std::isfinite(M_min) ? M_min : 1.0;
    c->sp = DevSpecies{n, c->d_kind.as<int32_t>(), c->d_mass.as<double>(), c->d_lev_off.as<int64_t>(),
                       c->d_lev_E.as<double>(), c->d_lev_g.as<double>(), c->d_el_off.as<int64_t>(),
                       c->d_el_T.as<double>(), c->d_el_g.as<double>(), c->d_el_J.as<int32_t>(),
                       c->d_vib_off.as<int64_t>(), c->d_vib_G.as<double>(), c->d_vib_B.as<double>(),
                       c->d_vib_D.as<double>()};
    c->thermo_ready = c->scale_ready = false;
    c->n_lines = -1;   // lines refer to species indices: must be set again
    c->n_cells = -1;
    return LRT_OK;
}

lrt_status lrt_set_lines(lrt_ctx *c, const lrt_lines *Lin)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (c->n_species < 1) return fail(c, LRT_E_STATE, "set species before lines");
    if (!Lin || Lin->n < 0) return fail(c, LRT_E_ARG, "lines NULL or negative count");
    if (Lin->n >= INT_MAX) return fail(c, LRT_E_ARG, "at most 2^31-2 lines");
    const int64_t n = Lin->n;
    if (n > 0 && (!Lin->nu0 || !Lin->A || !Lin->Eu_ev || !Lin->Eu_rot || !Lin->El_ev || !Lin->El_rot || !Lin->gu ||
                  !Lin->gl || !Lin->species))
        return fail(c, LRT_E_ARG, "line arrays must be non-NULL");
    // device arrays (a line list generated on the device): host copies, then
    // the same validation, sort and preparation as host arrays
    std::vector<double> hd[8];
    std::vector<int32_t> hs;
    lrt_lines Lh = *Lin;
    if (Lin->on_device && n > 0) {
        const double *src[8] = {Lin->nu0, Lin->A, Lin->Eu_ev, Lin->Eu_rot, Lin->El_ev, Lin->El_rot, Lin->gu, Lin->gl};
        for (int k = 0; k < 8; ++k) {
            hd[k].resize(n);
            LRT_HIP(c, hipMemcpy(hd[k].data(), src[k], n * 8, hipMemcpyDeviceToHost));
        }
        hs.resize(n);
        LRT_HIP(c, hipMemcpy(hs.data(), Lin->species, n * 4, hipMemcpyDeviceToHost));
        Lh.nu0 = hd[0].data(); Lh.A = hd[1].data(); Lh.Eu_ev = hd[2].data(); Lh.Eu_rot = hd[3].data();
        Lh.El_ev = hd[4].data(); Lh.El_rot = hd[5].data(); Lh.gu = hd[6].data(); Lh.gl = hd[7].data();
        Lh.species = hs.data();
    }
    const lrt_lines *L = &Lh;
    for (int64_t i = 0; i < n; ++i) {
        if (!(L->nu0[i] > 0.0) || !std::isfinite(L->nu0[i]))
            return fail(c, LRT_E_ARG, "line %lld: nu0 must be positive and finite", (long long)i);
        if (!(L->A[i] >= 0.0) || !std::isfinite(L->A[i]))
            return fail(c, LRT_E_ARG, "line %lld: A must be >= 0", (long long)i);
        if (!(L->gu[i] >= 1.0) || !(L->gl[i] >= 1.0) || !std::isfinite(L->gu[i]) || !std::isfinite(L->gl[i]))
            return fail(c, LRT_E_ARG, "line %lld: degeneracies must be >= 1", (long long)i);
        if (!std::isfinite(L->Eu_ev[i]) || !std::isfinite(L->Eu_rot[i]) || !std::isfinite(L->El_ev[i]) ||
            !std::isfinite(L->El_rot[i]))
            return fail(c, LRT_E_ARG, "line %lld: non-finite level energy", (long long)i);
        const int s = L->species[i];
        if (s < 0 || s >= c->n_species || c->sp_kind[s] == LRT_KIND_NONE)
            return fail(c, LRT_E_ARG, "line %lld: species %d is not a radiating species", (long long)i, s);
    }
    std::vector<int64_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return L->nu0[a] < L->nu0[b]; });
    std::vector<double> nu0(n), seta0(n), skap0(n), Eue(n), Eur(n), Ele(n), Elr(n), lngu(n);
    std::vector<int32_t> spc(n);
    for (int64_t j = 0; j < n; ++j) {
        const int64_t i = idx[j];
        nu0[j] = L->nu0[i];
        // eta_i = (hc/4pi) N_u A nu0 phi (W after the 1e-7);
        // kappa_i = A (N_l g_u/g_l)(1 - e^{-x}) phi / (8 pi c nu0^2)
        seta0[j] = (1e-7 * kPlanck * kLight / (4.0 * kPi)) * L->nu0[i] * L->A[i];
        skap0[j] = L->A[i] / ((8.0 * kPi * kLight) * L->nu0[i] * L->nu0[i]);
        Eue[j] = L->Eu_ev[i];
        Eur[j] = L->Eu_rot[i];
        Ele[j] = L->El_ev[i];
        Elr[j] = L->El_rot[i];
        lngu[j] = std::log(L->gu[i]);
        spc[j] = L->species[i];
    }
    // level-energy bins for the per-cell scale bound (1000 cm^-1 wide; the
    // bound then exceeds the true peak by at most e^{(beta_v + beta_tr) 1000}),
    // and each line's upper and lower bin
    std::vector<int32_t> b_sp, bin_u, bin_l;
    std::vector<double> b_Ev, b_Er, b_aeta, b_akap;
    {
        constexpr double kBinE = 1000.0;
        std::unordered_map<uint64_t, int64_t> slot;
        slot.reserve(4096);
        // key: (species, upper/lower, E_ev bin, E_rot bin), bins offset to be non-negative
        // returns the bin's index, -1 when the energies are out of range
        auto bin = [&](int32_t s, int lower, double Ev, double Er, double aeta, double akap) -> int32_t {
            const double fe = std::floor(Ev / kBinE) + 8388608.0, fr = std::floor(Er / kBinE) + 8388608.0;
            if (!(fe >= 0.0 && fe < 16777216.0 && fr >= 0.0 && fr < 16777216.0)) return -1;
            const uint64_t key = ((uint64_t)(2 * s + lower) << 48) | ((uint64_t)fe << 24) | (uint64_t)fr;
            auto it = slot.find(key);
            if (it == slot.end()) {
                slot.emplace(key, (int64_t)b_sp.size());
                b_sp.push_back(s);
                b_Ev.push_back(Ev);
                b_Er.push_back(Er);
                b_aeta.push_back(aeta);
                b_akap.push_back(akap);
                return (int32_t)(b_sp.size() - 1);
            }
            const int64_t k = it->second;
            b_Ev[k] = std::min(b_Ev[k], Ev);
            b_Er[k] = std::min(b_Er[k], Er);
            b_aeta[k] = std::max(b_aeta[k], aeta);
            b_akap[k] = std::max(b_akap[k], akap);
            return (int32_t)k;
        };
        const double ninf = -std::numeric_limits<double>::infinity();
        bin_u.assign(n, -1);
        bin_l.assign(n, -1);
        for (int64_t j = 0; j < n; ++j) {
            if (!(seta0[j] > 0.0)) continue;   // A = 0: the line has no strength
            const double ln_nu = std::log(nu0[j]);
            const double ae = std::log(seta0[j]) + lngu[j] - ln_nu;
            const double ak = std::log(skap0[j]) + lngu[j] - ln_nu;
            bin_u[j] = bin(spc[j], 0, Eue[j], Eur[j], ae, ak);
            bin_l[j] = bin(spc[j], 1, Ele[j], Elr[j], ninf, ak);
            if (bin_u[j] < 0 || bin_l[j] < 0)
                return fail(c, LRT_E_ARG, "line %lld: level energy beyond +-8e9 cm^-1", (long long)j);
        }
    }
    // per bin the range of line centres of its lines (upper and lower
    // levels): a spectral window's scale bound visits only the bins whose
    // lines can reach it
    std::vector<double> b_nlo(b_sp.size(), std::numeric_limits<double>::infinity());
    std::vector<double> b_nhi(b_sp.size(), -std::numeric_limits<double>::infinity());
    for (int64_t j = 0; j < n; ++j)
        for (int32_t b : {bin_u[j], bin_l[j]})
            if (b >= 0) {
                b_nlo[b] = std::min(b_nlo[b], nu0[j]);
                b_nhi[b] = std::max(b_nhi[b], nu0[j]);
            }
    lrt_status st;
    if ((st = upload_vec(c, c->d_bin_sp, b_sp)) || (st = upload_vec(c, c->d_bin_Ev, b_Ev)) ||
        (st = upload_vec(c, c->d_bin_Er, b_Er)) || (st = upload_vec(c, c->d_bin_aeta, b_aeta)) ||
        (st = upload_vec(c, c->d_bin_akap, b_akap)) || (st = upload_vec(c, c->d_bin_nlo, b_nlo)) ||
        (st = upload_vec(c, c->d_bin_nhi, b_nhi)))
        return st;
    c->n_bins = (int64_t)b_sp.size();
    if ((st = upload_vec(c, c->d_nu0, nu0)) || (st = upload_vec(c, c->d_seta0, seta0)) ||
        (st = upload_vec(c, c->d_skap0, skap0)) ||
        (st = upload_vec(c, c->d_Eu_ev, Eue)) || (st = upload_vec(c, c->d_Eu_rot, Eur)) ||
        (st = upload_vec(c, c->d_El_ev, Ele)) || (st = upload_vec(c, c->d_El_rot, Elr)) ||
        (st = upload_vec(c, c->d_lngu, lngu)) || (st = upload_vec(c, c->d_species, spc)))
        return st;
    c->h_nu0.swap(nu0);
    c->h_spc = spc;
    c->h_line_order.swap(idx);
    c->h_bin_u.swap(bin_u);
    c->h_bin_l.swap(bin_l);
    c->h_lev_u.clear();   // line levels refer to the old list
    c->h_lev_l.clear();
    c->line_lev_ready = false;
    c->h_Eu.resize(n);
    for (int64_t j = 0; j < n; ++j) c->h_Eu[j] = Eue[j] + Eur[j];
    c->n_lines = n;
    c->lines_grid_ready = false;
    c->scale_ready = false;
    c->thermo_ready = false;
    return line_widths(c);
}

lrt_status lrt_set_lorentz(lrt_ctx *c, const double *E_ion)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (c->n_species < 1) return fail(c, LRT_E_STATE, "set species before the Lorentz model");
    std::vector<double> e;
    if (E_ion) {
        e.assign(E_ion, E_ion + c->n_species);
        for (int s = 0; s < c->n_species; ++s)
            if (!(e[s] >= 0.0) || !std::isfinite(e[s])) return fail(c, LRT_E_ARG, "E_ion[%d] must be >= 0", s);
        lrt_status st = upload_vec(c, c->d_Eion, e);
        if (st) return st;
    }
    c->h_Eion.swap(e);
    return c->n_lines >= 0 ? line_widths(c) : LRT_OK;
}

lrt_status lrt_set_continuum(lrt_ctx *c, int n, const lrt_continuum *cont)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (c->n_species < 1) return fail(c, LRT_E_STATE, "set species before the continuum");
    if (n < 0 || (n > 0 && !cont)) return fail(c, LRT_E_ARG, "n must be >= 0 and cont non-NULL");
    std::vector<ContThr> thr;
    std::vector<ContRec> rec(n);
    for (int q = 0; q < n; ++q) {
        const lrt_continuum &x = cont[q];
        if (x.species < 0 || x.species >= c->n_species || c->sp_kind[x.species] != LRT_KIND_ATOM)
            return fail(c, LRT_E_ARG, "continuum %d: species %d is not an atom", q, x.species);
        if (x.ion < 0 || x.ion >= c->n_species) return fail(c, LRT_E_ARG, "continuum %d: ion out of range", q);
        if (!(x.E_ion > 0.0) || !(x.Q_ion > 0.0) || !(x.z > 0.0) || !std::isfinite(x.E_ion) ||
            !std::isfinite(x.Q_ion) || !std::isfinite(x.z))
            return fail(c, LRT_E_ARG, "continuum %d: E_ion, Q_ion and z must be positive", q);
        for (int j = 0; j < 8; ++j)
            if (!std::isfinite(x.peach[j])) return fail(c, LRT_E_ARG, "continuum %d: non-finite fit coefficient", q);
        rec[q].species = x.species;
        rec[q].ion = x.ion;
        rec[q].E_ion = x.E_ion;
        rec[q].Q_ion = x.Q_ion;
        rec[q].z4inv = 1.0 / (x.z * x.z * x.z * x.z);
        std::copy(x.peach, x.peach + 8, rec[q].peach);
        const int64_t l0 = c->h_lev_off[x.species], l1 = c->h_lev_off[x.species + 1];
        if (l1 > l0 && !x.sigma0) return fail(c, LRT_E_ARG, "continuum %d: sigma0 NULL", q);
        for (int64_t i = l0; i < l1; ++i) {
            const double s0 = x.sigma0[i - l0];
            if (!(s0 >= 0.0) || !std::isfinite(s0))
                return fail(c, LRT_E_ARG, "continuum %d level %lld: sigma0 must be >= 0", q, (long long)(i - l0));
            const double nu = x.E_ion - c->h_lev_E[i];
            if (s0 == 0.0 || !(nu > 0.0)) continue;   // no bound-free from this level
            thr.push_back(ContThr{nu, c->h_lev_E[i], c->h_lev_g[i], s0 * nu * nu * nu, q, (int32_t)(i - l0)});
        }
    }
    std::stable_sort(thr.begin(), thr.end(), [](const ContThr &a, const ContThr &b) { return a.nu < b.nu; });
    lrt_status st;
    if (n > 0 && ((st = upload(c, c->d_cont_rec, rec.data(), rec.size() * sizeof(ContRec))) ||
                  (st = upload(c, c->d_cont_thr, thr.empty() ? nullptr : thr.data(), thr.size() * sizeof(ContThr)))))
        return st;
    c->n_cont_rec = n;
    c->n_cont_thr = (int)thr.size();
    c->thermo_ready = c->scale_ready = false;
    return LRT_OK;
}

lrt_status lrt_set_grid(lrt_ctx *c, double nu_min, double nu_max, int64_t n_points, int64_t band_points)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (!(nu_min > 0.0) || !(nu_max > nu_min) || !std::isfinite(nu_max))
        return fail(c, LRT_E_ARG, "grid needs 0 < nu_min < nu_max");
    if (n_points < 2 || n_points >= ((int64_t)1 << 31))
        return fail(c, LRT_E_ARG, "n_points must be in [2, 2^31)");
    if (band_points < 1) return fail(c, LRT_E_ARG, "band_points must be >= 1");
    c->nu_min = nu_min;
    c->nu_max = nu_max;
    c->n_points = n_points;
    c->band_points = std::min(band_points, n_points);
    c->h = (nu_max - nu_min) / (double)(n_points - 1);
    c->have_grid = true;
    c->lines_grid_ready = false;
    c->scale_ready = false;
    return LRT_OK;
}

}  // extern "C"

// Cells given as device arrays: copied on the device, then validated there
// (one flag per rule); on failure the context is left without cells.
static lrt_status set_cells_device(lrt_ctx *c, const lrt_cells *x)
{
    const int64_t nc = x->n_cells, S = x->n_species;
    c->n_cells = 0;
    lrt_status st;
    if ((st = upload(c, c->d_T_tr, nullptr, nc * 8)) || (st = upload(c, c->d_T_v, nullptr, nc * 8)) ||
        (st = upload(c, c->d_N, nullptr, nc * S * 8)) || (st = upload(c, c->d_n_e, nullptr, nc * 8)) ||
        (st = upload(c, c->d_cc, nullptr, nc * sizeof(CellConst))) ||
        (st = upload(c, c->d_cs, nullptr, nc * S * sizeof(CellSpecies))) ||
        (st = upload(c, c->d_emax, nullptr, nc * 2 * sizeof(int32_t))) ||
        (st = upload(c, c->d_escale, nullptr, nc * 2 * sizeof(int32_t))) ||
        (st = ensure(c, c->w_count, 16)))
        return st;
    LRT_HIP(c, hipMemcpy(c->d_T_tr.p, x->T_tr, nc * 8, hipMemcpyDeviceToDevice));
    LRT_HIP(c, hipMemcpy(c->d_T_v.p, x->T_v, nc * 8, hipMemcpyDeviceToDevice));
    LRT_HIP(c, hipMemcpy(c->d_N.p, x->N, nc * S * 8, hipMemcpyDeviceToDevice));
    LRT_HIP(c, hipMemcpy(c->d_n_e.p, x->n_e, nc * 8, hipMemcpyDeviceToDevice));
    int32_t *flags = c->w_count.as<int32_t>();
    LRT_HIP(c, launch_fill_i32(flags, 0, 2, nullptr));
    const DevCells cells{(int32_t)nc, (int)S, c->d_T_tr.as<double>(), c->d_T_v.as<double>(),
                         c->d_N.as<double>(), c->d_n_e.as<double>()};
    LRT_HIP(c, launch_check_cells(cells, flags, nullptr));
    int32_t h[2] = {0, 0};
    LRT_HIP(c, hipMemcpy(h, flags, sizeof(h), hipMemcpyDeviceToHost));
    if (h[0]) return fail(c, LRT_E_ARG, "device cells: temperatures must be positive and finite");
    if (h[1]) return fail(c, LRT_E_ARG, "device cells: N and n_e must be finite and >= 0");
    c->n_cells = nc;
    c->thermo_ready = false;
    c->scale_ready = false;
    return LRT_OK;
}

extern "C" {

lrt_status lrt_set_cells(lrt_ctx *c, const lrt_cells *x)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (c->n_species < 1) return fail(c, LRT_E_STATE, "set species before cells");
    if (!x || x->n_cells < 1) return fail(c, LRT_E_ARG, "cells NULL or empty");
    if (x->n_cells >= INT_MAX) return fail(c, LRT_E_ARG, "too many cells");
    if (x->n_species != c->n_species)
        return fail(c, LRT_E_ARG, "cells have %d species, table has %d", x->n_species, c->n_species);
    if (!x->T_tr || !x->T_v || !x->N || !x->n_e) return fail(c, LRT_E_ARG, "cell arrays must be non-NULL");
    const int64_t nc = x->n_cells, S = x->n_species;
    if (x->on_device) return set_cells_device(c, x);
    for (int64_t i = 0; i < nc; ++i) {
        if (!(x->T_tr[i] > 0.0) || !(x->T_v[i] > 0.0) || !std::isfinite(x->T_tr[i]) || !std::isfinite(x->T_v[i]))
            return fail(c, LRT_E_ARG, "cell %lld: temperatures must be positive and finite", (long long)i);
        if (!(x->n_e[i] >= 0.0) || !std::isfinite(x->n_e[i]))
            return fail(c, LRT_E_ARG, "cell %lld: n_e must be >= 0", (long long)i);
        for (int64_t s = 0; s < S; ++s)
            if (!(x->N[i * S + s] >= 0.0) || !std::isfinite(x->N[i * S + s]))
                return fail(c, LRT_E_ARG, "cell %lld species %lld: N must be >= 0", (long long)i, (long long)s);
    }
    lrt_status st;
    if ((st = upload(c, c->d_T_tr, x->T_tr, nc * 8)) || (st = upload(c, c->d_T_v, x->T_v, nc * 8)) ||
        (st = upload(c, c->d_N, x->N, nc * S * 8)) || (st = upload(c, c->d_n_e, x->n_e, nc * 8)) ||
        (st = upload(c, c->d_cc, nullptr, nc * sizeof(CellConst))) ||
        (st = upload(c, c->d_cs, nullptr, nc * S * sizeof(CellSpecies))) ||
        (st = upload(c, c->d_emax, nullptr, nc * 2 * sizeof(int32_t))) ||
        (st = upload(c, c->d_escale, nullptr, nc * 2 * sizeof(int32_t))))
        return st;
    c->n_cells = nc;
    c->thermo_ready = false;
    c->scale_ready = false;
    return LRT_OK;
}

static lrt_status upload_rays(lrt_ctx *c)
{
    c->have_Tfar = false;   // a new ray set starts with free far boundaries
    lrt_status st;
    if ((st = upload_vec(c, c->d_off, c->h_off)) || (st = upload_vec(c, c->d_cell, c->h_cell)) ||
        (st = upload_vec(c, c->d_ds, c->h_ds)) || (st = upload_vec(c, c->d_weight, c->h_weight)) ||
        (st = upload_vec(c, c->d_wall_off, c->h_wall_off)))
        return st;
    return LRT_OK;
}

lrt_status lrt_set_rays_slab(lrt_ctx *c, int64_t n_cells, const double *dx, int n_mu)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (n_cells < 1 || n_cells >= INT_MAX || !dx || n_mu < 0)
        return fail(c, LRT_E_ARG, "slab needs n_cells >= 1, dx, n_mu >= 0");
    for (int64_t i = 0; i < n_cells; ++i)
        if (!(dx[i] > 0.0) || !std::isfinite(dx[i])) return fail(c, LRT_E_ARG, "dx[%lld] must be positive", (long long)i);
    std::vector<double> mu, w;
    if (n_mu > 0) gauss_legendre_01(n_mu, mu, w);
    c->h_off.assign(1, 0);
    c->h_cell.clear();
    c->h_ds.clear();
    c->h_weight.clear();
    c->h_ray_wall.clear();
    for (int r = 0; r <= n_mu; ++r) {
        const double m = (r == 0) ? 1.0 : mu[r - 1];
        for (int64_t i = 0; i < n_cells; ++i) {
            c->h_cell.push_back((int32_t)i);
            c->h_ds.push_back(r == 0 ? dx[i] : dx[i] / m);
        }
        c->h_off.push_back((int64_t)c->h_cell.size());
        c->h_weight.push_back(r == 0 ? 0.0 : 2.0 * kPi * w[r - 1] * mu[r - 1]);
        c->h_ray_wall.push_back(0);
    }
    c->h_wall_off = {0, (int64_t)n_mu + 1};
    lrt_status st = upload_rays(c);
    if (st) return st;
    c->n_rays = n_mu + 1;
    c->n_wall = 1;
    c->rays_cells = n_cells;
    return LRT_OK;
}

lrt_status lrt_set_rays_axi(lrt_ctx *c, int nx, int nr, double Lx, double R, int n_wall,
                            const double *wall_r, int n_mu, int n_phi)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (nx < 1 || nr < 1 || !(Lx > 0.0) || !(R > 0.0) || n_wall < 1 || !wall_r || n_mu < 1 || n_phi < 1)
        return fail(c, LRT_E_ARG, "axisymmetric rays need positive sizes");
    if ((int64_t)nx * nr >= INT_MAX) return fail(c, LRT_E_ARG, "grid too large");
    for (int w = 0; w < n_wall; ++w)
        if (!(wall_r[w] >= 0.0) || !(wall_r[w] < R)) return fail(c, LRT_E_ARG, "wall_r[%d] outside [0, R)", w);
    std::vector<double> mu, W;
    gauss_legendre_01(n_mu, mu, W);
    c->h_off.assign(1, 0);
    c->h_cell.clear();
    c->h_ds.clear();
    c->h_weight.clear();
    c->h_ray_wall.clear();
    c->h_wall_off.assign(1, 0);
    std::vector<int32_t> cell;
    std::vector<double> ds;
    // phi_j and 2 pi - phi_j = phi_{n_phi-1-j} give identical segment lists
    // (rho(s) depends on cos phi and sin^2 phi): trace j < n_phi/2 with twice
    // the weight, plus the self-symmetric middle azimuth when n_phi is odd.
    const int n_half = (n_phi + 1) / 2;
    for (int w = 0; w < n_wall; ++w) {
        for (int i = 0; i < n_mu; ++i) {
            for (int j = 0; j < n_half; ++j) {
                const double phi = (j + 0.5) * 2.0 * kPi / n_phi;
                const double mult = (2 * j + 1 == n_phi) ? 1.0 : 2.0;
                cell.clear();
                ds.clear();
                if (!traverse_axi(nx, nr, Lx, R, wall_r[w], mu[i], phi, cell, ds))
                    return fail(c, LRT_E_ARG, "ray traversal did not terminate (wall %d, mu %d, phi %d)", w, i, j);
                for (int64_t m = (int64_t)cell.size() - 1; m >= 0; --m) {   // far -> wall
                    c->h_cell.push_back(cell[m]);
                    c->h_ds.push_back(ds[m]);
                }
                c->h_off.push_back((int64_t)c->h_cell.size());
                c->h_weight.push_back(mult * W[i] * mu[i] * 2.0 * kPi / n_phi);
                c->h_ray_wall.push_back(w);
            }
        }
        c->h_wall_off.push_back((int64_t)c->h_weight.size());
    }
    lrt_status st = upload_rays(c);
    if (st) return st;
    c->n_rays = (int64_t)c->h_weight.size();
    c->n_wall = n_wall;
    c->rays_cells = (int64_t)nx * nr;
    return LRT_OK;
}

lrt_status lrt_set_rays_axi_fibonacci(lrt_ctx *c, int nx, int nr, double Lx, double R, int n_wall,
                                      const double *wall_r, int n_los, int n_polar, int n_azim)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (nx < 1 || nr < 1 || !(Lx > 0.0) || !(R > 0.0) || n_wall < 1 || !wall_r || n_los < 3 || n_polar < 1 ||
        n_azim < 1)
        return fail(c, LRT_E_ARG, "Fibonacci rays need positive sizes and n_los >= 3");
    if ((int64_t)nx * nr >= INT_MAX) return fail(c, LRT_E_ARG, "grid too large");
    for (int w = 0; w < n_wall; ++w)
        if (!(wall_r[w] >= 0.0) || !(wall_r[w] < R)) return fail(c, LRT_E_ARG, "wall_r[%d] outside [0, R)", w);
    std::vector<double> dir, wt;
    fibonacci_rule(n_los, n_polar, n_azim, dir, wt);
    c->h_off.assign(1, 0);
    c->h_cell.clear();
    c->h_ds.clear();
    c->h_weight.clear();
    c->h_ray_wall.clear();
    c->h_wall_off.assign(1, 0);
    std::vector<int32_t> cell;
    std::vector<double> ds;
    for (int w = 0; w < n_wall; ++w) {
        for (size_t q = 0; q < wt.size(); ++q) {
            const double mu = std::min(1.0, dir[3 * q]);
            const double phi = std::atan2(dir[3 * q + 2], dir[3 * q + 1]);
            cell.clear();
            ds.clear();
            if (!traverse_axi(nx, nr, Lx, R, wall_r[w], mu, phi, cell, ds))
                return fail(c, LRT_E_ARG, "ray traversal did not terminate (wall %d, LOS %zu)", w, q);
            for (int64_t m = (int64_t)cell.size() - 1; m >= 0; --m) {   // far -> wall
                c->h_cell.push_back(cell[m]);
                c->h_ds.push_back(ds[m]);
            }
            c->h_off.push_back((int64_t)c->h_cell.size());
            c->h_weight.push_back(wt[q]);
            c->h_ray_wall.push_back(w);
        }
        c->h_wall_off.push_back((int64_t)c->h_weight.size());
    }
    lrt_status st = upload_rays(c);
    if (st) return st;
    c->n_rays = (int64_t)c->h_weight.size();
    c->n_wall = n_wall;
    c->rays_cells = (int64_t)nx * nr;
    return LRT_OK;
}

lrt_status lrt_set_march(lrt_ctx *c, lrt_march_scheme scheme)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (scheme != LRT_MARCH_CELL && scheme != LRT_MARCH_LINEAR_J)
        return fail(c, LRT_E_ARG, "unknown march scheme %d", (int)scheme);
    c->march_scheme = (int)scheme;
    return LRT_OK;
}

lrt_status lrt_set_far_temperature(lrt_ctx *c, const double *T_far, int64_t n)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (c->n_rays < 1) return fail(c, LRT_E_STATE, "rays not set");
    if (n == 0) {
        c->have_Tfar = false;
        return LRT_OK;
    }
    if (!T_far || (n != 1 && n != c->n_rays))
        return fail(c, LRT_E_ARG, "T_far needs 1 or n_rays = %lld values", (long long)c->n_rays);
    std::vector<double> t((size_t)c->n_rays);
    for (int64_t r = 0; r < c->n_rays; ++r) {
        const double v = T_far[n == 1 ? 0 : r];
        if (!(v >= 0.0) || !std::isfinite(v)) return fail(c, LRT_E_ARG, "T_far[%lld] must be >= 0", (long long)r);
        t[(size_t)r] = v;
    }
    lrt_status st = upload_vec(c, c->d_Tfar, t);
    if (st) return st;
    c->have_Tfar = true;
    return LRT_OK;
}

lrt_status lrt_get_sizes(const lrt_ctx *c, int64_t *n_cells, int64_t *n_rays, int64_t *n_wall,
                         int64_t *n_points, int64_t *n_bands, int64_t *band_points)
{
    if (!c) return LRT_E_ARG;
    if (n_cells) *n_cells = std::max<int64_t>(c->n_cells, 0);
    if (n_rays) *n_rays = std::max<int64_t>(c->n_rays, 0);
    if (n_wall) *n_wall = c->n_wall;
    if (n_points) *n_points = c->have_grid ? c->n_points : 0;
    if (band_points) *band_points = c->have_grid ? c->band_points : 0;
    if (n_bands) *n_bands = c->have_grid ? (c->n_points + c->band_points - 1) / c->band_points : 0;
    return LRT_OK;
}

lrt_status lrt_get_ray(const lrt_ctx *cc, int64_t r, int64_t cap, int32_t *cell, double *ds, int64_t *n,
                       double *weight, int64_t *wall)
{
    lrt_ctx *c = const_cast<lrt_ctx *>(cc);
    if (!c) return LRT_E_ARG;
    if (r < 0 || r >= c->n_rays) return fail(c, LRT_E_ARG, "ray %lld out of range", (long long)r);
    const int64_t a = c->h_off[r], b = c->h_off[r + 1];
    if (n) *n = b - a;
    if (weight) *weight = c->h_weight[r];
    if (wall) *wall = c->h_ray_wall[r];
    if (cell || ds) {
        if (cap < b - a) return fail(c, LRT_E_ARG, "capacity %lld < %lld segments", (long long)cap, (long long)(b - a));
        for (int64_t m = a; m < b; ++m) {
            if (cell) cell[m - a] = c->h_cell[m];
            if (ds) ds[m - a] = c->h_ds[m];
        }
    }
    return LRT_OK;
}

}  // extern "C"

// ===========================================================================
// preparation and the compute entry points
// ===========================================================================

namespace lrt {

lrt_status prepare_lines(lrt_ctx *c)
{
    if (c->n_species < 1) return fail(c, LRT_E_STATE, "species not set");
    if (c->n_lines < 0) return fail(c, LRT_E_STATE, "lines not set");
    if (!c->have_grid) return fail(c, LRT_E_STATE, "grid not set");
    if (!c->lines_grid_ready) {
        // nu0 = nu_min + k0 h + frac0 with frac0 correctly rounded: k0 h and
        // nu_min + k0 h are carried as unevaluated sums (two-product by fma,
        // two-sum), so frac0 is the difference of nu0 and the exact grid point.
        const int64_t n = c->n_lines;
        std::vector<int32_t> k0(n);
        std::vector<double> fr(n);
        for (int64_t i = 0; i < n; ++i) {
            const double nu0 = c->h_nu0[i];
            double kk = std::nearbyint((nu0 - c->nu_min) / c->h);
            kk = std::max(-16777216.0, std::min(16777216.0, kk));
            const double p = kk * c->h;
            const double pe = std::fma(kk, c->h, -p);
            const double s = c->nu_min + p;
            const double bb = s - c->nu_min;
            const double se = (c->nu_min - (s - bb)) + (p - bb);
            fr[i] = (nu0 - s) - (se + pe);
            k0[i] = (int32_t)kk;
        }
        lrt_status r;
        if ((r = upload_vec(c, c->d_k0, k0)) || (r = upload_vec(c, c->d_frac0, fr))) return r;
        c->lines_grid_ready = true;
    }
    return LRT_OK;
}

lrt_status prepare(lrt_ctx *c, hipStream_t st, bool need_scale, bool force)
{
    if (force) {
        c->thermo_ready = false;
        c->scale_ready = false;
    }
    lrt_status r0 = prepare_lines(c);
    if (r0) return r0;
    if (c->n_cells < 1) return fail(c, LRT_E_STATE, "cells not set");
    if (!c->thermo_ready) {
        DevCells cells{(int32_t)c->n_cells, c->n_species, c->d_T_tr.as<double>(), c->d_T_v.as<double>(),
                       c->d_N.as<double>(), c->d_n_e.as<double>()};
        LRT_HIP(c, timed(c, LRT_K_THERMO, st, [&] {
                    return launch_thermo(c->sp, cells, dev_widths(c), c->M_min, 0, c->d_cc.as<CellConst>(),
                                         c->d_cs.as<CellSpecies>(), st);
                }));
        lrt_status rc = cr_run(c, cells, st);   // QSS-CR populations (Sec. 2.1)
        if (rc) return rc;
        if (c->n_cont_rec > 0) {
            lrt_status r;
            const size_t nc = (size_t)c->n_cells;
            if ((r = ensure(c, c->d_cont_cum, nc * 2 * (c->n_cont_thr + 1) * sizeof(double))) ||
                (r = ensure(c, c->d_cont_ff, nc * 2 * sizeof(double))) ||
                (r = ensure(c, c->d_cont_lnb, nc * 2 * sizeof(double))))
                return r;
            LRT_HIP(c, launch_cont_cells(c->d_cont_thr.as<ContThr>(), c->n_cont_thr, c->d_cont_rec.as<ContRec>(),
                                         c->n_cont_rec, cells, c->d_cs.as<CellSpecies>(), dev_cr(c), 0ull,
                                         c->nu_min, c->nu_max, c->d_cont_cum.as<double>(),
                                         c->d_cont_ff.as<double>(), c->d_cont_lnb.as<double>(), st));
        }
        c->thermo_ready = true;
    }
    if (need_scale && !c->scale_ready) {
        DevLines L{c->n_lines, c->d_nu0.as<double>(), c->d_Eu_ev.as<double>(),
                   c->d_Eu_rot.as<double>(), c->d_El_ev.as<double>(), c->d_El_rot.as<double>(),
                   c->d_lngu.as<double>(), c->d_seta0.as<double>(), c->d_skap0.as<double>(),
                   c->d_gN.as<double>(), c->d_gS.as<double>(), c->d_species.as<int32_t>(),
                   c->d_k0.as<int32_t>(), c->d_frac0.as<double>()};
        DevGrid g = dev_grid(c);
        DevBins B{(int32_t)c->n_bins, c->d_bin_sp.as<int32_t>(), c->d_bin_Ev.as<double>(),
                  c->d_bin_Er.as<double>(), c->d_bin_aeta.as<double>(), c->d_bin_akap.as<double>()};
        if (c->n_cr > 0 && c->line_lev_ready) {
            B.lev_off = c->d_bin_lev_off.as<int32_t>();
            B.lev = c->d_bin_lev.as<int32_t>();
            B.lnd = c->d_cr_lnd.as<double>();
            B.lnd_stride = c->n_cr * c->cr_LS;
        }
        LRT_HIP(c, timed(c, LRT_K_SCALE, st, [&] {
                    return launch_scale_bound(B, c->d_cc.as<CellConst>(), c->d_cs.as<CellSpecies>(),
                                              c->n_cont_rec > 0 ? c->d_cont_lnb.as<double>() : nullptr,
                                              (int32_t)c->n_cells, c->n_species, c->d_escale.as<int32_t>(),
                                              st);
                }));
        c->scale_ready = true;
    }
    return LRT_OK;
}

// Per-line natural width and Stark coefficient in cm^-1 (Sec. 2.2.1): for an
// atom with an ionization energy, gN = 1e7 * 5.9e-6 nm / lambda^2 =
// 5.9e-13 nu0^2 and gS = 1e7 * 1.69e3 / dE^2.623 (the lambda^2 of the nm-form
// coefficient cancels against 1e7 / lambda^2), dE = max(E_ion - E_u, E_H/25);
// every other line gN = 0, gS = 1 (the uniform law).
lrt_status line_widths(lrt_ctx *c)
{
    const int64_t n = std::max<int64_t>(c->n_lines, 0);
    constexpr double kEH = 109678.77;   // ionization energy of hydrogen, cm^-1
    std::vector<double> gN(n, 0.0), gS(n, 1.0);
    double gN_max = 0.0, gS_max = n > 0 ? 0.0 : 1.0;
    for (int64_t i = 0; i < n; ++i) {
        const int s = c->h_spc[i];
        if (!c->h_Eion.empty() && c->sp_kind[s] == LRT_KIND_ATOM && c->h_Eion[s] > 0.0) {
            const double nu0 = c->h_nu0[i];
            const double dE = std::max(c->h_Eion[s] - c->h_Eu[i], kEH / 25.0);
            gN[i] = 5.9e-13 * nu0 * nu0;
            gS[i] = 1.69e10 / std::pow(dE, 2.623);
        }
        gN_max = std::max(gN_max, gN[i]);
        gS_max = std::max(gS_max, gS[i]);
    }
    lrt_status st;
    if ((st = upload_vec(c, c->d_gN, gN)) || (st = upload_vec(c, c->d_gS, gS))) return st;
    c->gN_max = gN_max;
    c->gS_max = gS_max;
    c->thermo_ready = c->scale_ready = false;
    return LRT_OK;
}

DevLines dev_lines(const lrt_ctx *c)
{
    DevLines L{c->n_lines, c->d_nu0.as<double>(), c->d_Eu_ev.as<double>(),
               c->d_Eu_rot.as<double>(), c->d_El_ev.as<double>(), c->d_El_rot.as<double>(),
               c->d_lngu.as<double>(), c->d_seta0.as<double>(), c->d_skap0.as<double>(),
               c->d_gN.as<double>(), c->d_gS.as<double>(), c->d_species.as<int32_t>(),
               c->d_k0.as<int32_t>(), c->d_frac0.as<double>()};
    if (c->n_cr > 0 && c->line_lev_ready) {
        L.lev = c->d_line_lev.as<int32_t>();
        L.lnd = c->d_cr_lnd.as<double>();
        L.lnd_stride = c->n_cr * c->cr_LS;
    }
    return L;
}

lrt_status band_range(lrt_ctx *c, int64_t band, int32_t &k_first, int32_t &n_band)
{
    const int64_t nb = (c->n_points + c->band_points - 1) / c->band_points;
    if (band < 0 || band >= nb) return fail(c, LRT_E_ARG, "band %lld out of range [0, %lld)", (long long)band, (long long)nb);
    k_first = (int32_t)(band * c->band_points);
    n_band = (int32_t)std::min<int64_t>(c->band_points, c->n_points - k_first);
    return LRT_OK;
}

// Coefficients of every cell on grid points [k_first, k_first + n_band).
lrt_status coeffs_range(lrt_ctx *c, int32_t k_first, int32_t n_band, lrt_precision prec, void *eta,
                        void *kappa, int32_t *escale, hipStream_t st)
{
    if (prec != LRT_FP64 && prec != LRT_FP32_COMP) return fail(c, LRT_E_ARG, "unknown precision %d", (int)prec);
    if (!eta || !kappa) return fail(c, LRT_E_ARG, "eta and kappa must be non-NULL");
    lrt_status r;
    if ((r = prepare(c, st, prec == LRT_FP32_COMP))) return r;
    const int32_t n_tiles = (n_band + kTilePoints - 1) / kTilePoints;
    if ((r = ensure(c, c->w_ranges, (size_t)c->n_cells * n_tiles * sizeof(int2)))) return r;
    const DevLines L = dev_lines(c);
    const DevGrid g = dev_grid(c);
    const int32_t nc = (int32_t)c->n_cells;
    LRT_HIP(c, timed(c, LRT_K_RANGES, st, [&] {
                return launch_ranges(L, g, c->d_cc.as<CellConst>(), nc, k_first, n_band, kTilePoints,
                                     c->w_ranges.as<int2>(), st);
            }));
    DevCont ct{-1, nullptr, nullptr, nullptr, nullptr};
    if (c->n_cont_rec > 0)
        ct = DevCont{c->n_cont_thr, c->d_cont_thr.as<ContThr>(), c->d_cont_cum.as<double>(),
                     c->d_cont_ff.as<double>(), c->d_T_v.as<double>()};
    if (prec == LRT_FP32_COMP) {
        LRT_HIP(c, timed(c, LRT_K_ACCUM, st, [&] {
                    return launch_accum_f32(L, g, c->d_cc.as<CellConst>(), c->d_cs.as<CellSpecies>(),
                                            c->d_escale.as<int32_t>(), c->w_ranges.as<int2>(), nc,
                                            c->n_species, k_first, n_band, ct, (float *)eta, (float *)kappa,
                                            st);
                }));
        if (escale)
            LRT_HIP(c, hipMemcpyAsync(escale, c->d_escale.p, (size_t)nc * 2 * sizeof(int32_t),
                                      hipMemcpyDeviceToDevice, st));
    } else {
        LRT_HIP(c, timed(c, LRT_K_ACCUM, st, [&] {
                    return launch_accum_f64(L, g, c->d_cc.as<CellConst>(), c->d_cs.as<CellSpecies>(),
                                            c->w_ranges.as<int2>(), nc, c->n_species, k_first, n_band, ct,
                                            (double *)eta, (double *)kappa, st);
                }));
    }
    return LRT_OK;
}

lrt_status coeffs_impl(lrt_ctx *c, int64_t band, lrt_precision prec, void *eta, void *kappa,
                       int32_t *escale, hipStream_t st)
{
    if (!c->have_grid) return fail(c, LRT_E_STATE, "grid not set");
    int32_t k_first, n_band;
    lrt_status r;
    if ((r = band_range(c, band, k_first, n_band))) return r;
    return coeffs_range(c, k_first, n_band, prec, eta, kappa, escale, st);
}

// March of every ray over grid points [k_first, k_first + n_band).  The
// per-(ray, chunk) partial sums go to the context's workspace, or to
// `partials` (capacity `cap` doubles) when the caller brings its own buffer:
// then nothing is allocated and no launch is profiled.
lrt_status march_range(lrt_ctx *c, int32_t k_first, int32_t n_band, lrt_precision prec, const void *eta,
                       const void *kappa, const int32_t *escale, double *I_out, double *I_int_out,
                       hipStream_t st, double *partials, int64_t cap)
{
    if (prec != LRT_FP64 && prec != LRT_FP32_COMP) return fail(c, LRT_E_ARG, "unknown precision %d", (int)prec);
    if (!eta || !kappa || !I_int_out) return fail(c, LRT_E_ARG, "eta, kappa and I_int_out must be non-NULL");
    if (prec == LRT_FP32_COMP && !escale) return fail(c, LRT_E_ARG, "escale required for LRT_FP32_COMP");
    if (c->n_rays < 1) return fail(c, LRT_E_STATE, "rays not set");
    if (!c->have_grid) return fail(c, LRT_E_STATE, "grid not set");
    if (c->n_cells < 1) return fail(c, LRT_E_STATE, "cells not set");
    if (c->rays_cells != c->n_cells)
        return fail(c, LRT_E_STATE, "rays expect %lld cells, %lld set", (long long)c->rays_cells, (long long)c->n_cells);
    lrt_status r;
    const int32_t ppt = march_points_per_lane(c->h_off.back(), c->n_cells), chunk_points = 64 * ppt;
    const int32_t n_chunks = (n_band + chunk_points - 1) / chunk_points;
    const int64_t need = c->n_rays * (int64_t)n_chunks;
    if (partials) {
        if (need > cap)
            return fail(c, LRT_E_ARG, "the march needs %lld partial sums (rays x %d-point chunks), the buffer holds %lld",
                        (long long)need, chunk_points, (long long)cap);
    } else {
        if ((r = ensure(c, c->w_partials, (size_t)need * sizeof(double)))) return r;
    }
    double *part = partials ? partials : c->w_partials.as<double>();
    DevRays rays{(int32_t)c->n_rays, c->d_off.as<int64_t>(), c->d_cell.as<int32_t>(), c->d_ds.as<double>()};
    // every wall point with the same number of rays: the march may take them
    // direction-major
    if (c->n_wall > 0 && c->n_rays % c->n_wall == 0 && (int64_t)c->h_wall_off.size() == c->n_wall + 1) {
        const int64_t per = c->n_rays / c->n_wall;
        bool same = true;
        for (int64_t w = 0; w < c->n_wall && same; ++w) same = c->h_wall_off[w + 1] - c->h_wall_off[w] == per;
        if (same) rays.per_wall = (int32_t)per;
    }
    const DevGrid g = dev_grid(c);
    auto go = [&] {
        return launch_march(prec == LRT_FP32_COMP, c->march_scheme == LRT_MARCH_LINEAR_J, ppt, rays, g, k_first, n_band,
                            eta, kappa, escale, c->have_Tfar ? c->d_Tfar.as<double>() : nullptr, I_out, part,
                            n_chunks, st);
    };
    if (partials) LRT_HIP(c, go());
    else LRT_HIP(c, timed(c, LRT_K_MARCH, st, go));
    LRT_HIP(c, launch_reduce_rows(part, (int32_t)c->n_rays, n_chunks, I_int_out, st));
    return LRT_OK;
}

lrt_status march_impl(lrt_ctx *c, int64_t band, lrt_precision prec, const void *eta, const void *kappa,
                      const int32_t *escale, double *I_out, double *I_int_out, hipStream_t st)
{
    if (!c->have_grid) return fail(c, LRT_E_STATE, "grid not set");
    int32_t k_first, n_band;
    lrt_status r;
    if ((r = band_range(c, band, k_first, n_band))) return r;
    return march_range(c, k_first, n_band, prec, eta, kappa, escale, I_out, I_int_out, st, nullptr, 0);
}

// The whole path over a list of point ranges, each like one band: per-cell
// quantities recomputed once, then per range the coefficients, the march and
// the per-range wall sums; q and I_int are the sums over the ranges.
lrt_status solve_ranges(lrt_ctx *c, lrt_precision prec, int64_t n_rng, const int32_t *k_first,
                        const int32_t *n_pts, int64_t max_pts, double *q, double *I_int, double *q_rng,
                        hipStream_t st)
{
    if (prec != LRT_FP64 && prec != LRT_FP32_COMP) return fail(c, LRT_E_ARG, "unknown precision %d", (int)prec);
    if (c->n_rays < 1) return fail(c, LRT_E_STATE, "rays not set");
    const size_t esz = prec == LRT_FP64 ? 8 : 4;
    const size_t plane = (size_t)std::max<int64_t>(c->n_cells, 1) * (size_t)max_pts * esz;
    lrt_status r;
    if ((r = ensure(c, c->w_eta, plane)) || (r = ensure(c, c->w_kappa, plane)) ||
        (r = ensure(c, c->w_Iband, (size_t)c->n_rays * 8)) || (r = ensure(c, c->w_Itot, (size_t)c->n_rays * 8)) ||
        (r = ensure(c, c->w_qband, (size_t)c->n_wall * n_rng * 8)))
        return r;
    // zero the accumulators (all-zero bits are +0.0)
    LRT_HIP(c, launch_fill_u64(c->w_Itot.as<unsigned long long>(), 0ull, c->n_rays, st));
    LRT_HIP(c, launch_fill_u64(c->w_qband.as<unsigned long long>(), 0ull, c->n_wall * n_rng, st));
    int32_t *esc = (prec == LRT_FP32_COMP) ? c->d_escale.as<int32_t>() : nullptr;
    // populations and scales belong to the path: recompute them on every call
    if ((r = prepare(c, st, prec == LRT_FP32_COMP, true))) return r;
    for (int64_t b = 0; b < n_rng; ++b) {
        if ((r = coeffs_range(c, k_first[b], n_pts[b], prec, c->w_eta.p, c->w_kappa.p, nullptr, st))) return r;
        if ((r = march_range(c, k_first[b], n_pts[b], prec, c->w_eta.p, c->w_kappa.p, esc, nullptr,
                             c->w_Iband.as<double>(), st, nullptr, 0)))
            return r;
        LRT_HIP(c, launch_add(c->w_Itot.as<double>(), c->w_Iband.as<double>(), (int32_t)c->n_rays, st));
        // per-range wall flux into row b of the [n_rng][n_wall] staging array
        LRT_HIP(c, launch_wall_sum(c->w_Iband.as<double>(), c->d_weight.as<double>(), c->d_wall_off.as<int64_t>(),
                                   (int32_t)c->n_wall, c->w_qband.as<double>() + b * c->n_wall, st));
    }
    std::vector<double> qb((size_t)c->n_wall * n_rng), it((size_t)c->n_rays);
    LRT_HIP(c, hipMemcpyAsync(qb.data(), c->w_qband.p, qb.size() * 8, hipMemcpyDeviceToHost, st));
    LRT_HIP(c, hipMemcpyAsync(it.data(), c->w_Itot.p, it.size() * 8, hipMemcpyDeviceToHost, st));
    LRT_HIP(c, hipStreamSynchronize(st));
    for (int64_t w = 0; w < c->n_wall; ++w) {
        double sum = 0.0;
        for (int64_t b = 0; b < n_rng; ++b) {
            sum += qb[b * c->n_wall + w];
            if (q_rng) q_rng[w * n_rng + b] = qb[b * c->n_wall + w];
        }
        if (q) q[w] = sum;
    }
    if (I_int) std::copy(it.begin(), it.end(), I_int);
    return LRT_OK;
}

// In-window terms (and core terms) over grid points [k_first, k_first + n).
lrt_status count_range(lrt_ctx *c, int32_t k_first, int32_t n_band, int64_t *count, int64_t *core_count,
                       hipStream_t st)
{
    lrt_status r;
    if ((r = prepare(c, st, false))) return r;
    if ((r = ensure(c, c->w_count, 16)) || (r = ensure(c, c->w_ranges, (size_t)c->n_cells * sizeof(int2))))
        return r;
    LRT_HIP(c, launch_fill_u64(c->w_count.as<unsigned long long>(), 0ull, 2, st));
    const DevGrid g = dev_grid(c);
    const DevLines L = dev_lines(c);
    // candidate lines of each cell for the whole range (one tile spanning it)
    LRT_HIP(c, launch_ranges(L, g, c->d_cc.as<CellConst>(), (int32_t)c->n_cells, k_first, n_band, n_band,
                             c->w_ranges.as<int2>(), st));
    LRT_HIP(c, launch_count(L, g, c->d_cc.as<CellConst>(), c->d_cs.as<CellSpecies>(), c->w_ranges.as<int2>(),
                            (int32_t)c->n_cells, c->n_species, k_first, n_band,
                            c->w_count.as<unsigned long long>(), st));
    unsigned long long v[2] = {0, 0};
    LRT_HIP(c, hipMemcpyAsync(v, c->w_count.p, 16, hipMemcpyDeviceToHost, st));
    LRT_HIP(c, hipStreamSynchronize(st));
    *count = (int64_t)v[0];
    if (core_count) *core_count = (int64_t)v[1];
    return LRT_OK;
}

// Validates a list of point ranges against the grid; returns the longest.
lrt_status check_ranges(lrt_ctx *c, int64_t n, const int64_t *k_first, const int64_t *n_points,
                        std::vector<int32_t> &kf, std::vector<int32_t> &np, int64_t &max_pts)
{
    if (!c->have_grid) return fail(c, LRT_E_STATE, "grid not set");
    if (n < 1 || !k_first || !n_points) return fail(c, LRT_E_ARG, "need at least one range");
    kf.resize(n);
    np.resize(n);
    max_pts = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (k_first[i] < 0 || n_points[i] < 1 || n_points[i] > c->n_points - k_first[i])
            return fail(c, LRT_E_ARG, "range %lld [%lld, +%lld) outside the grid of %lld points", (long long)i,
                        (long long)k_first[i], (long long)n_points[i], (long long)c->n_points);
        if (n_points[i] > c->band_points)
            return fail(c, LRT_E_ARG, "range %lld longer than the band length %lld", (long long)i,
                        (long long)c->band_points);
        kf[i] = (int32_t)k_first[i];
        np[i] = (int32_t)n_points[i];
        max_pts = std::max<int64_t>(max_pts, n_points[i]);
    }
    return LRT_OK;
}

}  // namespace lrt

extern "C" {

lrt_status lrt_coeffs(lrt_ctx *c, int64_t band, lrt_precision prec, void *eta, void *kappa,
                      int32_t *escale, void *stream)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    return coeffs_impl(c, band, prec, eta, kappa, escale, (hipStream_t)stream);
}

lrt_status lrt_march(lrt_ctx *c, int64_t band, lrt_precision prec, const void *eta, const void *kappa,
                     const int32_t *escale, double *I_out, double *I_int_out, void *stream)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    return march_impl(c, band, prec, eta, kappa, escale, I_out, I_int_out, (hipStream_t)stream);
}

lrt_status lrt_solve(lrt_ctx *c, lrt_precision prec, int64_t first_band, double *q, double *I_int,
                     double *q_band, void *stream)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (prec != LRT_FP64 && prec != LRT_FP32_COMP) return fail(c, LRT_E_ARG, "unknown precision %d", (int)prec);
    if (!c->have_grid) return fail(c, LRT_E_STATE, "grid not set");
    if (c->n_rays < 1) return fail(c, LRT_E_STATE, "rays not set");
    const int64_t nb = (c->n_points + c->band_points - 1) / c->band_points;
    if (first_band < 0 || first_band >= nb) return fail(c, LRT_E_ARG, "first_band out of range");
    // the bands as point ranges
    const int64_t n = nb - first_band;
    std::vector<int32_t> kf(n), np(n);
    for (int64_t b = first_band; b < nb; ++b) {
        lrt_status r = band_range(c, b, kf[b - first_band], np[b - first_band]);
        if (r) return r;
    }
    std::vector<double> qr(q_band ? (size_t)c->n_wall * n : 0);
    lrt_status r = solve_ranges(c, prec, n, kf.data(), np.data(), std::min(c->band_points, c->n_points), q, I_int,
                                q_band ? qr.data() : nullptr, (hipStream_t)stream);
    if (r) return r;
    if (q_band)
        for (int64_t w = 0; w < c->n_wall; ++w)
            for (int64_t b = first_band; b < nb; ++b) q_band[w * nb + b] = qr[w * n + (b - first_band)];
    return LRT_OK;
}

lrt_status lrt_count_terms(lrt_ctx *c, int64_t band, int64_t *count, int64_t *core_count, void *stream)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (!count) return fail(c, LRT_E_ARG, "count must be non-NULL");
    hipStream_t st = (hipStream_t)stream;
    if (!c->have_grid) return fail(c, LRT_E_STATE, "grid not set");
    int32_t k_first, n_band;
    lrt_status r;
    if ((r = band_range(c, band, k_first, n_band))) return r;
    return count_range(c, k_first, n_band, count, core_count, st);
}

lrt_status lrt_solve_ranges(lrt_ctx *c, lrt_precision prec, int64_t n, const int64_t *k_first,
                            const int64_t *n_points, double *q, double *I_int, double *q_range, void *stream)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    std::vector<int32_t> kf, np;
    int64_t max_pts = 0;
    lrt_status r;
    if ((r = check_ranges(c, n, k_first, n_points, kf, np, max_pts))) return r;
    return solve_ranges(c, prec, n, kf.data(), np.data(), max_pts, q, I_int, q_range, (hipStream_t)stream);
}

lrt_status lrt_count_terms_ranges(lrt_ctx *c, int64_t n, const int64_t *k_first, const int64_t *n_points,
                                  int64_t *count, int64_t *core_count, void *stream)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (!count) return fail(c, LRT_E_ARG, "count must be non-NULL");
    std::vector<int32_t> kf, np;
    int64_t max_pts = 0;
    lrt_status r;
    if ((r = check_ranges(c, n, k_first, n_points, kf, np, max_pts))) return r;
    int64_t tot = 0, tot_core = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t a = 0, b = 0;
        if ((r = count_range(c, kf[i], np[i], &a, &b, (hipStream_t)stream))) return r;
        tot += a;
        tot_core += b;
    }
    *count = tot;
    if (core_count) *core_count = tot_core;
    return LRT_OK;
}

lrt_status lrt_profile(lrt_ctx *c, int enable)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    LRT_HIP(c, hipDeviceSynchronize());
    c->clear_events();
    c->prof = enable != 0;
    return LRT_OK;
}

lrt_status lrt_profile_read(lrt_ctx *c, int kernel, double *ms, int64_t *launches)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (kernel < 0 || kernel >= LRT_K_COUNT) return fail(c, LRT_E_ARG, "unknown kernel id %d", kernel);
    double tot = 0.0;
    for (auto &p : c->ev[kernel]) {
        LRT_HIP(c, hipEventSynchronize(p.second));
        float t = 0.0f;
        LRT_HIP(c, hipEventElapsedTime(&t, p.first, p.second));
        tot += t;
    }
    if (ms) *ms = tot;
    if (launches) *launches = (int64_t)c->ev[kernel].size();
    return LRT_OK;
}

}  // extern "C"
