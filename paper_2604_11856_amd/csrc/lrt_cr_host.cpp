// Host side of the QSS collisional-radiative populations (arXiv 2604.11856,
// Sec. 2.1 CR model): validation and upload of the atoms' rate data, the
// line-to-level map the line setup reads, and the per-cell solve launched with
// the other per-cell quantities.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/lrt.h"
#include "lrt_ctx.h"
#include "lrt_internal.h"

using namespace lrt;

namespace {

bool finite_nonneg(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!(p[i] >= 0.0) || !std::isfinite(p[i])) return false;
    return true;
}

// Arrhenius triples: C >= 0, n and E_a finite.
bool triples_ok(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!(p[3 * i] >= 0.0) || !std::isfinite(p[3 * i]) || !std::isfinite(p[3 * i + 1]) ||
            !std::isfinite(p[3 * i + 2]))
            return false;
    return true;
}

}  // namespace

namespace lrt {

DevCR dev_cr(const lrt_ctx *c)
{
    if (c->n_cr < 1) return DevCR{0, 0, nullptr, nullptr, nullptr, nullptr, nullptr};
    return DevCR{c->n_cr, c->cr_LS, c->d_cr_rec.as<CRRec>(), c->d_cr_slot.as<int32_t>(),
                 c->d_cr_w.as<double>(), c->d_cr_pop.as<double>(), c->d_cr_lnd.as<double>()};
}

// Pack the line levels into offsets of a cell's departure row:
// (slot * LS + level) of the upper level in the low 16 bits, of the lower
// level in the high 16 bits; -1 for a line without levels or whose species
// has no QSS-CR record.  Also list, per scale bin, the offsets of the levels its
// lines belong to (-1 for Boltzmann lines), so that the per-cell scale bound
// takes each bin's own largest departure.
lrt_status cr_build_line_levels(lrt_ctx *c)
{
    c->line_lev_ready = false;
    if (c->n_cr < 1 || c->h_lev_u.empty() || c->n_lines < 1) return LRT_OK;
    const int64_t n = c->n_lines;
    std::vector<int32_t> packed(n, -1);
    // the scale bins' level lists: (bin, offset) pairs, sorted and unique
    std::vector<std::pair<int32_t, int32_t>> bl;
    bl.reserve(2 * (size_t)n);
    bool any = false;
    for (int64_t j = 0; j < n; ++j) {
        const int32_t u = c->h_lev_u[j], l = c->h_lev_l[j];
        const int32_t slot = u >= 0 ? c->h_cr_slot[c->h_spc[j]] : -1;
        const int32_t ou = slot >= 0 ? slot * c->cr_LS + u : -1;
        const int32_t ol = slot >= 0 ? slot * c->cr_LS + l : -1;
        if (slot >= 0) {
            packed[j] = ou | (ol << 16);
            any = true;
        }
        if (c->h_bin_u[j] >= 0) bl.push_back({c->h_bin_u[j], ou});
        if (c->h_bin_l[j] >= 0) bl.push_back({c->h_bin_l[j], ol});
    }
    if (!any) return LRT_OK;
    std::sort(bl.begin(), bl.end());
    bl.erase(std::unique(bl.begin(), bl.end()), bl.end());
    std::vector<int32_t> off(c->n_bins + 1, 0), lev(bl.size());
    for (size_t t = 0; t < bl.size(); ++t) {
        ++off[bl[t].first + 1];
        lev[t] = bl[t].second;
    }
    for (int64_t b = 0; b < c->n_bins; ++b) off[b + 1] += off[b];
    lrt_status st;
    if ((st = upload(c, c->d_line_lev, packed.data(), packed.size() * sizeof(int32_t))) ||
        (st = upload(c, c->d_bin_lev_off, off.data(), off.size() * sizeof(int32_t))) ||
        (st = upload(c, c->d_bin_lev, lev.data(), std::max<size_t>(1, lev.size()) * sizeof(int32_t))))
        return st;
    c->line_lev_ready = true;
    c->scale_ready = false;
    return LRT_OK;
}

// Populations of every (cell, CR species), after the thermo kernel (they need its
// ln(N/Q)).
lrt_status cr_run(lrt_ctx *c, const DevCells &cells, hipStream_t st)
{
    if (c->n_cr < 1) return LRT_OK;
    const size_t rows = (size_t)c->n_cells * c->n_cr * c->cr_LS;
    lrt_status r;
    if ((r = ensure(c, c->d_cr_pop, rows * sizeof(double))) || (r = ensure(c, c->d_cr_lnd, rows * sizeof(double))))
        return r;
    int32_t max_lev = 0;
    for (int32_t v : c->h_cr_nlev) max_lev = std::max(max_lev, v);
    const DevCR cr = dev_cr(c);
    LRT_HIP(c, timed(c, LRT_K_CR, st, [&] {
                return launch_cr(c->sp, cells, cr, c->cr_max_l, max_lev, c->d_cs.as<CellSpecies>(), st);
            }));
    return LRT_OK;
}

}  // namespace lrt

extern "C" {

lrt_status lrt_set_cr(lrt_ctx *c, int n, const lrt_cr_species *recs, const double *collider_w)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (c->n_species < 1) return fail(c, LRT_E_STATE, "set species before the QSS-CR species");
    if (n < 0 || (n > 0 && (!recs || !collider_w)))
        return fail(c, LRT_E_ARG, "n must be >= 0, records and collider_w non-NULL");
    const int S = c->n_species;
    if (n > 0 && !finite_nonneg(collider_w, S))
        return fail(c, LRT_E_ARG, "collider weights must be finite and >= 0");
    std::vector<int32_t> slot(S, -1), nlev(n);
    std::vector<CRRec> rec(n);
    std::vector<double> tab;
    constexpr int kTabs = 7;   // hpie, eie, A, eii, ce, hpid, eid
    std::vector<size_t> off(n * kTabs);
    int LS = 0, max_l = 0;
    auto valid_sp = [&](int s) { return s >= 0 && s < S; };
    auto n_levels = [&](int s) { return (int)(c->h_lev_off[s + 1] - c->h_lev_off[s]); };
    for (int q = 0; q < n; ++q) {
        const lrt_cr_species &x = recs[q];
        if (!valid_sp(x.species) || (c->sp_kind[x.species] != LRT_KIND_ATOM && c->sp_kind[x.species] != LRT_KIND_MOLECULE))
            return fail(c, LRT_E_ARG, "CR record %d: species %d is neither an atom nor a molecule", q, x.species);
        if (slot[x.species] >= 0) return fail(c, LRT_E_ARG, "CR record %d: species %d given twice", q, x.species);
        const bool mol = c->sp_kind[x.species] == LRT_KIND_MOLECULE;
        const int NL = mol ? (int)(c->h_el_off[x.species + 1] - c->h_el_off[x.species]) : n_levels(x.species);
        if (NL > kCRMaxLevels) return fail(c, LRT_E_ARG, "CR record %d: more than %d states", q, kCRMaxLevels);
        const int L = x.n_model;
        if (L < 2 || L > NL) return fail(c, LRT_E_ARG, "CR record %d: n_model %d outside [2, %d]", q, L, NL);
        if (!(x.nu_cut >= 0.0) || std::isnan(x.nu_cut)) return fail(c, LRT_E_ARG, "CR record %d: nu_cut must be >= 0", q);
        for (int k = 0; k < 12; ++k)
            if (!(x.texp[k] >= 0.0 && x.texp[k] <= 1.0))
                return fail(c, LRT_E_ARG, "CR record %d: texp[%d] outside [0, 1]", q, k);
        if (!x.hpie || !x.eie || !x.A) return fail(c, LRT_E_ARG, "CR record %d: NULL rate table", q);
        const size_t LL = (size_t)L * L;
        if (!triples_ok(x.hpie, LL) || !triples_ok(x.eie, LL) || !finite_nonneg(x.A, LL))
            return fail(c, LRT_E_ARG, "CR record %d: negative or non-finite rate data", q);
        CRRec &R = rec[q];
        std::memset(&R, 0, sizeof(CRRec));
        R.species = x.species;
        R.n_model = L;
        R.n_lev = NL;
        R.kind = mol ? 2 : 1;
        R.nu_cut = x.nu_cut;
        R.ion = R.partner = R.partner_ion = R.diss_x = R.diss_y = -1;
        std::copy(x.texp, x.texp + 12, R.texp);
        const double *src[kTabs] = {x.hpie, x.eie, x.A, nullptr, nullptr, nullptr, nullptr};
        if (!mol) {
            if (x.diss_x != -1 || x.diss_y != -1)
                return fail(c, LRT_E_ARG, "CR record %d: dissociation given to an atom", q);
            if (x.ion != -1 && !valid_sp(x.ion)) return fail(c, LRT_E_ARG, "CR record %d: ion out of range", q);
            if (x.partner != -1) {
                if (!valid_sp(x.partner) || x.partner == x.species || c->sp_kind[x.partner] != LRT_KIND_ATOM)
                    return fail(c, LRT_E_ARG, "CR record %d: partner must be another atom", q);
                if (!valid_sp(x.partner_ion)) return fail(c, LRT_E_ARG, "CR record %d: partner ion out of range", q);
                if (x.ion < 0) return fail(c, LRT_E_ARG, "CR record %d: charge exchange needs the atom's ion", q);
                if (!(x.partner_E_ion > 0.0) || !(x.partner_Q_ion > 0.0) || !std::isfinite(x.partner_E_ion) ||
                    !std::isfinite(x.partner_Q_ion))
                    return fail(c, LRT_E_ARG, "CR record %d: partner E_ion and Q_ion must be positive", q);
            }
            if (!(x.E_ion > 0.0) || !(x.Q_ion > 0.0) || !std::isfinite(x.E_ion) || !std::isfinite(x.Q_ion))
                return fail(c, LRT_E_ARG, "CR record %d: E_ion and Q_ion must be positive", q);
            if (!x.eii || (x.partner >= 0 && !x.ce)) return fail(c, LRT_E_ARG, "CR record %d: NULL rate table", q);
            if (!triples_ok(x.eii, L) || (x.partner >= 0 && !triples_ok(x.ce, L)))
                return fail(c, LRT_E_ARG, "CR record %d: negative or non-finite rate data", q);
            src[3] = x.eii;
            src[4] = x.partner >= 0 ? x.ce : nullptr;
            R.ion = x.ion;
            R.partner = x.partner;
            R.partner_ion = x.partner >= 0 ? x.partner_ion : -1;
            R.pn_lev = x.partner >= 0 ? n_levels(x.partner) : 0;
            R.lev0 = c->h_lev_off[x.species];
            R.plev0 = x.partner >= 0 ? c->h_lev_off[x.partner] : 0;
            R.E_ion = x.E_ion;
            R.Q_ion = x.Q_ion;
            R.pE_ion = x.partner >= 0 ? x.partner_E_ion : 0.0;
            R.pQ_ion = x.partner >= 0 ? x.partner_Q_ion : 1.0;
        } else {
            if (x.ion != -1 || x.partner != -1)
                return fail(c, LRT_E_ARG, "CR record %d: ionization and charge exchange are for atoms", q);
            R.e0 = c->h_el_off[x.species];
            if (x.diss_x != -1 || x.diss_y != -1) {
                if (!valid_sp(x.diss_x) || !valid_sp(x.diss_y))
                    return fail(c, LRT_E_ARG, "CR record %d: dissociation product out of range", q);
                if (!x.hpid || !x.eid) return fail(c, LRT_E_ARG, "CR record %d: NULL rate table", q);
                if (!triples_ok(x.hpid, L) || !triples_ok(x.eid, L))
                    return fail(c, LRT_E_ARG, "CR record %d: negative or non-finite rate data", q);
                if (!std::isfinite(x.E_diss)) return fail(c, LRT_E_ARG, "CR record %d: non-finite E_diss", q);
                const int p[2] = {x.diss_x, x.diss_y};
                const double Qc[2] = {x.Q_x, x.Q_y};
                for (int k = 0; k < 2; ++k)
                    if (c->sp_kind[p[k]] != LRT_KIND_ATOM && !(Qc[k] > 0.0 && std::isfinite(Qc[k])))
                        return fail(c, LRT_E_ARG, "CR record %d: product %d is not an atom and has no Q > 0", q, p[k]);
                src[5] = x.hpid;
                src[6] = x.eid;
                R.diss_x = x.diss_x;
                R.diss_y = x.diss_y;
                R.nx_lev = c->sp_kind[x.diss_x] == LRT_KIND_ATOM ? n_levels(x.diss_x) : 0;
                R.ny_lev = c->sp_kind[x.diss_y] == LRT_KIND_ATOM ? n_levels(x.diss_y) : 0;
                R.x_lev0 = c->h_lev_off[x.diss_x];
                R.y_lev0 = c->h_lev_off[x.diss_y];
                R.Q_x = x.Q_x;
                R.Q_y = x.Q_y;
                R.E_diss = x.E_diss;
                const double mx = c->sp_mass[x.diss_x], my = c->sp_mass[x.diss_y];
                R.mu = mx * my / (mx + my) * (1.0 / 6.02214076e23);
            }
        }
        // tables concatenated (zeros for the ones a record has no use for)
        const size_t len[kTabs] = {3 * LL, 3 * LL, LL, 3 * (size_t)L, 3 * (size_t)L, 3 * (size_t)L, 3 * (size_t)L};
        for (int t = 0; t < kTabs; ++t) {
            off[kTabs * q + t] = tab.size();
            if (src[t]) tab.insert(tab.end(), src[t], src[t] + len[t]);
            else tab.insert(tab.end(), len[t], 0.0);
        }
        slot[x.species] = q;
        nlev[q] = NL;
        LS = std::max(LS, NL);
        max_l = std::max(max_l, L);
    }
    if (n > 0) {
        lrt_status st;
        if ((st = upload(c, c->d_cr_tab, tab.data(), tab.size() * sizeof(double)))) return st;
        const double *base = c->d_cr_tab.as<double>();
        for (int q = 0; q < n; ++q) {
            const double **ptr[kTabs] = {&rec[q].hpie, &rec[q].eie, &rec[q].A, &rec[q].eii, &rec[q].ce,
                                         &rec[q].hpid, &rec[q].eid};
            for (int t = 0; t < kTabs; ++t) *ptr[t] = base + off[kTabs * q + t];
        }
        if ((st = upload(c, c->d_cr_rec, rec.data(), rec.size() * sizeof(CRRec))) ||
            (st = upload(c, c->d_cr_slot, slot.data(), slot.size() * sizeof(int32_t))) ||
            (st = upload(c, c->d_cr_w, collider_w, (size_t)S * sizeof(double))))
            return st;
    }
    c->n_cr = n;
    c->cr_LS = LS;
    c->cr_max_l = max_l;
    c->h_cr_slot = slot;
    c->h_cr_nlev = nlev;
    c->thermo_ready = c->scale_ready = false;
    return cr_build_line_levels(c);
}

lrt_status lrt_set_line_levels(lrt_ctx *c, const int32_t *lev_u, const int32_t *lev_l, int64_t n)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (c->n_lines < 0) return fail(c, LRT_E_STATE, "set lines before their levels");
    if (!lev_u && !lev_l) {
        c->h_lev_u.clear();
        c->h_lev_l.clear();
        c->line_lev_ready = false;
        c->scale_ready = false;
        return LRT_OK;
    }
    if (!lev_u || !lev_l) return fail(c, LRT_E_ARG, "lev_u and lev_l must both be NULL or both non-NULL");
    if (n != c->n_lines) return fail(c, LRT_E_ARG, "%lld levels for %lld lines", (long long)n, (long long)c->n_lines);
    std::vector<int32_t> u(n), l(n);
    for (int64_t j = 0; j < n; ++j) {
        const int64_t i = c->h_line_order[j];   // caller's index of sorted line j
        const int32_t a = lev_u[i], b = lev_l[i];
        if (a == -1 && b == -1) {
            u[j] = l[j] = -1;
            continue;
        }
        const int s = c->h_spc[j];
        const int64_t NL = c->sp_kind[s] == LRT_KIND_ATOM ? c->h_lev_off[s + 1] - c->h_lev_off[s]
                                                           : c->h_el_off[s + 1] - c->h_el_off[s];
        if (a < 0 || b < 0 || a >= NL || b >= NL)
            return fail(c, LRT_E_ARG, "line %lld: states (%d, %d) outside the species' %lld states", (long long)i, a,
                        b, (long long)NL);
        u[j] = a;
        l[j] = b;
    }
    c->h_lev_u.swap(u);
    c->h_lev_l.swap(l);
    c->scale_ready = false;
    return cr_build_line_levels(c);
}

lrt_status lrt_cr_populations(lrt_ctx *c, int rec, double *pop, void *stream)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (c->n_cr < 1) return fail(c, LRT_E_STATE, "no QSS-CR atoms set");
    if (rec < 0 || rec >= c->n_cr) return fail(c, LRT_E_ARG, "CR record %d out of range", rec);
    if (!pop) return fail(c, LRT_E_ARG, "pop must be non-NULL");
    hipStream_t st = (hipStream_t)stream;
    lrt_status r;
    if ((r = prepare(c, st, false))) return r;
    const int NL = c->h_cr_nlev[rec];
    const size_t pitch = (size_t)c->n_cr * c->cr_LS * sizeof(double);
    LRT_HIP(c, hipMemcpy2DAsync(pop, NL * sizeof(double), c->d_cr_pop.as<double>() + (size_t)rec * c->cr_LS, pitch,
                                NL * sizeof(double), (size_t)c->n_cells, hipMemcpyDeviceToHost, st));
    LRT_HIP(c, hipStreamSynchronize(st));
    return LRT_OK;
}

}  // extern "C"
