/*
 * Plain FP64 CPU oracle of the line-by-line + ray-march radiation path of
 * arXiv 2604.11856 ("RAPRAL").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load or call this file.  It shares no
 * code, header, table or helper with the GPU library; the two meet only at
 * the seeded inputs.
 *
 * Every quantity is the plain definition written out in double precision,
 * in the order the paper states it.  Two choices go beyond "plain double":
 *   - the grid offset nu_k - nu0 is formed in __float128 and rounded once, so
 *     that it is the correctly rounded difference of the real grid point and
 *     the line centre (forming nu_min + k h in double first would lose ~1e-11
 *     cm^-1, i.e. ~1e-10 of a narrow profile);
 *   - lines that provably cannot reach a requested grid point are skipped
 *     (bound: Voigt HWHM <= Lorentz HWHM + Doppler HWHM, which holds because
 *     the bracket of the Olivero fit is <= 1 on d in [-1, 1]); the sum at each
 *     point is still taken over every covering line in line-list order.
 *
 * Units are cm^-1 for wavenumbers and energies (the paper's wavelength forms
 * are converted by the exact change of variables), K, cm^-3, cm.  eta is in
 * W cm^-3 sr^-1 (cm^-1)^-1, kappa in cm^-1, I in W cm^-2 sr^-1 (cm^-1)^-1,
 * q in W cm^-2.  CGS products are multiplied by 1e-7 to give W.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA exact SI values, in CGS units */
#define ORC_H 6.62607015e-27   /* Planck constant, erg s */
#define ORC_C 2.99792458e10    /* speed of light, cm s^-1 */
#define ORC_KB 1.380649e-16    /* Boltzmann constant, erg K^-1 */
#define ORC_PI 3.14159265358979323846

typedef struct {
    int n_species;
    const int *kind;          /* 0 none, 1 atom, 2 diatomic molecule */
    const double *mass;       /* g/mol */
    /* atoms: levels lev_off[s] .. lev_off[s+1]-1 */
    const int64_t *lev_off;
    const double *lev_E, *lev_g;
    /* molecules: electronic states el_off[s] .. el_off[s+1]-1 */
    const int64_t *el_off;
    const double *el_T, *el_g;
    const int *el_Jmax;
    /* vibrational levels of electronic state e: vib_off[e] .. vib_off[e+1]-1 */
    const int64_t *vib_off;
    const double *vib_G, *vib_B, *vib_D;
    /* ionization energies, cm^-1, per species: an atom with E_ion > 0 gives
     * its lines the full Lorentz width (NULL: the uniform Stark law for all) */
    const double *E_ion;
} orc_species;

typedef struct {
    int64_t n;
    const double *nu0, *A, *Eu_ev, *Eu_rot, *El_ev, *El_rot, *gu, *gl;
    const int32_t *species;
    /* optional (NULL: none): the line's upper and lower level in its atom's
     * level table, -1 for a line without levels */
    const int32_t *lev_u, *lev_l;
} orc_lines;

typedef struct {
    int64_t n_cells;
    int n_species;
    const double *T_tr, *T_v, *N, *n_e;   /* N is [n_cells][n_species] */
    /* optional (NULL: none): state populations [n_cells][lev_off[n_species]
     * + el_off[n_species]] (atom levels, then molecular electronic states)
     * that replace the Boltzmann ones of the species with lev_on[s] != 0 */
    const double *N_lev;
    const int *lev_on;
} orc_cells;

/* Everything the method fixes for one (cell, line) pair. */
typedef struct {
    double Nu, Nl;          /* upper / lower level populations, cm^-3 */
    double S_eta;           /* eta_i(nu) = S_eta * phi(nu) */
    double B_line;          /* kappa_i(nu) = eta_i(nu) / B_line */
    double gG, gL, gV;      /* Doppler, Lorentz, Voigt HWHM, cm^-1 */
    int64_t klo, khi;       /* grid window, inclusive; empty if klo > khi */
} orc_pair;

double orc_c2(void) { return ORC_H * ORC_C / ORC_KB; }

/* ---------------------------------------------------------------------- */
/* Sec. 2.1: Boltzmann populations                                         */
/* ---------------------------------------------------------------------- */

/* Atomic electronic partition function sum_j g_j exp(-hc E_j / k T_ee),
 * Sec. 2.1 Boltzmann relation; T_ee = T_v in the two-temperature model. */
double orc_partition_atom(int64_t n, const double *E, const double *g, double Tv)
{
    double q = 0.0;
    for (int64_t j = 0; j < n; ++j)
        q += g[j] * exp(-orc_c2() * E[j] / Tv);
    return q;
}

/* Molecular partition function, Sec. 2.1 molecular Boltzmann relation:
 * sum_e g_e exp(-hc T_e/kT_v) Q_vr,e with
 * Q_vr,e = sum_v exp(-hc G_v/kT_v) sum_J (2J+1) exp(-hc F_v(J)/kT_r),
 * F_v(J) = B_v J(J+1) - D_v J^2 (J+1)^2 (Hund (a) term, Sec. 2.2.2).
 * The symmetry number and line-alternation factor are 1 (they cancel
 * between the level population and the partition function). */
double orc_partition_molecule(const orc_species *sp, int s, double Tv, double Ttr)
{
    const double c2 = orc_c2();
    double q = 0.0;
    for (int64_t e = sp->el_off[s]; e < sp->el_off[s + 1]; ++e) {
        double qvr = 0.0;
        for (int64_t v = sp->vib_off[e]; v < sp->vib_off[e + 1]; ++v) {
            double qr = 0.0;
            for (int J = 0; J <= sp->el_Jmax[e]; ++J) {
                double jj = (double)J * (J + 1.0);
                double F = sp->vib_B[v] * jj - sp->vib_D[v] * jj * jj;
                qr += (2.0 * J + 1.0) * exp(-c2 * F / Ttr);
            }
            qvr += exp(-c2 * sp->vib_G[v] / Tv) * qr;
        }
        q += sp->el_g[e] * exp(-c2 * sp->el_T[e] / Tv) * qvr;
    }
    return q;
}

/* Partition function of one state of species s (energy zero as in the
 * species' own partition function): an atom's level `state`,
 * g e^{-c2 E/T_v}, or a molecule's electronic state `state`,
 * g_e e^{-c2 T_e/T_v} Q_vr,e with Q_vr,e as above. */
double orc_state_partition(const orc_species *sp, int s, int64_t state, double Tv, double Ttr)
{
    const double c2 = orc_c2();
    if (sp->kind[s] == 1) {
        int64_t j = sp->lev_off[s] + state;
        return sp->lev_g[j] * exp(-c2 * sp->lev_E[j] / Tv);
    }
    int64_t e = sp->el_off[s] + state;
    double qvr = 0.0;
    for (int64_t v = sp->vib_off[e]; v < sp->vib_off[e + 1]; ++v) {
        double qr = 0.0;
        for (int J = 0; J <= sp->el_Jmax[e]; ++J) {
            double jj = (double)J * (J + 1.0);
            double F = sp->vib_B[v] * jj - sp->vib_D[v] * jj * jj;
            qr += (2.0 * J + 1.0) * exp(-c2 * F / Ttr);
        }
        qvr += exp(-c2 * sp->vib_G[v] / Tv) * qr;
    }
    return sp->el_g[e] * exp(-c2 * sp->el_T[e] / Tv) * qvr;
}

double orc_partition(const orc_species *sp, int s, double Tv, double Ttr)
{
    if (sp->kind[s] == 1)
        return orc_partition_atom(sp->lev_off[s + 1] - sp->lev_off[s],
                                  sp->lev_E + sp->lev_off[s], sp->lev_g + sp->lev_off[s], Tv);
    if (sp->kind[s] == 2)
        return orc_partition_molecule(sp, s, Tv, Ttr);
    return 0.0;
}

/* Population of one level of energy E_ev (electronic + vibrational, at T_v)
 * + E_rot (rotational, at T_tr) and degeneracy g: N g exp(-hc E/kT) / Q. */
double orc_level_population(double N, double Q, double g, double E_ev, double E_rot,
                            double Tv, double Ttr)
{
    const double c2 = orc_c2();
    return N * g * exp(-c2 * E_ev / Tv - c2 * E_rot / Ttr) / Q;
}

/* ---------------------------------------------------------------------- */
/* Sec. 2.2.1: line shape                                                  */
/* ---------------------------------------------------------------------- */

/* Doppler HWHM: (7.16233e-7 / 2) nu0 sqrt(T_t / M). */
double orc_doppler_hwhm(double nu0, double Ttr, double M)
{
    return 7.16233e-7 / 2.0 * nu0 * sqrt(Ttr / M);
}

/* Lorentz HWHM: the Stark law (T_ee/1e4)^0.33 (N_e/1e16) with a reference
 * width of 1 cm^-1, i.e. 1e-16 n_e (T_v/1e4)^0.33 cm^-1. */
double orc_lorentz_hwhm(double ne, double Tv)
{
    return 1e-16 * ne * pow(Tv / 1e4, 0.33);
}

/* Lorentz HWHM of line i in a cell with the per-species densities N_cell
 * (Sec. 2.2.1 pressure broadening).  An atom with an ionization energy gets
 * the sum of natural (5.9e-6 nm), Stark
 * (1.69e3 lambda^2 / dE^2.623 (T_ee/1e4)^0.33 (N_e/1e16), dE = max(E_ion - E_u,
 * E_ion(H)/25)) and van der Waals (lambda^2 [6.65e-29 N (2 T_t/M)^0.5 +
 * 2.925e-29 N_others (2 T_t/M_others)^0.5]) widths in nm at lambda = 1e7/nu0 nm,
 * converted to cm^-1 by dnu = 1e7 dlambda / lambda^2; resonance broadening is
 * left out.  N_others: every other species but the electrons (M < 0.01 g/mol),
 * M_others their density-weighted mean molar mass.  Other lines: the uniform
 * Stark law. */
#define ORC_E_H 109678.77   /* ionization energy of hydrogen, cm^-1 */
double orc_lorentz_line(const orc_species *sp, const orc_lines *L, int64_t i, double Ttr,
                        double Tv, double ne, const double *N_cell, int S)
{
    int s = L->species[i];
    if (!sp->E_ion || !(sp->E_ion[s] > 0.0) || sp->kind[s] != 1) return orc_lorentz_hwhm(ne, Tv);
    double lam = 1e7 / L->nu0[i];   /* nm */
    double dl_N = 5.9e-6;
    double Eu = L->Eu_ev[i] + L->Eu_rot[i];
    double dE = fmax(sp->E_ion[s] - Eu, ORC_E_H / 25.0);
    double dl_S = 1.69e3 * lam * lam / pow(dE, 2.623) * pow(Tv / 1e4, 0.33) * (ne / 1e16);
    double Noth = 0.0, NMoth = 0.0;
    for (int t = 0; t < S; ++t) {
        if (t == s || sp->mass[t] < 0.01) continue;
        Noth += N_cell[t];
        NMoth += N_cell[t] * sp->mass[t];
    }
    double lw0 = 6.65e-29 * N_cell[s] * sqrt(2.0 * Ttr / sp->mass[s]);
    if (Noth > 0.0) lw0 += 2.925e-29 * Noth * sqrt(2.0 * Ttr / (NMoth / Noth));
    double dl_W = lw0 * lam * lam;
    return 1e7 * (dl_N + dl_S + dl_W) / (lam * lam);
}

/* Voigt HWHM (Olivero-type fit) from the Lorentz and Doppler HWHMs. */
double orc_voigt_hwhm(double gL, double gG)
{
    double d = (gL - gG) / (gL + gG);
    double f = 1.0 - 0.18121 * (1.0 - d * d)
               - (0.023665 * exp(0.6 * d) + 0.00418 * exp(-1.9 * d)) * sin(ORC_PI * d);
    return f * (gL + gG);
}

/* Whiting-type Voigt profile, per cm^-1, at offset delta from line centre. */
double orc_voigt_profile(double delta, double gV, double gL)
{
    double r = gL / gV;
    double x = fabs(delta) / (2.0 * gV);
    double x225 = pow(x, 2.25);
    double shape = (1.0 - r) * exp(-2.772 * x * x)
                   + r / (1.0 + 4.0 * x * x)
                   + 0.016 * r * (1.0 - r) * (exp(-0.4 * x225) - 1.0 / (1.0 + 0.1 * x225));
    return shape / (2.0 * gV * (1.065 + 0.447 * r + 0.058 * r * r));
}

/* Grid window of a line: all k with |nu_k - nu0| <= 100 gV, nu_k = nu_min + k h,
 * as integer bounds clamped to [0, n_points-1]. */
void orc_window(double nu0, double gV, double nu_min, double h, int64_t n_points,
                int64_t *klo, int64_t *khi)
{
    double W = 100.0 * gV;
    double lo = ceil((nu0 - W - nu_min) / h);
    double hi = floor((nu0 + W - nu_min) / h);
    if (lo < 0.0) lo = 0.0;
    if (hi > (double)(n_points - 1)) hi = (double)(n_points - 1);
    *klo = (int64_t)lo;
    *khi = (int64_t)hi;
    if (lo > hi) { *klo = 1; *khi = 0; }
}

/* Grid offset nu_k - nu0, correctly rounded. */
double orc_grid_offset(double nu_min, double h, int64_t k, double nu0)
{
    __float128 v = (__float128)nu_min + (__float128)k * (__float128)h - (__float128)nu0;
    return (double)v;
}

/* Planck function per cm^-1 in W cm^-2 sr^-1 (cm^-1)^-1 (Sec. 2.2, wavenumber form). */
double orc_planck(double nu, double T)
{
    return 1e-7 * 2.0 * ORC_H * ORC_C * ORC_C * nu * nu * nu / expm1(orc_c2() * nu / T);
}

/* ---------------------------------------------------------------------- */
/* One (cell, line) pair: Sec. 2.2.1 emission, absorption and widths        */
/* ---------------------------------------------------------------------- */

/* Population of a line's level from the population Nlev of the table level
 * (energy E_lev, degeneracy g_lev) it belongs to: the line's level takes its
 * Boltzmann share g e^{-c2 (E_ev - E_lev)/T_v - c2 E_rot/T_tr} / g_lev. */
static double orc_sublevel_population(double Nlev, double g_lev, double E_lev, double g,
                                      double E_ev, double E_rot, double Tv, double Ttr)
{
    const double c2 = orc_c2();
    return Nlev * (g / g_lev) * exp(-c2 * (E_ev - E_lev) / Tv - c2 * E_rot / Ttr);
}

/* Nlev: NULL, or the level populations of the line's species in this cell
 * (Sec. 2.1 CR model); a line with levels then takes its populations from
 * them instead of the Boltzmann relation. */
void orc_line_pair(const orc_species *sp, const orc_lines *L, int64_t i,
                   double Ttr, double Tv, double ne, const double *N_cell, int S, double N_s,
                   double Q_s, const double *Nlev, double nu_min, double h, int64_t n_points,
                   orc_pair *p)
{
    int s = L->species[i];
    double nu0 = L->nu0[i];
    if (Nlev && L->lev_u && L->lev_u[i] >= 0 && sp->kind[s] == 1) {
        const int64_t o = sp->lev_off[s];
        const int u = L->lev_u[i], l = L->lev_l[i];
        p->Nu = orc_sublevel_population(Nlev[u], sp->lev_g[o + u], sp->lev_E[o + u], L->gu[i],
                                        L->Eu_ev[i], L->Eu_rot[i], Tv, Ttr);
        p->Nl = orc_sublevel_population(Nlev[l], sp->lev_g[o + l], sp->lev_E[o + l], L->gl[i],
                                        L->El_ev[i], L->El_rot[i], Tv, Ttr);
    } else if (Nlev && L->lev_u && L->lev_u[i] >= 0) {
        /* a molecule's rovibronic level takes its Boltzmann share of its
         * electronic state: g e^{-c2 E_ev/T_v - c2 E_rot/T_tr} / Q_state */
        const double c2 = orc_c2();
        const int u = L->lev_u[i], l = L->lev_l[i];
        p->Nu = Nlev[u] * L->gu[i] * exp(-c2 * L->Eu_ev[i] / Tv - c2 * L->Eu_rot[i] / Ttr)
                / orc_state_partition(sp, s, u, Tv, Ttr);
        p->Nl = Nlev[l] * L->gl[i] * exp(-c2 * L->El_ev[i] / Tv - c2 * L->El_rot[i] / Ttr)
                / orc_state_partition(sp, s, l, Tv, Ttr);
    } else {
        p->Nu = orc_level_population(N_s, Q_s, L->gu[i], L->Eu_ev[i], L->Eu_rot[i], Tv, Ttr);
        p->Nl = orc_level_population(N_s, Q_s, L->gl[i], L->El_ev[i], L->El_rot[i], Tv, Ttr);
    }
    /* j = (hc/4pi) N_u A_ul nu0 phi, nu0 the line centre (CGS -> W: 1e-7) */
    p->S_eta = 1e-7 * ORC_H * ORC_C * nu0 * p->Nu * L->A[i] / (4.0 * ORC_PI);
    /* kappa = j / B with exp(hc nu/kT) replaced by N_l g_u / (N_u g_l) */
    p->B_line = 1e-7 * 2.0 * ORC_H * ORC_C * ORC_C * nu0 * nu0 * nu0
                / (p->Nl * L->gu[i] / (p->Nu * L->gl[i]) - 1.0);
    p->gG = orc_doppler_hwhm(nu0, Ttr, sp->mass[s]);
    p->gL = orc_lorentz_line(sp, L, i, Ttr, Tv, ne, N_cell, S);
    p->gV = orc_voigt_hwhm(p->gL, p->gG);
    orc_window(nu0, p->gV, nu_min, h, n_points, &p->klo, &p->khi);
}

/* The state populations of species s in cell c, or NULL (Boltzmann).
 * N_lev holds, per cell, the atoms' levels (lev_off) followed by the
 * molecules' electronic states (el_off). */
static const double *orc_cell_levels(const orc_species *sp, const orc_cells *C, int64_t c, int s)
{
    if (!C->N_lev || !C->lev_on || !C->lev_on[s]) return NULL;
    const int64_t NL = sp->lev_off[sp->n_species], NE = sp->el_off[sp->n_species];
    const double *row = C->N_lev + c * (NL + NE);
    return sp->kind[s] == 2 ? row + NL + sp->el_off[s] : row + sp->lev_off[s];
}

/* first index with a[i] >= v in a sorted array */
static int64_t lower_bound(const double *a, int64_t n, double v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t m = lo + (hi - lo) / 2;
        if (a[m] < v) lo = m + 1; else hi = m;
    }
    return lo;
}

/* first index with ks[j] >= v in a sorted int64 array */
static int64_t lower_bound_i(const int64_t *a, int64_t n, int64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t m = lo + (hi - lo) / 2;
        if (a[m] < v) lo = m + 1; else hi = m;
    }
    return lo;
}

/* eta and kappa of one cell at the sorted grid indices ks[0..n_k-1]:
 * eta(nu_k) = sum_i eta_i(nu_k), kappa(nu_k) = sum_i eta_i(nu_k) / B_line_i,
 * over the lines i whose window holds k, in line-list order.
 * Lines must be sorted by nu0.  Returns the number of (line, point) terms. */
int64_t orc_cell_coeffs(const orc_species *sp, const orc_lines *L, const orc_cells *C,
                        int64_t c, double nu_min, double nu_max, int64_t n_points,
                        int64_t n_k, const int64_t *ks, double *eta, double *kappa)
{
    const double h = (nu_max - nu_min) / (double)(n_points - 1);
    const int S = C->n_species;
    const double Ttr = C->T_tr[c], Tv = C->T_v[c], ne = C->n_e[c];
    const double *N = C->N + c * S;
    double *Q = (double *)malloc(sizeof(double) * S);
    double Mmin = 1e300;
    for (int s = 0; s < S; ++s) {
        Q[s] = orc_partition(sp, s, Tv, Ttr);
        if (sp->kind[s] != 0 && sp->mass[s] < Mmin) Mmin = sp->mass[s];
    }
    for (int64_t j = 0; j < n_k; ++j) { eta[j] = 0.0; kappa[j] = 0.0; }
    if (n_k == 0 || L->n == 0) { free(Q); return 0; }

    /* Skip bound: a line reaches nu only if |nu - nu0| <= 100 (gL + b nu0),
     * gL the largest Lorentz HWHM of any line in this cell, b = Doppler
     * coefficient at the lightest radiator. Widened by 1e-6. */
    double gL = orc_lorentz_hwhm(ne, Tv);
    if (sp->E_ion)
        for (int64_t i = 0; i < L->n; ++i) {
            double gi = orc_lorentz_line(sp, L, i, Ttr, Tv, ne, N, S);
            if (gi > gL) gL = gi;
        }
    const double b = 7.16233e-7 / 2.0 * sqrt(Ttr / Mmin) * (1.0 + 1e-6);
    const double g = 100.0 * gL * (1.0 + 1e-6) + h;
    const double a = 100.0 * b;

    /* union of candidate index ranges over the requested points, walked in
     * ascending line order */
    int64_t i_next = 0, count = 0;
    int64_t j = 0;
    while (j < n_k) {
        double nu_lo = nu_min + (double)ks[j] * h;
        /* extend the run while candidate ranges overlap */
        int64_t i0 = lower_bound(L->nu0, L->n, (nu_lo - g) / (1.0 + a));
        int64_t jj = j;
        int64_t i1 = lower_bound(L->nu0, L->n, (nu_min + (double)ks[jj] * h + g) / (1.0 - a));
        while (jj + 1 < n_k) {
            int64_t n0 = lower_bound(L->nu0, L->n, (nu_min + (double)ks[jj + 1] * h - g) / (1.0 + a));
            if (n0 > i1) break;
            ++jj;
            i1 = lower_bound(L->nu0, L->n, (nu_min + (double)ks[jj] * h + g) / (1.0 - a));
        }
        if (i0 < i_next) i0 = i_next;
        for (int64_t i = i0; i < i1; ++i) {
            int s = L->species[i];
            if (sp->kind[s] == 0 || N[s] <= 0.0) continue;
            orc_pair p;
            orc_line_pair(sp, L, i, Ttr, Tv, ne, N, S, N[s], Q[s], orc_cell_levels(sp, C, c, s),
                          nu_min, h, n_points, &p);
            if (p.klo > p.khi) continue;
            int64_t a0 = lower_bound_i(ks, n_k, p.klo);
            for (int64_t t = a0; t < n_k && ks[t] <= p.khi; ++t) {
                double delta = orc_grid_offset(nu_min, h, ks[t], L->nu0[i]);
                double e = p.S_eta * orc_voigt_profile(delta, p.gV, p.gL);
                eta[t] += e;
                kappa[t] += e / p.B_line;
                ++count;
            }
        }
        if (i1 > i_next) i_next = i1;
        j = jj + 1;
    }
    free(Q);
    return count;
}

/* All cells (OpenMP over cells; each cell is independent).  eta/kappa are
 * [n_cells][n_k].  Returns the total number of (cell, line, point) terms. */
int64_t orc_coeffs(const orc_species *sp, const orc_lines *L, const orc_cells *C,
                   double nu_min, double nu_max, int64_t n_points,
                   int64_t n_k, const int64_t *ks, double *eta, double *kappa, int n_threads)
{
    int64_t total = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
#endif
    for (int64_t c = 0; c < C->n_cells; ++c)
        total += orc_cell_coeffs(sp, L, C, c, nu_min, nu_max, n_points, n_k, ks,
                                 eta + c * n_k, kappa + c * n_k);
    return total;
}

/* Brute force for tiny inputs: every line, every point, window tested by
 * |nu_k - nu0| <= 100 gV on the correctly rounded offset.  eta/kappa are
 * [n_cells][n_points]. */
void orc_coeffs_bruteforce(const orc_species *sp, const orc_lines *L, const orc_cells *C,
                           double nu_min, double nu_max, int64_t n_points,
                           double *eta, double *kappa)
{
    const double h = (nu_max - nu_min) / (double)(n_points - 1);
    const int S = C->n_species;
    for (int64_t c = 0; c < C->n_cells; ++c) {
        for (int64_t k = 0; k < n_points; ++k) { eta[c * n_points + k] = 0.0; kappa[c * n_points + k] = 0.0; }
        for (int64_t i = 0; i < L->n; ++i) {
            int s = L->species[i];
            double Ns = C->N[c * S + s];
            if (sp->kind[s] == 0 || Ns <= 0.0) continue;
            double Q = orc_partition(sp, s, C->T_v[c], C->T_tr[c]);
            orc_pair p;
            orc_line_pair(sp, L, i, C->T_tr[c], C->T_v[c], C->n_e[c], C->N + c * S, S, Ns, Q,
                          orc_cell_levels(sp, C, c, s), nu_min, h, n_points, &p);
            for (int64_t k = 0; k < n_points; ++k) {
                double delta = orc_grid_offset(nu_min, h, k, L->nu0[i]);
                if (fabs(delta) > 100.0 * p.gV) continue;
                double e = p.S_eta * orc_voigt_profile(delta, p.gV, p.gL);
                eta[c * n_points + k] += e;
                kappa[c * n_points + k] += e / p.B_line;
            }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Sec. 2.2.3: march along a line of sight                                  */
/* ---------------------------------------------------------------------- */

/* Cell-constant solution of dI/ds = j - kappa I over a segment of length ds:
 * I <- I exp(-tau) + j ds F(tau), tau = kappa ds, F(t) = (1 - e^-t)/t, F(0) = 1
 * (the Johnston-Mazaheri segment scheme with j constant, alpha + beta).
 * Segments are given far -> target; the far boundary is free (I = I_far).
 * eta/kappa are [n_cells][n_k]; I_out is [n_k]. */
void orc_march(int64_t n_seg, const int64_t *cell, const double *ds,
               int64_t n_k, const double *eta, const double *kappa,
               const double *I_far, double *I_out)
{
    for (int64_t k = 0; k < n_k; ++k) {
        double I = I_far ? I_far[k] : 0.0;
        for (int64_t m = 0; m < n_seg; ++m) {
            double kap = kappa[cell[m] * n_k + k];
            double j = eta[cell[m] * n_k + k];
            double tau = kap * ds[m];
            double F = (tau == 0.0) ? 1.0 : -expm1(-tau) / tau;
            I = I * exp(-tau) + j * ds[m] * F;
        }
        I_out[k] = I;
    }
}

/* ---------------------------------------------------------------------- */
/* Sec. 2.2.1 atomic continuum: bound-free and free-free                    */
/* ---------------------------------------------------------------------- */

#define ORC_ME 9.1093837015e-28   /* electron mass, g */

/* Saha-Boltzmann volume (h^2 / (2 pi m_e k T))^{3/2}, cm^3: the printed
 * factor with its SI-to-CGS conversions (1e6, 1e-3) carried out. */
double orc_saha_volume(double T)
{
    return pow(ORC_H * ORC_H / (2.0 * ORC_PI * ORC_ME * ORC_KB * T), 1.5);
}

/* Hydrogenic free-free cross section per (ion, electron) pair, cm^5, from
 * the fit z^4 s^3 sigma 1e40 = A1(T)/s + A2(T), A1 = c1 + c2 e^{-c3 T},
 * A2 = c4 + c5 e^{-c6 T} + c7 e^{-c8 T}, with s = lambda_H / lambda the
 * dimensionless wavelength parameter (lambda_H = 91.1267 nm). */
double orc_peach_ff(const double *c, double z, double s, double T)
{
    double A1 = c[0] + c[1] * exp(-c[2] * T);
    double A2 = c[3] + c[4] * exp(-c[5] * T) + c[6] * exp(-c[7] * T);
    return (A1 / s + A2) * 1e-40 / (z * z * z * z * s * s * s);
}

typedef struct {
    int species, ion;
    double E_ion, Q_ion;
    const double *sigma0;   /* [levels of the atom] */
    const double *peach;    /* c1..c8 */
    double z;
} orc_cont;

/* Continuum eta and kappa of every cell at grid points ks (added to eta /
 * kappa [n_cells][n_k]).  Per atom a with ion +: T = T_ee = T_v;
 *   bound-free from level i (threshold nu_i = E_ion - E_i, nu >= nu_i):
 *     kappa = N_i sigma_i(nu), N_i = N_a g_i e^{-c2 E_i/T} / Q_a (or the
 *     cell's level population when the atom has them),
 *     eta = B(nu, T) sigma_i(nu) N_+ n_e V(T) g_i e^{c2 (E_ion - E_i)/T} / (2 Q_+)
 *     (the LTE population per ion-electron pair in Kirchhoff's law), with the
 *     synthetic hydrogenic shape sigma_i(nu) = sigma0_i (nu_i / nu)^3;
 *   free-free: kappa = N_+ n_e sigma_H(s, T) (1 + D), D = 0 (the normalization
 *     table is not available), eta = B(nu, T) kappa. */
void orc_continuum(const orc_species *sp, const orc_cells *C, int n_cont, const orc_cont *cont,
                   double nu_min, double h, int64_t n_k, const int64_t *ks, double *eta, double *kappa)
{
    const double c2 = orc_c2();
    const double nu_H = 1e7 / 91.1267;
    for (int64_t c = 0; c < C->n_cells; ++c) {
        double T = C->T_v[c];
        for (int r = 0; r < n_cont; ++r) {
            const orc_cont *q = &cont[r];
            int a = q->species;
            double Na = C->N[c * C->n_species + a];
            double Np = C->N[c * C->n_species + q->ion];
            double ne = C->n_e[c];
            double Qa = orc_partition(sp, a, C->T_v[c], C->T_tr[c]);
            const double *Nlev = orc_cell_levels(sp, C, c, a);
            for (int64_t t = 0; t < n_k; ++t) {
                double nu = nu_min + (double)ks[t] * h;
                double B = orc_planck(nu, T);
                double kap = 0.0, em = 0.0;
                for (int64_t i = sp->lev_off[a]; i < sp->lev_off[a + 1]; ++i) {
                    int64_t li = i - sp->lev_off[a];
                    double Ei = sp->lev_E[i], gi = sp->lev_g[i];
                    double nui = q->E_ion - Ei;
                    if (q->sigma0[li] == 0.0 || !(nui > 0.0) || nu < nui) continue;
                    double sig = q->sigma0[li] * pow(nui / nu, 3.0);
                    double Ni = Nlev ? Nlev[li] : (Qa > 0.0) ? Na * gi * exp(-c2 * Ei / T) / Qa : 0.0;
                    kap += Ni * sig;
                    em += B * sig * Np * ne * orc_saha_volume(T) * gi * exp(c2 * (q->E_ion - Ei) / T)
                          / (2.0 * q->Q_ion);
                }
                double ff = Np * ne * orc_peach_ff(q->peach, q->z, nu / nu_H, T);
                kap += ff;
                em += B * ff;
                kappa[c * n_k + t] += kap;
                eta[c * n_k + t] += em;
            }
        }
    }
}

/* Sec. 2.2.3, Johnston-Mazaheri segment with linear j: over [s_i, s_{i+1}]
 * kappa is the far node's value and j varies linearly.  Integrating the
 * transfer equation over the segment (the derivation printed with the scheme)
 * gives, with t = kappa ds and f(t) = (1 - e^{-t}) / t,
 *   I_{i+1} = I_i e^{-t} + ds [ W_far(t) j_i + W_near(t) j_{i+1} ],
 *   W_near(t) = (1 - f(t)) / t,   W_far(t) = (f(t) - e^{-t}) / t.
 * (The closing formula of the scheme pairs these two coefficients with the
 * other node; its own derivation, and the limit t -> infinity where only the
 * node next to the target can matter, fix the pairing used here.)
 * Where t is small both differences cancel, so there the weights come from
 * their Taylor series (the paper's thin-layer branch, carried to double
 * precision):  W_near(t) = sum_{n>=0} (-t)^n / (n+2)!,
 *              W_far(t)  = sum_{n>=0} (-1)^n (n+1) t^n / (n+2)!.            */
void orc_linear_j_weights(double t, double *w_far, double *w_near)
{
    if (fabs(t) >= 0.05) {
        double e = exp(-t);
        double f = -expm1(-t) / t;
        *w_near = (1.0 - f) / t;
        *w_far = (f - e) / t;
        return;
    }
    double a = 0.0, b = 0.0, fact = 2.0, tn = 1.0;   /* fact = (n+2)!, tn = (-t)^n */
    for (int n = 0; n < 20; ++n) {
        a += tn / fact;
        b += (n + 1) * tn / fact;
        tn *= -t;
        fact *= (double)(n + 3);
    }
    *w_near = a;
    *w_far = b;
}

/* March over nodes 0..n_node-1 (far -> target): node i carries the cell
 * node_cell[i] whose eta/kappa it takes, dsn[i] is the distance from node i
 * to node i+1.  I starts from I_far (NULL: 0) at node 0. */
void orc_march_nodes(int64_t n_node, const int64_t *node_cell, const double *dsn,
                     int64_t n_k, const double *eta, const double *kappa,
                     const double *I_far, double *I_out)
{
    for (int64_t k = 0; k < n_k; ++k) {
        double I = I_far ? I_far[k] : 0.0;
        for (int64_t i = 0; i + 1 < n_node; ++i) {
            double kap = kappa[node_cell[i] * n_k + k];
            double j_far = eta[node_cell[i] * n_k + k];
            double j_near = eta[node_cell[i + 1] * n_k + k];
            double wf, wn;
            orc_linear_j_weights(kap * dsn[i], &wf, &wn);
            I = I * exp(-kap * dsn[i]) + dsn[i] * (wf * j_far + wn * j_near);
        }
        I_out[k] = I;
    }
}

/* ---------------------------------------------------------------------- */
/* Sec. 2.2.3 ray geometry: axisymmetric cell traversal                      */
/* ---------------------------------------------------------------------- */

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Segments of the ray from wall point (x = 0, radius rw) with direction
 * (mu, sqrt(1-mu^2) cos phi, sqrt(1-mu^2) sin phi) through the nx x nr
 * grid on [0, Lx] x [0, R] (cell c = ix * nr + ir).  All crossings of the
 * x-planes and r-shells before the exit are collected and sorted; each piece
 * between consecutive crossings is assigned the cell of its midpoint.
 * Output order is far -> wall.  Returns the segment count (<= cap), or -1
 * when cap is too small. */
int64_t orc_axi_segments(int nx, int nr, double Lx, double R, double rw,
                         double mu, double phi, int64_t cap, int64_t *cell_out, double *ds_out)
{
    double st = sqrt(1.0 - mu * mu);
    double a = st * cos(phi), b = st * sin(phi);
    double dx = Lx / nx, dr = R / nr;
    /* exit: x = Lx or rho = R (largest root) */
    double s_exit = (mu > 0.0) ? Lx / mu : INFINITY;
    double A2 = a * a + b * b;
    if (A2 > 0.0) {
        double disc = rw * rw * a * a - A2 * (rw * rw - R * R);
        double sR = (-rw * a + sqrt(disc)) / A2;
        if (sR < s_exit) s_exit = sR;
    }
    int64_t nb_cap = (int64_t)nx + 2 * (int64_t)nr + 4;
    double *bp = (double *)malloc(sizeof(double) * nb_cap);
    int64_t nb = 0;
    bp[nb++] = 0.0;
    bp[nb++] = s_exit;
    for (int i = 1; i < nx; ++i) {
        double s = i * dx / mu;
        if (mu > 0.0 && s > 0.0 && s < s_exit) bp[nb++] = s;
    }
    if (A2 > 0.0) {
        /* A wall point on a radial face gives a root at s = 0 that rounding can
         * move to ~1e-15: a crossing within 1e-12 of the domain size of the
         * wall point is the wall point itself, not the start of a segment. */
        double s_min = 1e-12 * (Lx + R);
        for (int j = 1; j < nr; ++j) {
            double rj = j * dr;
            double disc = rw * rw * a * a - A2 * (rw * rw - rj * rj);
            if (disc < 0.0) continue;
            double sq = sqrt(disc);
            double r1 = (-rw * a - sq) / A2, r2 = (-rw * a + sq) / A2;
            if (r1 > s_min && r1 < s_exit) bp[nb++] = r1;
            if (r2 > s_min && r2 < s_exit && r2 != r1) bp[nb++] = r2;
        }
    }
    qsort(bp, (size_t)nb, sizeof(double), cmp_double);
    int64_t n = 0;
    for (int64_t t = nb - 1; t >= 1; --t) {   /* far -> wall */
        double s0 = bp[t - 1], s1 = bp[t];
        if (!(s1 > s0)) continue;
        double sm = 0.5 * (s0 + s1);
        double xm = sm * mu;
        double ym = rw + sm * a, zm = sm * b;
        double rho = sqrt(ym * ym + zm * zm);
        int ix = (int)floor(xm / dx), ir = (int)floor(rho / dr);
        if (ix < 0) ix = 0;
        if (ix >= nx) ix = nx - 1;
        if (ir < 0) ir = 0;
        if (ir >= nr) ir = nr - 1;
        if (n >= cap) { free(bp); return -1; }
        cell_out[n] = (int64_t)ix * nr + ir;
        ds_out[n] = s1 - s0;
        ++n;
    }
    free(bp);
    return n;
}

/* Knife edges: (cell, grid index) of window bounds whose real-valued position
 * (nu0 -+ 100 gV - nu_min)/h lies within tol (grid steps) of an integer.  At such a point
 * a one-ulp difference in gV between two correct implementations moves the
 * bound, so comparisons exclude it.  Cells are scanned in parallel; cell c
 * writes at most cap_per_cell entries at cell_out/k_out + c * cap_per_cell and
 * its count to count_out[c]. */
void orc_knife_edges(const orc_species *sp, const orc_lines *L, const orc_cells *C,
                     double nu_min, double nu_max, int64_t n_points, double tol,
                     int64_t cap_per_cell, int64_t *cell_out, int64_t *k_out, int64_t *count_out)
{
    const double h = (nu_max - nu_min) / (double)(n_points - 1);
    const int S = C->n_species;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t c = 0; c < C->n_cells; ++c) {
        int64_t n = 0;
        int64_t *co = cell_out + c * cap_per_cell, *ko = k_out + c * cap_per_cell;
        for (int64_t i = 0; i < L->n; ++i) {
            int s = L->species[i];
            double Ns = C->N[c * S + s];
            if (sp->kind[s] == 0 || Ns <= 0.0) continue;
            double gG = orc_doppler_hwhm(L->nu0[i], C->T_tr[c], sp->mass[s]);
            double gL = orc_lorentz_line(sp, L, i, C->T_tr[c], C->T_v[c], C->n_e[c], C->N + c * S, S);
            double W = 100.0 * orc_voigt_hwhm(gL, gG);
            double b[2] = {(L->nu0[i] - W - nu_min) / h, (L->nu0[i] + W - nu_min) / h};
            for (int e = 0; e < 2; ++e) {
                double r = nearbyint(b[e]);
                if (fabs(b[e] - r) <= tol && r >= -1 && r <= (double)n_points) {
                    for (int64_t d = -1; d <= 1; ++d) {
                        int64_t k = (int64_t)r + d;
                        if (k < 0 || k >= n_points) continue;
                        if (n < cap_per_cell) { co[n] = c; ko[n] = k; }
                        ++n;
                    }
                }
            }
        }
        count_out[c] = n < cap_per_cell ? n : cap_per_cell;
    }
}
