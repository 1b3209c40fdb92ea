/*
 * lrt.h -- C ABI of liblrt, an MI355X (gfx950) implementation of the
 * line-by-line + ray-tracing radiation hot path of arXiv 2604.11856:
 *
 *   per-cell Boltzmann populations (Sec. 2.1)
 *     -> per-(cell, line) emission / absorption strengths, Doppler, Lorentz
 *        and Voigt widths (Sec. 2.2.1)
 *     -> line-to-grid accumulation of the Whiting-Voigt profile into the
 *        spectral emission coefficient eta and absorption coefficient kappa
 *        of every cell (Sec. 2.2.1)
 *     -> march of the radiative transfer equation along rays, far boundary
 *        to wall, with piecewise-constant cells (Sec. 2.2.3)
 *     -> spectral (trapezoid) and angular (Gauss-Legendre polar x uniform
 *        azimuth) quadrature to the wall radiative heat flux (Sec. 2.2.3).
 *
 * Conventions for every call:
 *   - Units: wavenumber and level energies in cm^-1, temperatures in K,
 *     number densities in cm^-3, lengths in cm.  eta in W cm^-3 sr^-1
 *     (cm^-1)^-1, kappa in cm^-1, intensity in W cm^-2 sr^-1 (cm^-1)^-1,
 *     spectrally integrated intensity in W cm^-2 sr^-1, flux in W cm^-2.
 *   - Every entry returns an lrt_status; nothing throws or aborts across the
 *     ABI.  Arguments are validated before any device work; on error nothing
 *     has been launched and lrt_last_error() describes the failure.
 *   - Host pointers are read during the call only and never retained.  The
 *     library owns the context and the device copies of species, lines,
 *     grid, cells and rays.  The caller owns every output buffer.
 *   - "stream" is a hipStream_t passed as void* (NULL = default stream).
 *     Calls that write only device buffers are stream-ordered and return
 *     before the work is done; calls that write host buffers synchronise.
 *   - One context is used by one host thread at a time.
 */
#ifndef LRT_H
#define LRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lrt_ctx lrt_ctx;

typedef enum {
    LRT_OK = 0,
    LRT_E_ARG = 1,        /* invalid argument (value, size, pointer) */
    LRT_E_OOM = 2,        /* device or host allocation failed */
    LRT_E_DEVICE = 3,     /* HIP runtime error (message in lrt_last_error) */
    LRT_E_BUDGET = 4,     /* request larger than the configured memory budget */
    LRT_E_NOT_READY = 5,  /* result not available yet */
    LRT_E_STATE = 6       /* call made in the wrong state (missing set_* call) */
} lrt_status;

typedef enum {
    LRT_FP64 = 0,       /* every step in double precision */
    LRT_FP32_COMP = 1   /* populations, widths, windows and quadrature in double;
                           profile evaluation in single precision; at each grid
                           point lines are summed in blocks of 64 whose partials
                           are merged with Kahan's compensation; eta/kappa stored
                           as float with a per-cell power-of-two scale */
} lrt_precision;

enum { LRT_KIND_NONE = 0, LRT_KIND_ATOM = 1, LRT_KIND_MOLECULE = 2 };

/* Level table of one species (Sec. 2.1).
 * kind == LRT_KIND_ATOM: n_levels electronic levels (energy level_E, degeneracy
 *   level_g); Q = sum_j g_j exp(-c2 E_j / T_v).
 * kind == LRT_KIND_MOLECULE: n_el electronic states (term el_T, degeneracy el_g)
 *   with el_nv[e] vibrational levels each (term values vib_G, rotational
 *   constants vib_B, vib_D, concatenated over e) and J = 0..el_Jmax[e];
 *   Q = sum_e g_e exp(-c2 T_e/T_v) sum_v exp(-c2 G_v/T_v)
 *       sum_J (2J+1) exp(-c2 (B_v J(J+1) - D_v J^2(J+1)^2) / T_tr).
 *   Symmetry number and line-alternation factor are taken as 1.  A state
 *   has at most 2^30 (v, J) terms.
 * kind == LRT_KIND_NONE: species that carries no lines (number density only).
 * mass: molar mass in g/mol (Doppler width). */
typedef struct {
    int kind;
    double mass;
    int n_levels;
    const double *level_E, *level_g;
    int n_el;
    const double *el_T, *el_g;
    const int *el_nv, *el_Jmax;
    const double *vib_G, *vib_B, *vib_D;
} lrt_species;

/* Line list, structure of arrays, any order (Sec. 2.2.1-2.2.2).
 * nu0 > 0 line centre; A >= 0 Einstein coefficient (s^-1); upper / lower level
 * energy split into an electronic+vibrational part (populated at T_v) and a
 * rotational part (populated at T_tr; 0 for atoms); gu, gl >= 1 level
 * degeneracies; species indexes the species table.  Host pointers
 * (on_device == 0) or device pointers of the context's device (on_device !=
 * 0, e.g. the output of lrt_gen_rovib_lines), read during the call only. */
typedef struct {
    int64_t n;
    const double *nu0, *A, *Eu_ev, *Eu_rot, *El_ev, *El_rot, *gu, *gl;
    const int32_t *species;
    int on_device;
} lrt_lines;

/* One electronic band system of a diatomic radiator, upper state u -> lower
 * state l (Sec. 2.2.2), the input of lrt_gen_rovib_lines.  Per state: |Lambda|,
 * electronic term T_e and degeneracy factor g_e (a level's degeneracy is
 * g_e (2J + 1)), vibrational constants w_e, w_e x_e, w_e y_e (vibrational
 * term E_V = w_e (V + 1/2) - w_e x_e (V + 1/2)^2 + w_e y_e (V + 1/2)^3),
 * rotational constants B_e, alpha_e, D_e, beta_e (B_v = B_e - alpha_e
 * (V + 1/2), D_v = D_e + beta_e (V + 1/2)), spin-rotation constant gamma,
 * all in cm^-1, and nv vibrational levels V = 0..nv-1.  hund: LRT_HUND_A
 * (rotational term B_v J(J+1) - D_v J^2 (J+1)^2; Hoenl-London factors of
 * the case (a) table for Lambda_u, Lambda_l with |dLambda| <= 1; levels J >=
 * Lambda; J_u = 0..J_max with its P, Q and R lines) or LRT_HUND_B (a doublet
 * Sigma-Sigma system: levels N = J - S, S = +-1/2, term B_v N(N+1) -
 * D_v N^2 (N+1)^2 + S gamma (N + 1/2 - S); Hoenl-London factors of the case
 * (b) table in J_l; lower levels N_l = 0..J_max, from each a P and an R line
 * keeping the spin component and a Q line changing it).  Re2 (host,
 * [nv_u][nv_l]): the squared rotationless transition moment Re'^2 = Re^2
 * F_vv of each band in units of e a0.  A line exists when both of its levels
 * do and its Hoenl-London factor is positive. */
enum { LRT_HUND_A = 0, LRT_HUND_B = 1 };
typedef struct {
    int32_t species;       /* the molecule (an LRT_KIND_MOLECULE species) */
    int32_t hund;
    int32_t Lambda_u, Lambda_l;
    double Te_u, Te_l, g_u, g_l;
    double we_u, wexe_u, weye_u, Be_u, ae_u, De_u, be_u, gamma_u;
    double we_l, wexe_l, weye_l, Be_l, ae_l, De_l, be_l, gamma_l;
    int32_t nv_u, nv_l, J_max;
    const double *Re2;
} lrt_band_system;

/* Output arrays of a generated line list (device pointers, caller-owned,
 * capacity given to the call). */
typedef struct {
    double *nu0, *A, *Eu_ev, *Eu_rot, *El_ev, *El_rot, *gu, *gl;
    int32_t *species;
} lrt_line_buffers;

/* Flowfield cell states (Sec. 2.3 flowfield interface, the two-temperature
 * state of Sec. 2.1): T_tr translational-rotational temperature, T_v
 * vibrational = electron-electronic temperature, N[c * n_species + s] number
 * densities, n_e electron number density (Lorentz width).  Structure of
 * arrays owned by the caller: host pointers (on_device == 0) or device
 * pointers of the context's HIP device (on_device != 0); read during the call
 * only. */
typedef struct {
    int64_t n_cells;
    int n_species;
    const double *T_tr, *T_v, *N, *n_e;
    int on_device;
} lrt_cells;

/* Library version as "major.minor.patch". */
const char *lrt_version(void);

/* Text of a status code (static storage). */
const char *lrt_status_string(lrt_status s);

/* Create a context on HIP device `device`.  *out receives the context, or NULL
 * on failure.  Errors: LRT_E_ARG (bad device or out == NULL), LRT_E_DEVICE. */
lrt_status lrt_create(int device, lrt_ctx **out);

/* Destroy a context and free its device memory.  NULL is accepted. */
void lrt_destroy(lrt_ctx *ctx);

/* Message of the last failed call on this context ("" if none); valid until
 * the next call on the context.  NULL ctx returns the last lrt_create error. */
const char *lrt_last_error(const lrt_ctx *ctx);

/* Species level tables (copied).  Must precede lrt_set_lines/lrt_set_cells.
 * Errors: LRT_E_ARG on n_species < 1, non-positive mass, unknown kind, a
 * molecule / atom without levels, non-finite values. */
lrt_status lrt_set_species(lrt_ctx *ctx, int n_species, const lrt_species *species);

/* Line list (copied to device memory, sorted by nu0 there, kept resident;
 * device arrays are copied to the host first, then handled alike).
 * Errors: LRT_E_ARG (nu0 <= 0, A < 0, g < 1, non-finite energy, species index
 * out of range or pointing to a species of kind NONE), LRT_E_STATE (no
 * species), LRT_E_OOM. */
lrt_status lrt_set_lines(lrt_ctx *ctx, const lrt_lines *lines);

/* Uniform spectral grid of the line-by-line evaluation (Sec. 2.2.1: each
 * line's profile is evaluated at the nodes of a spectral grid, at the
 * distance of the node from the line centre; Sec. 2.2.3: the spectral
 * integral of the wall intensity runs over the same nodes): nu_k = nu_min + k h, h = (nu_max - nu_min) / (n_points - 1), both
 * ends included, processed in bands of band_points points (the last band may
 * be shorter).  Errors: LRT_E_ARG (n_points < 2, nu_max <= nu_min,
 * nu_min <= 0, band_points < 1, n_points >= 2^31). */
lrt_status lrt_set_grid(lrt_ctx *ctx, double nu_min, double nu_max, int64_t n_points,
                        int64_t band_points);

/* Cell states (copied to device memory, resident).  Device arrays are
 * copied on the device and validated there (the call synchronises the
 * device).  Errors: LRT_E_ARG (n_species differs from the species table,
 * T <= 0 or non-finite, N < 0, n_e < 0; the context then has no cells),
 * LRT_E_STATE (no species), LRT_E_DEVICE. */
lrt_status lrt_set_cells(lrt_ctx *ctx, const lrt_cells *cells);

/* Lorentz width of atomic lines (Sec. 2.2.1 pressure broadening).  With
 * E_ion == NULL (the default) every line has gamma_L = 1e-16 n_e (T_v/1e4)^0.33
 * cm^-1.  With E_ion[s] > 0 (cm^-1, host, [n_species]) the lines of atom s get
 * the sum of the natural width 5.9e-6 nm, the Stark width
 * 1.69e3 lambda^2 / dE^2.623 (T_v/1e4)^0.33 (n_e/1e16) nm with
 * dE = max(E_ion - E_u, E_ion(H)/25), and the van der Waals width
 * lambda^2 [6.65e-29 N_s (2 T_tr/M_s)^0.5 + 2.925e-29 N_o (2 T_tr/M_o)^0.5] nm
 * (N_o, M_o: the other species but electrons, density-weighted molar mass),
 * each converted to cm^-1 by dnu = 1e7 dlambda / lambda^2 (lambda = 1e7/nu0
 * nm); resonance broadening is left out.  Other lines keep the uniform law.
 * Kept until changed; new species clear it.  Errors: LRT_E_STATE (no
 * species), LRT_E_ARG (negative or non-finite E_ion). */
lrt_status lrt_set_lorentz(lrt_ctx *ctx, const double *E_ion);

/* Atomic continuum of one atom (Sec. 2.2.1 bound-free and free-free), added
 * to eta and kappa of every cell and grid point by lrt_coeffs and lrt_solve.
 * With T = T_v (the electron temperature), N_a, N_+ the cell's densities of
 * `species` and `ion`, n_e its electron density and nu in cm^-1:
 *   bound-free from level i of the atom (threshold nu_i = E_ion - E_i,
 *   nu >= nu_i, cross section sigma0[i] (nu_i/nu)^3):
 *     kappa += N_a g_i e^{-c2 E_i/T} / Q_a  sigma_i(nu),
 *     eta   += B(nu, T) sigma_i(nu) N_+ n_e V(T) g_i e^{c2 (E_ion - E_i)/T} / (2 Q_ion),
 *     V(T) = (h^2 / (2 pi m_e k T))^{3/2} (the LTE population per ion-electron
 *     pair, so that eta = B kappa in Saha equilibrium);
 *   free-free (hydrogenic fit, s = nu / (1e7 / 91.1267 cm^-1)):
 *     kappa += N_+ n_e 1e-40 (A1/s + A2) / (z^4 s^3),
 *     A1 = c1 + c2 e^{-c3 T}, A2 = c4 + c5 e^{-c6 T} + c7 e^{-c8 T},
 *     eta += B(nu, T) times that (the fit's normalisation factor D is 0).
 * sigma0 has one entry per level of the atom (0: no bound-free from it); all
 * c zero: no free-free. */
typedef struct {
    int32_t species;       /* the atom (an LRT_KIND_ATOM species) */
    int32_t ion;           /* species index of its singly charged ion */
    double E_ion;          /* ionization energy from the ground level, cm^-1 */
    double Q_ion;          /* partition function of the ion, held constant */
    const double *sigma0;  /* [levels of the atom], cm^2, host */
    double peach[8];       /* c1..c8 of the free-free fit, cm^5 */
    double z;              /* ion charge in the free-free fit */
} lrt_continuum;

/* Set (n > 0) or clear (n = 0) the continuum records; copied.  Errors:
 * LRT_E_STATE (no species), LRT_E_ARG (species not an atom, index out of
 * range, E_ion, Q_ion or z <= 0, negative or non-finite sigma0). */
lrt_status lrt_set_continuum(lrt_ctx *ctx, int n, const lrt_continuum *cont);

/* Quasi-steady-state collisional-radiative (QSS-CR) data of one atom or
 * diatomic molecule (Sec. 2.1 CR model, master equation in QSS form,
 * ground-state closure, R n = b solved by LU).  The states are the atom's
 * table levels (energies E_i, degeneracies g_i) or the molecule's electronic
 * states (terms T_e, with their vibrational and rotational ladders).  With
 * l = n_model, states 0..l-1 are solved for in every cell; the states above
 * stay in Boltzmann ratio with state l-1 at (T_v, T_tr) (the closure row sums
 * all of them to the species' density N).  Row i >= 1 balances state i: its
 * losses by heavy-particle (HPIE) and electron impact (EIE) transitions to
 * every other solved state, spontaneous emission to lower states, and
 *   atoms: electron impact ionization (EII) and charge exchange (CE) with the
 *   partner ion;
 *   molecules: heavy-particle (HPID) and electron impact (EID) dissociation
 *   into diss_x + diss_y;
 * against its gains by the same transitions from the other states and, as
 * sources b, three-body recombination of the ion, charge exchange of the ion
 * with the partner atom, or three-body recombination of the dissociation
 * products.  Two-body rates are k / N_A times the collider density (heavy
 * colliders: sum over species of collider_w[s] N_s; electrons: n_e).
 * Forward rate coefficients are Arrhenius triples (C, n, E_a): k = C T^n
 * e^{-E_a/T} (cm^3 mol^-1 s^-1, E_a in K); reverse rates follow detailed
 * balance at the backward temperature T_b:
 *   de-excitation hi -> lo:  [k(lo -> hi) Q_lo / Q_hi]_{T_b},
 *   recombination into i:    [k_EII(i) Q_i / (Q_ion e^{-c2 E_ion/T} Q_e)]_{T_b},
 *   CE into i:               [k_CE(i) Q_i Q_B+ / (Q_A+ Q_B)]_{T_b},
 *   X + Y into i:            [k_D(i) Q_i / (Q_X Q_Y)]_{T_b} (h^2/(2 pi mu k T_b))^{3/2}
 *                            e^{c2 E_diss / T_b},
 * with Q_i = g_i e^{-c2 E_i/T} for an atomic level and g_e e^{-c2 T_e/T}
 * Q_vr,e(T) for a molecular state (every mode at T), Q_A+ = Q_ion
 * e^{-c2 E_ion/T}, Q_B+ likewise for the partner, Q_B the partner's full
 * partition function, Q_e = 2 (2 pi m_e k T / h^2)^{3/2}, Q_X and Q_Y the
 * level sums of atomic products (else the constants Q_x, Q_y), mu the pair's
 * reduced mass.  Rates of mechanism m (0 HPIE, 1 EIE, 2 EII, 3 CE, 4 HPID,
 * 5 EID) are taken at T = T_tr^a T_v^(1-a) with a = texp[2m] (forward) and
 * texp[2m+1] (backward).  The escape factor is 0 (optically thick) for
 * transitions above nu_cut cm^-1 (state energy difference), 1 below;
 * absorption of radiation is left out.  The populations replace the
 * Boltzmann ones for the lines given states by lrt_set_line_levels and for
 * an atom's bound-free absorption.  T_v and T_tr must keep every partition
 * function and e^{c2 E_diss/T} representable (T above a few hundred K).
 * Rate tables are host arrays (copied), row-major: */
typedef struct {
    int32_t species;        /* the atom or molecule (at most 64 levels / electronic states) */
    int32_t ion;            /* atom: species of its singly charged ion, or -1 (ion density 0); molecule: -1 */
    int32_t partner;        /* atom: charge-exchange partner atom, or -1; molecule: -1 */
    int32_t partner_ion;    /* the partner's ion (with a partner) */
    int32_t n_model;        /* l: 2 <= l <= the species' state count */
    int32_t diss_x, diss_y; /* molecule: dissociation products (species), or -1, -1 (none) */
    double E_ion, Q_ion;    /* atom: ionization energy (cm^-1) and partition function of the ion */
    double partner_E_ion, partner_Q_ion;
    double Q_x, Q_y;        /* partition function of a product that is not an atom (> 0) */
    double E_diss;          /* cm^-1: products above the molecule's energy zero */
    double nu_cut;          /* optically thick above, cm^-1 (5e4: 200 nm) */
    double texp[12];        /* temperature exponents, each in [0, 1] */
    const double *hpie;     /* [l][l][3]: HPIE lo -> hi at [lo][hi] (lo < hi; rest ignored) */
    const double *eie;      /* [l][l][3]: EIE likewise */
    const double *A;        /* [l][l]: spontaneous emission hi -> lo at [hi][lo], s^-1 */
    const double *eii;      /* [l][3]: atom: EII of each level (row 0 unused) */
    const double *ce;       /* [l][3]: atom: CE of each level (ignored without a partner) */
    const double *hpid;     /* [l][3]: molecule: HPID of each state (row 0 unused) */
    const double *eid;      /* [l][3]: molecule: EID of each state (row 0 unused) */
} lrt_cr_species;

/* Set (n > 0) or clear (n = 0) the QSS-CR species, at most one record per
 * species; collider_w (host, [n_species]) weights the species as heavy
 * colliders (0 for electrons).  Copied; kept until changed; new species clear
 * it.  The populations are recomputed with the other per-cell quantities.
 * Errors: LRT_E_STATE (no species), LRT_E_ARG (species neither atom nor
 * molecule or with more than 64 states, index out of range, duplicate
 * species, l out of range, an atom's E_ion or Q_ion <= 0, ionization or
 * charge exchange given to a molecule, dissociation given to an atom, a
 * non-atomic product without Q > 0, texp outside [0, 1], negative or
 * non-finite rate data or collider weight, NULL table). */
lrt_status lrt_set_cr(lrt_ctx *ctx, int n, const lrt_cr_species *sp, const double *collider_w);

/* Upper and lower state of every line (host, [n_lines] each, in the order the
 * lines were given to lrt_set_lines): a level of its atom's table, or an
 * electronic state of its molecule; -1 for both: such a line keeps Boltzmann
 * populations, as does every line of a species without QSS-CR data.  A line
 * with states takes N_u = N_CR(u) times its Boltzmann share of that state
 * (an atom's line g e^{-c2 (E - E_u)/T_v} g_u^-1, 1 when its E and g are the
 * level's; a molecule's rovibronic level g e^{-c2 E_ev/T_v - c2 E_rot/T_tr}
 * / Q_u(T_v, T_tr)), likewise N_l, and kappa from N_l g_u/g_l - N_u.  Both
 * NULL: clear.  Copied; new lines clear it.  Errors: LRT_E_STATE (no lines),
 * LRT_E_ARG (n != n_lines, one of the two states -1, a state outside its
 * species' table). */
lrt_status lrt_set_line_levels(lrt_ctx *ctx, const int32_t *lev_u, const int32_t *lev_l, int64_t n);

/* The QSS-CR state populations (cm^-3) of record `rec` (as given to
 * lrt_set_cr) in every cell: pop (host, [n_cells][states of the species]).
 * Computes the per-cell quantities if they are not current.  A cell without
 * the species has all zero; a singular system gives NaN.  Synchronises the
 * stream.  Errors: LRT_E_STATE (no QSS-CR data, cells missing), LRT_E_ARG. */
lrt_status lrt_cr_populations(lrt_ctx *ctx, int rec, double *pop, void *stream);

/* Rays of a 1-D slab seen from the wall (Sec. 2.2.3 with a tangent-slab
 * geometry): cells 0..n_cells-1 ordered from the far (free) boundary to the
 * wall with thicknesses dx (host).  Ray 0 is the wall normal; if n_mu > 0,
 * rays 1..n_mu follow the Gauss-Legendre nodes mu_i on [0, 1] with path
 * length dx/mu_i per cell and flux weight 2 pi W_i mu_i (ray 0 has weight 0).
 * One wall point.  Errors: LRT_E_ARG (n_cells < 1, dx <= 0, n_mu < 0). */
lrt_status lrt_set_rays_slab(lrt_ctx *ctx, int64_t n_cells, const double *dx, int n_mu);

/* Rays of an axisymmetric structured grid (Sec. 2.2.3, LOS through the
 * flowfield): nx x nr uniform cells over x in [0, Lx], r in [0, R], cell index
 * c = ix * nr + ir.  The wall is the plane x = 0; wall point w sits at radius
 * wall_r[w] (host) and sees rays of direction (mu_i, sin cos phi_j, sin sin
 * phi_j) with mu_i Gauss-Legendre on [0, 1] and phi_j = (j + 1/2) 2 pi / n_phi,
 * flux weight W_i mu_i 2 pi / n_phi.  Rays end at x = Lx or r = R (free
 * boundary, I = 0); the axis is transparent.  Segments are built on the host
 * in double precision by cell-to-cell traversal.
 * Errors: LRT_E_ARG (non-positive sizes, wall_r outside [0, R), n_mu or
 * n_phi < 1). */
lrt_status lrt_set_rays_axi(lrt_ctx *ctx, int nx, int nr, double Lx, double R, int n_wall,
                            const double *wall_r, int n_mu, int n_phi);

/* Rays of the axisymmetric grid of lrt_set_rays_axi along Fibonacci-sphere
 * lines of sight (Sec. 2.2.3): of n_los directions i = 1..n_los with polar
 * component w = 1 - 2(i-1)/(n_los-1) along the wall normal (+x) and azimuth
 * (i-1)(sqrt 5 - 1) pi, those with w > 0 are traced from every wall point.
 * Flux weights: the LOS results are carried to the nodes of a uniform grid of
 * n_polar polar intervals on [0, pi/2] and n_azim azimuth intervals on
 * [0, 2 pi] (each node takes its nearest LOS), and each grid cell adds the mean
 * of its four corners times its integral of sin(phi) cos(phi) dphi dtheta;
 * the weights of a wall point sum to pi.  All symmetry is ignored: every
 * direction is traced.  Errors: LRT_E_ARG (non-positive sizes, n_los < 3,
 * wall_r outside [0, R)). */
lrt_status lrt_set_rays_axi_fibonacci(lrt_ctx *ctx, int nx, int nr, double Lx, double R, int n_wall,
                                      const double *wall_r, int n_los, int n_polar, int n_azim);

/* Host-only (no device, no context): the directions (dirs[3*i..3*i+2], unit,
 * normal component first) and flux weights of lrt_set_rays_axi_fibonacci's
 * angular rule; *n receives the number of directions with a positive normal
 * component, at most cap are written.  Errors: LRT_E_ARG (bad sizes, cap too
 * small). */
lrt_status lrt_fibonacci_quadrature(int n_los, int n_polar, int n_azim, int64_t cap, double *dirs,
                                    double *weights, int64_t *n);

/* March scheme used by lrt_march and lrt_solve (Sec. 2.2.3).
 *   LRT_MARCH_CELL: piecewise-constant cells along each segment,
 *     I <- I e^{-tau} + eta ds F(tau) (the default).
 *   LRT_MARCH_LINEAR_J: the Johnston-Mazaheri segment with kappa from the far
 *     node and j linear between LOS nodes, placed at the far end of each ray,
 *     the midpoint of every cell segment and the target (a node takes the
 *     state of its cell); I <- I e^{-kappa_f L} + L (W_far j_f + W_near j_n),
 *     W_near = (1 - f)/tau, W_far = (f - e^{-tau})/tau, f = (1 - e^{-tau})/tau,
 *     with a Taylor branch for thin segments. */
typedef enum { LRT_MARCH_CELL = 0, LRT_MARCH_LINEAR_J = 1 } lrt_march_scheme;

/* Select the march scheme (kept until changed).  Errors: LRT_E_ARG. */
lrt_status lrt_set_march(lrt_ctx *ctx, lrt_march_scheme scheme);

/* Far boundary of every ray (Sec. 2.2.3): a solid surface at temperature
 * T_far starts the march with the blackbody intensity B(nu, T_far); 0 means a
 * free boundary (I = 0).  n = 1 applies T_far[0] to every ray, n = n_rays
 * gives one value per ray (host array), n = 0 makes every ray free again.
 * Setting new rays resets all rays to free.  Errors: LRT_E_STATE (no rays),
 * LRT_E_ARG (n not 0, 1 or n_rays; T < 0 or non-finite). */
lrt_status lrt_set_far_temperature(lrt_ctx *ctx, const double *T_far, int64_t n);

/* Host-only (no device, no context): segments of one ray of the axisymmetric
 * geometry of lrt_set_rays_axi, from wall radius rw along (mu, sqrt(1-mu^2)
 * cos phi, sqrt(1-mu^2) sin phi), far -> wall order, at most cap entries.
 * *n receives the count.  Errors: LRT_E_ARG (bad sizes, mu not in (0, 1],
 * rw outside [0, R), cap too small). */
lrt_status lrt_trace_axi_ray(int nx, int nr, double Lx, double R, double rw, double mu, double phi,
                             int64_t cap, int32_t *cell, double *ds, int64_t *n);

/* Sizes of the current state: cells, rays, wall points, grid points, bands,
 * band length (0 for what is not set).  Any pointer may be NULL. */
lrt_status lrt_get_sizes(const lrt_ctx *ctx, int64_t *n_cells, int64_t *n_rays, int64_t *n_wall,
                         int64_t *n_points, int64_t *n_bands, int64_t *band_points);

/* Copy ray r's segments to host: up to cap entries of cell index and path
 * length, far -> wall order; *n receives the segment count, *weight the flux
 * weight and *wall the wall point of the ray.  Errors: LRT_E_ARG (r out of
 * range, cap < count). */
lrt_status lrt_get_ray(const lrt_ctx *ctx, int64_t r, int64_t cap, int32_t *cell, double *ds,
                       int64_t *n, double *weight, int64_t *wall);

/* Emission and absorption coefficients of every cell on band `band`
 * (grid indices [band * band_points, min(n_points, (band+1) * band_points)))
 * (Sec. 2.1 populations, Sec. 2.2.1 bound-bound emission, absorption and
 * Voigt profile, cut at +-100 Voigt HWHM).  eta and kappa are device buffers
 * of [n_cells][band_len] doubles (LRT_FP64) or floats (LRT_FP32_COMP).  For
 * LRT_FP32_COMP, escale (device, [n_cells][2] int32) receives per cell the
 * power-of-two scale of eta and of kappa: value = stored * 2^escale (0 when
 * the cell is representable unscaled); escale may be NULL for LRT_FP64.
 * Large grids are launched in pieces; the band's 512-point tiles times the
 * cells must stay below 2^32 (LRT_E_DEVICE otherwise).
 * Stream-ordered.  Errors: LRT_E_STATE (species, lines, grid or cells
 * missing), LRT_E_ARG (band out of range, NULL buffer, unknown precision). */
lrt_status lrt_coeffs(lrt_ctx *ctx, int64_t band, lrt_precision prec, void *eta, void *kappa,
                      int32_t *escale, void *stream);

/* March every ray through eta / kappa of band `band` (as written by
 * lrt_coeffs with the same precision) and integrate over the band's grid
 * points (Sec. 2.2.3): per ray and point, starting from the far boundary's
 * intensity (0, or B(nu, T_far) of lrt_set_far_temperature), with the scheme
 * of lrt_set_march; by default I <- I exp(-tau) + eta ds F(tau),
 * tau = kappa ds, F(t) = (1 - e^-t)/t, F(0) = 1.  I_out (device, [n_rays][band_len] doubles) receives the wall
 * intensity, or pass NULL; I_int_out (device, [n_rays] doubles) receives the
 * band's trapezoid sum with global-index weights (h/2 at grid ends, h inside).
 * The march works on chunks of 128 grid points when the rays cross each
 * cell at least 128 times on average (segments / cells), else of 256; the
 * rays over 4 times the band's chunks must stay below 2^32 (LRT_E_DEVICE
 * otherwise).
 * Stream-ordered.  Errors: LRT_E_STATE (no rays, cells/rays mismatch),
 * LRT_E_ARG. */
lrt_status lrt_march(lrt_ctx *ctx, int64_t band, lrt_precision prec, const void *eta,
                     const void *kappa, const int32_t *escale, double *I_out, double *I_int_out,
                     void *stream);

/* lrt_march for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same arguments, kernels and results as lrt_march, but the per-(ray, chunk)
 * partial sums of the spectral trapezoid go to a static device array of the
 * library (2^23 doubles, 64 MiB, held on each device the library runs on
 * until the process ends) instead of a workspace the context allocates; no
 * launch is profiled.  Calls that overlap on one device share that array and
 * race.  Errors: as lrt_march, and LRT_E_ARG when the rays times the band's
 * chunks (as lrt_march describes) exceed 2^23. */
lrt_status lrt_march_noalloc(lrt_ctx *ctx, int64_t band, lrt_precision prec, const void *eta,
                             const void *kappa, const int32_t *escale, double *I_out, double *I_int_out,
                             void *stream);

/* The whole path of Sec. 2.2.3 (steps: populations of every cell, Sec. 2.1;
 * emission and absorption coefficients on the grid, Sec. 2.2.1; the formal
 * solution of the transfer equation along every ray; the wall flux integral
 * over wavenumber and solid angle) over bands first_band..n_bands-1:
 * per-cell populations and scales (recomputed on every call), coefficients,
 * march, spectral and angular quadrature.  Outputs (host, may be NULL): q[n_wall]
 * wall flux summed over the processed bands, I_int[n_rays] spectrally
 * integrated intensity per ray, q_band[n_wall][n_bands] per-band flux (bands
 * before first_band are left untouched, so a run resumed at first_band fills
 * in the rest).  Workspace is allocated by the library and kept for reuse.
 * Synchronises the stream.  Errors: as lrt_coeffs and lrt_march, LRT_E_OOM. */
lrt_status lrt_solve(lrt_ctx *ctx, lrt_precision prec, int64_t first_band, double *q,
                     double *I_int, double *q_band, void *stream);

/* The whole path of lrt_solve over an explicit list of n grid-point ranges
 * [k_first[i], k_first[i] + n_points[i]) instead of the bands (a spectral
 * window of a coupled solver, or a stratified sample of the spectrum): per-cell
 * populations and scales once, then per range the coefficients of every cell,
 * the march of every ray and the flux sums (Sec. 2.2.3 steps as for
 * lrt_solve).  Each range is processed like a band (at most band_points
 * points); the trapezoid weights stay those of the whole grid (h/2 only at
 * its two ends), so ranges that tile the grid sum to lrt_solve's results.
 * Outputs (host, may be NULL): q[n_wall] and I_int[n_rays] summed over the
 * ranges, q_range[n_wall][n] per range.  Synchronises the stream.  Errors:
 * LRT_E_ARG (n < 1, a range outside the grid or longer than band_points, NULL
 * arrays), LRT_E_STATE, LRT_E_OOM, LRT_E_DEVICE. */
lrt_status lrt_solve_ranges(lrt_ctx *ctx, lrt_precision prec, int64_t n, const int64_t *k_first,
                            const int64_t *n_points, double *q, double *I_int, double *q_range,
                            void *stream);

/* Number of in-window (cell, line, grid point) terms of band `band`, i.e. the
 * Voigt evaluations the accumulation performs usefully, and (core_count, may
 * be NULL) how many of them the single-precision form evaluates with the
 * profile's two exponential terms: every point within 25 Voigt HWHM of the
 * line centre (beyond it both terms are exactly zero in single precision)
 * plus at most one point of margin on each side.  Synchronises. */
lrt_status lrt_count_terms(lrt_ctx *ctx, int64_t band, int64_t *count, int64_t *core_count,
                           void *stream);

/* As lrt_count_terms, summed over the grid-point ranges of lrt_solve_ranges
 * (same rules for the ranges).  Synchronises. */
lrt_status lrt_count_terms_ranges(lrt_ctx *ctx, int64_t n, const int64_t *k_first,
                                  const int64_t *n_points, int64_t *count, int64_t *core_count,
                                  void *stream);

/* The rovibronic line list of n band systems on the device (Sec. 2.2.2): for
 * every line, nu0 = E_u - E_l with E = T_e + E_V + E_rot of its state, the
 * molecular Einstein coefficient A = 64 pi^4 nu0^3 (e a0 Re')^2 S_JJ /
 * (3 h (2 J_u + 1)) in CGS (e the elementary charge in statcoulomb, a0 =
 * 5.291772083e-9 cm), the degeneracies g_e (2J + 1), the energies split into
 * T_e + E_V (Eu_ev, El_ev) and E_rot (Eu_rot, El_rot), and the species; lines
 * with nu0 outside [nu_min, nu_max] are dropped.  Order: system, V_u, V_l,
 * then J_u (case a) or N_l and S_l = +1/2, -1/2 (case b), then the branch P,
 * Q, R.  Writes at most cap lines into out (device) and the number of lines
 * to *n_out; cap = 0 (out ignored) only counts them.  Stream-ordered kernels,
 * then the call synchronises the stream.  Errors: LRT_E_ARG (n < 1, a
 * species that is not a molecule, nv < 1, J_max < 0, unknown hund, |dLambda|
 * > 1 in case (a) or Lambda != 0 in case (b), negative or non-finite Re2 or
 * degeneracy, nu_min >= nu_max, cap > 0 below the line count (*n_out is
 * then set)), LRT_E_STATE (no species), LRT_E_OOM, LRT_E_DEVICE. */
lrt_status lrt_gen_rovib_lines(lrt_ctx *ctx, int n, const lrt_band_system *sys, double nu_min, double nu_max,
                               int64_t cap, const lrt_line_buffers *out, int64_t *n_out, void *stream);

/* Kernel families timed by the profiler. */
typedef enum {
    LRT_K_THERMO = 0,   /* partition functions, per-cell constants */
    LRT_K_SCALE = 1,    /* per-cell power-of-two scale (single-precision form) */
    LRT_K_RANGES = 2,   /* candidate line ranges per tile */
    LRT_K_ACCUM = 3,    /* line-to-grid Voigt accumulation */
    LRT_K_MARCH = 4,    /* ray march + spectral trapezoid */
    LRT_K_CR = 5,       /* QSS collisional-radiative populations */
    LRT_K_COUNT = 6
} lrt_kernel;

/* enable != 0: from now on every kernel launch of the context is bracketed by
 * HIP events recorded on the stream it is launched on; any earlier record is
 * discarded.  enable == 0: stop recording and discard. */
lrt_status lrt_profile(lrt_ctx *ctx, int enable);

/* Total device time (ms, from the event pairs) and number of launches of one
 * kernel family since profiling was enabled.  Waits for the recorded events. */
lrt_status lrt_profile_read(lrt_ctx *ctx, int kernel, double *ms, int64_t *launches);

/* Throughput probes of the chip (measurement support, not part of the path):
 * the measured denominators of the roofline beside the nominal peaks. */
typedef enum {
    LRT_PROBE_FMA_F32 = 0,  /* single-precision FMA, lane-ops/s (2 flops each) */
    LRT_PROBE_FMA_F64 = 1,  /* double-precision FMA, lane-ops/s */
    LRT_PROBE_EXP_F32 = 2,  /* v_exp_f32 (2^x), lane-ops/s */
    LRT_PROBE_LOG_F32 = 3,  /* v_log_f32 (log2), lane-ops/s */
    LRT_PROBE_RCP_F32 = 4,  /* v_rcp_f32, lane-ops/s */
    LRT_PROBE_MIX_F32 = 5,  /* a wing term's mix: 3 transcendentals + 10 other
                               single-precision operations, lane-ops/s */
    LRT_PROBE_COPY = 6      /* 4 GiB device-to-device copy, bytes read + written per s */
} lrt_probe_kind;

/* Runs one probe on HIP device `device` (8 waves per SIMD on every compute
 * unit, 8 independent chains per lane; one untimed launch, then one launch
 * timed with HIP events) and returns its rate and time (ms, may be NULL).
 * Allocates and frees its own buffers; synchronises the device.  Errors:
 * LRT_E_ARG (unknown kind or device, rate NULL), LRT_E_OOM, LRT_E_DEVICE. */
lrt_status lrt_probe(int device, int kind, double *rate, double *ms);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of line-of-sight requests                     */
/* ------------------------------------------------------------------------ */

typedef struct lrt_server lrt_server;

/* One line of sight from a coupled flow solver: cells ordered from the far
 * (free) boundary to the observer with path length ds[c] (cm), cell states as
 * in lrt_cells (host pointers, copied at submit), a window of n_window grid
 * points starting at k_first on the context's resident grid, and the species
 * that radiate (bit s of species_mask; 0 = every species): lines of a species
 * outside the mask, and the atomic continuum of an atom outside it, are left
 * out.
 * keep_spectrum != 0 keeps I over the window for lrt_poll / lrt_wait.  T_far
 * (K) is the temperature of a solid far boundary whose blackbody intensity
 * B(nu, T_far) starts the march (Sec. 2.2.3 boundary intensity); 0: a free
 * boundary (intensity 0).  scheme: the segment scheme of the march
 * (lrt_march_scheme: LRT_MARCH_CELL or LRT_MARCH_LINEAR_J, as lrt_set_march
 * describes; the linear-j nodes are the far end, the cell midpoints and the
 * observer). */
typedef struct {
    int64_t n_cells;
    int n_species;
    const double *T_tr, *T_v, *N, *n_e, *ds;
    int64_t k_first, n_window;
    uint64_t species_mask;
    int keep_spectrum;
    double T_far;
    int scheme;
} lrt_los_request;

/* Result of one request: status (LRT_OK, or the error that ended it;
 * LRT_E_STATE for a cancelled request), the spectral integral of the observer
 * intensity over the window (trapezoid, h/2 at both window ends; W cm^-2
 * sr^-1), the window length, and host-clock times from submission to
 * admission and to the result being available (ms). */
typedef struct {
    lrt_status status;
    double I_int;
    int64_t n_window;
    double queue_ms, latency_ms;
} lrt_los_result;

/* Start the serving loop on ctx, whose species, lines and grid must be set
 * (ctx cells and rays are not used; ctx must not be used for other calls until
 * lrt_server_stop).  hbm_budget_bytes of device memory are allocated once and
 * shared by admitted requests; at most max_slots requests are admitted at a
 * time (each slot also holds 8 bytes of pinned host memory, where the device
 * writes the request's integral).  Each request is computed by fused kernels (populations, setups,
 * accumulation and march per spectral tile and chunk of cells, then the
 * chunks composed in order), single-precision compensated profile sums, FP64
 * march state and quadrature; no eta/kappa array is stored.  The context's
 * Lorentz model, atomic continuum and QSS-CR data (lrt_set_lorentz,
 * lrt_set_continuum, lrt_set_cr, lrt_set_line_levels) apply, the CR
 * populations solved for each request's cells at admission (collision
 * partners at the request's densities, whatever its species mask);
 * lrt_set_march and lrt_set_far_temperature do not (a request carries its
 * own far boundary and segment scheme).  Errors:
 * LRT_E_ARG (max_slots < 1, budget < 1 MiB), LRT_E_STATE (missing set_*),
 * LRT_E_OOM, LRT_E_DEVICE. */
lrt_status lrt_server_start(lrt_ctx *ctx, size_t hbm_budget_bytes, int max_slots, lrt_server **out);

/* Copy a request in and queue it; never waits for the GPU.  *ticket receives
 * its handle.  Errors: LRT_E_ARG (invalid cells, ds <= 0, window outside the
 * grid, species count, T_far < 0 or non-finite, unknown scheme), LRT_E_BUDGET (the request could never fit the budget),
 * LRT_E_STATE (server stopping), LRT_E_DEVICE (server failed). */
lrt_status lrt_submit(lrt_server *s, const lrt_los_request *req, uint64_t *ticket);

/* LRT_E_NOT_READY until the request is finished; then fills *out (and the
 * n_window doubles of spectrum, if non-NULL and the request kept it), forgets
 * the ticket and returns LRT_OK.  LRT_E_ARG for an unknown ticket. */
lrt_status lrt_poll(lrt_server *s, uint64_t ticket, lrt_los_result *out, double *spectrum);

/* As lrt_poll, waiting up to timeout_ms (negative: no limit). */
lrt_status lrt_wait(lrt_server *s, uint64_t ticket, double timeout_ms, lrt_los_result *out,
                    double *spectrum);

/* Withdraw a request that has not been admitted yet (its result then reports
 * LRT_E_STATE).  LRT_E_STATE if it is already admitted, LRT_E_ARG if unknown. */
lrt_status lrt_cancel(lrt_server *s, uint64_t ticket);

/* Counters: requests waiting for admission, admitted and not finished,
 * completed so far, epochs launched, arena bytes in use.  Any pointer may be
 * NULL. */
lrt_status lrt_server_info(lrt_server *s, int64_t *pending, int64_t *admitted, int64_t *completed,
                           int64_t *epochs, size_t *bytes_in_use);

/* Finish every queued and admitted request, then free the server.  Results
 * not yet taken are dropped.  NULL is accepted. */
lrt_status lrt_server_stop(lrt_server *s);

#ifdef __cplusplus
}
#endif

#endif /* LRT_H */
