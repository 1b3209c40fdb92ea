"""Plain FP64 CPU oracle of the line-by-line + ray-march path of
arXiv 2604.11856 (Sec. 2.1 populations, Boltzmann or QSS collisional-radiative,
Sec. 2.2.1 line emission / absorption / Voigt shape and atomic continuum,
Sec. 2.2.3 march and flux integral).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does.  It shares no code with the GPU library: it reads the same seeded
inputs (paper_2604_11856_amd.synth) and nothing else.

The arithmetic lives in oracle.c (plain loops in double precision); this file
marshals arrays, lays out the geometry (rays, quadrature weights) and
assembles the QSS collisional-radiative system of Sec. 2.1 in plain Python
loops (solved by LAPACK's LU), citing the passage each step follows.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Species(C.Structure):
    _fields_ = [("n_species", C.c_int), ("kind", _ip), ("mass", _dp),
                ("lev_off", _i64p), ("lev_E", _dp), ("lev_g", _dp),
                ("el_off", _i64p), ("el_T", _dp), ("el_g", _dp), ("el_Jmax", _ip),
                ("vib_off", _i64p), ("vib_G", _dp), ("vib_B", _dp), ("vib_D", _dp),
                ("E_ion", _dp)]


class _Lines(C.Structure):
    _fields_ = [("n", C.c_int64), ("nu0", _dp), ("A", _dp), ("Eu_ev", _dp), ("Eu_rot", _dp),
                ("El_ev", _dp), ("El_rot", _dp), ("gu", _dp), ("gl", _dp), ("species", _i32p),
                ("lev_u", _i32p), ("lev_l", _i32p)]


class _Cont(C.Structure):
    _fields_ = [("species", C.c_int), ("ion", C.c_int), ("E_ion", C.c_double),
                ("Q_ion", C.c_double), ("sigma0", _dp), ("peach", _dp), ("z", C.c_double)]


class _Cells(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_species", C.c_int), ("T_tr", _dp), ("T_v", _dp),
                ("N", _dp), ("n_e", _dp), ("N_lev", _dp), ("lev_on", _ip)]


class _Pair(C.Structure):
    _fields_ = [("Nu", C.c_double), ("Nl", C.c_double), ("S_eta", C.c_double),
                ("B_line", C.c_double), ("gG", C.c_double), ("gL", C.c_double),
                ("gV", C.c_double), ("klo", C.c_int64), ("khi", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB: an instrumented build of oracle.c (the sanitizer test)
        path = os.environ.get("ORACLE_LIB")
        if not path:
            path = build()
        L = C.CDLL(path)
        d, i64 = C.c_double, C.c_int64
        sig = {
            "orc_c2": (d, []),
            "orc_partition_atom": (d, [i64, _dp, _dp, d]),
            "orc_partition": (d, [C.POINTER(_Species), C.c_int, d, d]),
            "orc_state_partition": (d, [C.POINTER(_Species), C.c_int, i64, d, d]),
            "orc_level_population": (d, [d, d, d, d, d, d, d]),
            "orc_doppler_hwhm": (d, [d, d, d]),
            "orc_lorentz_hwhm": (d, [d, d]),
            "orc_voigt_hwhm": (d, [d, d]),
            "orc_voigt_profile": (d, [d, d, d]),
            "orc_window": (None, [d, d, d, d, i64, _i64p, _i64p]),
            "orc_grid_offset": (d, [d, d, i64, d]),
            "orc_planck": (d, [d, d]),
            "orc_line_pair": (None, [C.POINTER(_Species), C.POINTER(_Lines), i64, d, d, d, _dp,
                                     C.c_int, d, d, _dp, d, d, i64, C.POINTER(_Pair)]),
            "orc_lorentz_line": (d, [C.POINTER(_Species), C.POINTER(_Lines), i64, d, d, d, _dp,
                                     C.c_int]),
            "orc_coeffs": (i64, [C.POINTER(_Species), C.POINTER(_Lines), C.POINTER(_Cells),
                                 d, d, i64, i64, _i64p, _dp, _dp, C.c_int]),
            "orc_coeffs_bruteforce": (None, [C.POINTER(_Species), C.POINTER(_Lines),
                                             C.POINTER(_Cells), d, d, i64, _dp, _dp]),
            "orc_march": (None, [i64, _i64p, _dp, i64, _dp, _dp, _dp, _dp]),
            "orc_linear_j_weights": (None, [d, _dp, _dp]),
            "orc_saha_volume": (d, [d]),
            "orc_peach_ff": (d, [_dp, d, d, d]),
            "orc_continuum": (None, [C.POINTER(_Species), C.POINTER(_Cells), C.c_int,
                                     C.POINTER(_Cont), d, d, i64, _i64p, _dp, _dp]),
            "orc_march_nodes": (None, [i64, _i64p, _dp, i64, _dp, _dp, _dp, _dp]),
            "orc_axi_segments": (i64, [C.c_int, C.c_int, d, d, d, d, d, i64, _i64p, _dp]),
            "orc_knife_edges": (None, [C.POINTER(_Species), C.POINTER(_Lines), C.POINTER(_Cells),
                                       d, d, i64, d, i64, _i64p, _i64p, _i64p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


# ---------------------------------------------------------------------------
# marshalling of the seeded inputs
# ---------------------------------------------------------------------------

class SpeciesTable:
    """Flattened level tables of a species list (keeps the arrays alive)."""

    def __init__(self, species, E_ion=None):
        """E_ion: per-species ionization energies (cm^-1) that switch atomic
        lines to the full Lorentz width, or None (uniform Stark law)."""
        S = len(species)
        self.E_ion = None if E_ion is None else np.ascontiguousarray(E_ion, np.float64)
        self.kind = np.array([s.kind for s in species], np.int32)
        self.mass = np.array([s.mass for s in species], np.float64)
        lev_E, lev_g, lev_off = [], [], [0]
        el_T, el_g, el_J, el_off = [], [], [], [0]
        vib_G, vib_B, vib_D, vib_off = [], [], [], [0]
        for s in species:
            lev_E.append(np.asarray(s.level_E, np.float64))
            lev_g.append(np.asarray(s.level_g, np.float64))
            lev_off.append(lev_off[-1] + len(s.level_E))
            pos = 0
            for e in range(len(s.el_T)):
                nv = int(s.el_nv[e])
                el_T.append(s.el_T[e]); el_g.append(s.el_g[e]); el_J.append(int(s.el_Jmax[e]))
                vib_G.append(s.vib_G[pos:pos + nv]); vib_B.append(s.vib_B[pos:pos + nv])
                vib_D.append(s.vib_D[pos:pos + nv])
                vib_off.append(vib_off[-1] + nv)
                pos += nv
            el_off.append(el_off[-1] + len(s.el_T))
        cat = lambda xs: np.ascontiguousarray(np.concatenate(xs) if xs else np.zeros(1), np.float64)
        self.lev_E, self.lev_g = cat(lev_E + [np.zeros(1)]), cat(lev_g + [np.zeros(1)])
        self.lev_off = np.array(lev_off, np.int64)
        self.el_T = np.array(el_T + [0.0], np.float64)
        self.el_g = np.array(el_g + [0.0], np.float64)
        self.el_J = np.array(el_J + [0], np.int32)
        self.el_off = np.array(el_off, np.int64)
        self.vib_G = cat(vib_G + [np.zeros(1)])
        self.vib_B = cat(vib_B + [np.zeros(1)])
        self.vib_D = cat(vib_D + [np.zeros(1)])
        self.vib_off = np.array(vib_off, np.int64)
        self.s = _Species(S, _p(self.kind, _ip), _p(self.mass), _p(self.lev_off, _i64p),
                          _p(self.lev_E), _p(self.lev_g), _p(self.el_off, _i64p), _p(self.el_T),
                          _p(self.el_g), _p(self.el_J, _ip), _p(self.vib_off, _i64p),
                          _p(self.vib_G), _p(self.vib_B), _p(self.vib_D),
                          None if self.E_ion is None else _p(self.E_ion))


class LineTable:
    def __init__(self, lines, levels=None):
        """levels: None, or [n_lines, 2] (upper, lower) level indices (-1: none)."""
        if lines.n > 1 and np.any(np.diff(lines.nu0) < 0):
            raise ValueError("oracle expects lines sorted by nu0")
        self.a = {f: np.ascontiguousarray(getattr(lines, f), np.float64)
                  for f in ("nu0", "A", "Eu_ev", "Eu_rot", "El_ev", "El_rot", "gu", "gl")}
        self.sp = np.ascontiguousarray(lines.species, np.int32)
        self.lev = None
        if levels is not None:
            lev = np.asarray(levels, np.int32).reshape(lines.n, 2)
            self.lev = (np.ascontiguousarray(lev[:, 0]), np.ascontiguousarray(lev[:, 1]))
        a = self.a
        self.s = _Lines(lines.n, _p(a["nu0"]), _p(a["A"]), _p(a["Eu_ev"]), _p(a["Eu_rot"]),
                        _p(a["El_ev"]), _p(a["El_rot"]), _p(a["gu"]), _p(a["gl"]),
                        _p(self.sp, _i32p),
                        None if self.lev is None else _p(self.lev[0], _i32p),
                        None if self.lev is None else _p(self.lev[1], _i32p))


class CellTable:
    def __init__(self, cells, levels=None):
        """levels: None, or (N_lev [n_cells, total levels], lev_on [n_species])."""
        self.T_tr = np.ascontiguousarray(cells.T_tr, np.float64)
        self.T_v = np.ascontiguousarray(cells.T_v, np.float64)
        self.N = np.ascontiguousarray(cells.N, np.float64)
        self.n_e = np.ascontiguousarray(cells.n_e, np.float64)
        self.N_lev = self.lev_on = None
        if levels is not None:
            self.N_lev = np.ascontiguousarray(levels[0], np.float64)
            self.lev_on = np.ascontiguousarray(levels[1], np.int32)
        self.s = _Cells(self.T_tr.shape[0], self.N.shape[1], _p(self.T_tr), _p(self.T_v),
                        _p(self.N), _p(self.n_e),
                        None if self.N_lev is None else _p(self.N_lev),
                        None if self.lev_on is None else _p(self.lev_on, _ip))


# ---------------------------------------------------------------------------
# scalar functions (Sec. 2.1, 2.2.1)
# ---------------------------------------------------------------------------

def c2() -> float:
    return lib().orc_c2()


def partition(species, s: int, Tv: float, Ttr: float) -> float:
    t = SpeciesTable(species)
    return lib().orc_partition(C.byref(t.s), s, Tv, Ttr)


def level_population(N, Q, g, E_ev, E_rot, Tv, Ttr) -> float:
    return lib().orc_level_population(N, Q, g, E_ev, E_rot, Tv, Ttr)


def doppler_hwhm(nu0, Ttr, M) -> float:
    return lib().orc_doppler_hwhm(nu0, Ttr, M)


def lorentz_hwhm(ne, Tv) -> float:
    return lib().orc_lorentz_hwhm(ne, Tv)


def voigt_hwhm(gL, gG) -> float:
    return lib().orc_voigt_hwhm(gL, gG)


def voigt_profile(delta, gV, gL):
    f = lib().orc_voigt_profile
    d = np.atleast_1d(np.asarray(delta, np.float64))
    return np.array([f(float(x), gV, gL) for x in d]) if d.size > 1 else f(float(d[0]), gV, gL)


def window(nu0, gV, nu_min, h, n_points) -> Tuple[int, int]:
    lo, hi = C.c_int64(), C.c_int64()
    lib().orc_window(nu0, gV, nu_min, h, n_points, C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def grid_offset(nu_min, h, k, nu0) -> float:
    return lib().orc_grid_offset(nu_min, h, int(k), nu0)


def planck(nu, T) -> float:
    return lib().orc_planck(nu, T)


def line_pair(species, lines, i, Ttr, Tv, ne, N_s, Q_s, grid, N_cell=None, E_ion=None,
              line_levels=None, N_lev_s=None):
    """Per-(cell, line) quantities: populations, S_eta, B_line, widths, window.
    N_cell (all species densities of the cell) and E_ion matter only for the
    full Lorentz width; line_levels ([n_lines, 2]) with N_lev_s (the level
    populations of the line's species in this cell) replace the Boltzmann
    populations of a line that has levels."""
    st, lt = SpeciesTable(species, E_ion), LineTable(lines, line_levels)
    p = _Pair()
    h = grid_step(grid)
    Nc = np.ascontiguousarray(np.zeros(len(species)) if N_cell is None else N_cell, np.float64)
    Nl = None if N_lev_s is None else np.ascontiguousarray(N_lev_s, np.float64)
    lib().orc_line_pair(C.byref(st.s), C.byref(lt.s), int(i), Ttr, Tv, ne, _p(Nc), len(species),
                        N_s, Q_s, None if Nl is None else _p(Nl), grid.nu_min, h, grid.n_points,
                        C.byref(p))
    return {f: getattr(p, f) for f, _ in _Pair._fields_}


def grid_step(grid) -> float:
    return (grid.nu_max - grid.nu_min) / (grid.n_points - 1)


# ---------------------------------------------------------------------------
# Sec. 2.1 collisional-radiative model, QSS form
# ---------------------------------------------------------------------------

N_AVOGADRO = 6.02214076e23   # mol^-1 (exact SI value)
H_CGS = 6.62607015e-27        # erg s
KB_CGS = 1.380649e-16         # erg / K


def arrhenius(C_a: float, n_a: float, E_a: float, T: float) -> float:
    """Sec. 2.1 rate formula: k = C_a T^n_a exp(-E_a / T), E_a in K."""
    return C_a * T ** n_a * math.exp(-E_a / T)


def rate_temperature(a: float, T_tr: float, T_v: float) -> float:
    """Characteristic temperature T_tr^a T_v^(1-a) of a rate."""
    return T_tr ** a * T_v ** (1.0 - a)


def state_partition(E: float, g: float, T: float) -> float:
    """Partition function of one atomic state, g e^{-c2 E / T} (energy zero
    at the atom's ground state)."""
    return g * math.exp(-c2() * E / T)


M_PROTON_G = 1.0 / N_AVOGADRO   # g per (g/mol)
KIND_ATOM = 1                   # species kind of an atom (2: diatomic molecule)


def _cr_states(rec, species):
    """State energies (level energies of an atom, electronic terms of a
    molecule) and a partition-function callable q(i, T_v, T_tr) of one state
    with the species' own energy zero."""
    sp = species[rec.species]
    if sp.kind == KIND_ATOM:
        E, g = np.asarray(sp.level_E, np.float64), np.asarray(sp.level_g, np.float64)
        return E, lambda i, Tv, Ttr: state_partition(E[i], g[i], Tv)
    table = SpeciesTable(species)
    keep = table   # keeps the arrays alive for the C calls
    return (np.asarray(sp.el_T, np.float64),
            lambda i, Tv, Ttr: lib().orc_state_partition(C.byref(keep.s), rec.species, int(i),
                                                         float(Tv), float(Ttr)))


def cr_system(rec, species, T_tr: float, T_v: float, N_cell, n_e: float, collider_w):
    """The QSS system R n = b of Sec. 2.1 for one atom or molecule (CR record
    rec) in one cell, n = populations of its states 0..l-1 (the atom's table
    levels or the molecule's electronic states; state 0 the ground state,
    l = rec.n_model).

    Row 0 is the closure: the populations of all levels add up to the atom's
    density, the levels p >= l standing in Boltzmann ratio Q_p/Q_(l-1) (at
    T_v) with level l-1.  Row i >= 1 is the QSS balance of level i: R[i, i]
    holds minus every loss rate of i (heavy-particle and electron impact
    transitions to every other level, spontaneous emission to lower levels
    with escape factor 0 above nu_cut and 1 below, electron impact
    ionization, charge exchange with the partner ion), R[i, j] the rate of
    every process taking level j to level i, and b[i] minus the sources from
    outside the atom (three-body recombination of the ion, charge exchange
    of the ion with the partner atom).  Two-body rates are the Arrhenius
    coefficient over Avogadro's number times the collider density (heavy
    colliders: sum_s collider_w[s] N_s); reverse rates follow the paper's
    detailed-balance relation evaluated at the backward temperature, with
    the state partition functions (g e^{-c2 E/T} for an atomic level, g_e
    e^{-c2 T_e/T} Q_vr(T) for a molecular electronic state, all modes at the
    rate's temperature), the ion's Q_ion e^{-c2 E_ion/T} and the free
    electron's 2 (2 pi m_e k T / h^2)^{3/2}.

    A molecule's state i also dissociates into X + Y by heavy-particle and
    electron impact (loss k_f N_M / N_A, k_f n_e / N_A), and X + Y recombine
    into it (source k_b N_X N_Y N_M / N_A, k_b N_X N_Y n_e / N_A) with the
    detailed-balance rate k_b = [k_f Q_i / (Q_X Q_Y)]_{T_b} (h^2 / (2 pi mu k
    T_b))^{3/2} e^{c2 E_diss / T_b}: the translational partition function of
    the pair (reduced mass mu) and the energy of X + Y above the molecule's
    energy zero.  The closure's Boltzmann tail of a molecule takes the
    state partition functions at (T_v, T_tr)."""
    sp = species[rec.species]
    E, q2 = _cr_states(rec, species)
    Lm, Ls = int(rec.n_model), E.size
    NA = N_AVOGADRO
    N_cell = np.asarray(N_cell, np.float64)
    N_M = sum(float(collider_w[s]) * float(N_cell[s]) for s in range(N_cell.size))
    N_ion = float(N_cell[rec.ion]) if rec.ion >= 0 else 0.0
    Tm = [(rate_temperature(rec.texp[2 * m], T_tr, T_v),
           rate_temperature(rec.texp[2 * m + 1], T_tr, T_v)) for m in range(len(rec.texp) // 2)]
    Q = lambda i, T: q2(i, T, T)

    def k_exc(table, m, i, j):
        """rate coefficient of the transition i -> j of mechanism m (0 HPIE, 1 EIE)"""
        T_f, T_b = Tm[m]
        if j > i:
            return arrhenius(*table[i, j], T_f)
        return arrhenius(*table[j, i], T_b) * Q(j, T_b) / Q(i, T_b)

    def escape(hi, lo):
        return 0.0 if E[hi] - E[lo] > rec.nu_cut else 1.0

    diss = getattr(rec, "diss_x", -1) >= 0
    if diss:
        def product_q(p, Qc, T):
            ps = species[p]
            if ps.kind == KIND_ATOM:
                return sum(state_partition(ps.level_E[k], ps.level_g[k], T) for k in range(len(ps.level_E)))
            return Qc
        mX, mY = species[rec.diss_x].mass, species[rec.diss_y].mass
        mu = mX * mY / (mX + mY) * M_PROTON_G
        N_X, N_Y = float(N_cell[rec.diss_x]), float(N_cell[rec.diss_y])

    R = np.zeros((Lm, Lm))
    b = np.zeros(Lm)
    R[0, :] = 1.0
    R[0, Lm - 1] = 1.0 + sum(q2(p, T_v, T_tr) / q2(Lm - 1, T_v, T_tr) for p in range(Lm, Ls))
    b[0] = float(N_cell[rec.species])
    for i in range(1, Lm):
        loss = 0.0
        for m in range(Lm):
            if m != i:
                loss += k_exc(rec.hpie, 0, i, m) / NA * N_M + k_exc(rec.eie, 1, i, m) / NA * n_e
        for m in range(i):
            loss += escape(i, m) * rec.A[i, m]
        if not diss:
            loss += arrhenius(*rec.eii[i], Tm[2][0]) / NA * n_e
            if rec.partner >= 0:
                loss += arrhenius(*rec.ce[i], Tm[3][0]) / NA * float(N_cell[rec.partner_ion])
        else:
            loss += arrhenius(*rec.hpid[i], Tm[4][0]) / NA * N_M + arrhenius(*rec.eid[i], Tm[5][0]) / NA * n_e
        R[i, i] = -loss
        for j in range(Lm):
            if j == i:
                continue
            gain = k_exc(rec.hpie, 0, j, i) / NA * N_M + k_exc(rec.eie, 1, j, i) / NA * n_e
            if j > i:
                gain += escape(j, i) * rec.A[j, i]
            R[i, j] = gain
        if diss:
            src = 0.0
            for m, coll in ((4, N_M), (5, n_e)):
                T_b = Tm[m][1]
                table = rec.hpid if m == 4 else rec.eid
                Vmu = (H_CGS * H_CGS / (2.0 * math.pi * mu * KB_CGS * T_b)) ** 1.5
                k_b = (arrhenius(*table[i], T_b) * Q(i, T_b)
                       / (product_q(rec.diss_x, rec.Q_x, T_b) * product_q(rec.diss_y, rec.Q_y, T_b))
                       * Vmu * math.exp(c2() * rec.E_diss / T_b))
                src += k_b / NA * N_X * N_Y * coll
            b[i] = -src
            continue
        T_b = Tm[2][1]
        k_rec = (arrhenius(*rec.eii[i], T_b) * Q(i, T_b)
                 / (rec.Q_ion * math.exp(-c2() * rec.E_ion / T_b) * (2.0 / saha_volume(T_b))))
        src = k_rec / NA * N_ion * n_e * n_e
        if rec.partner >= 0:
            T_b = Tm[3][1]
            pb = species[rec.partner]
            Q_B = sum(state_partition(pb.level_E[k], pb.level_g[k], T_b) for k in range(len(pb.level_E)))
            Q_Bp = rec.partner_Q_ion * math.exp(-c2() * rec.partner_E_ion / T_b)
            Q_Ap = rec.Q_ion * math.exp(-c2() * rec.E_ion / T_b)
            k_b = arrhenius(*rec.ce[i], T_b) * Q(i, T_b) * Q_Bp / (Q_Ap * Q_B)
            src += k_b / NA * N_ion * float(N_cell[rec.partner])
        b[i] = -src
    return R, b


def cr_level_populations(rec, species, T_tr, T_v, N_cell, n_e, collider_w):
    """Populations of every level of the atom's table in one cell: levels
    0..l-1 from the LU solution of R n = b (LAPACK's partially pivoted LU),
    the levels above from their Boltzmann ratio to level l-1 at T_v; all zero
    in a cell without the atom."""
    E, q2 = _cr_states(rec, species)
    if not float(N_cell[rec.species]) > 0.0:
        return np.zeros(E.size)   # none of the species in the cell: no state populations
    R, b = cr_system(rec, species, T_tr, T_v, N_cell, n_e, collider_w)
    n = np.linalg.solve(R, b)
    Lm = int(rec.n_model)
    out = np.empty(E.size)
    out[:Lm] = n
    q_top = q2(Lm - 1, T_v, T_tr)
    for p in range(Lm, E.size):
        out[p] = n[Lm - 1] * q2(p, T_v, T_tr) / q_top
    return out


def cr_populations(cr, species, cells):
    """Per CR record, the state populations [n_cells, n_states] of its species."""
    out = []
    for rec in cr.species:
        out.append(np.stack([cr_level_populations(rec, species, float(cells.T_tr[c]),
                                                  float(cells.T_v[c]), cells.N[c],
                                                  float(cells.n_e[c]), cr.collider_w)
                             for c in range(cells.n)]) if cells.n else
                   np.zeros((0, _cr_states(rec, species)[0].size)))
    return out


def cr_level_table(cr, species, cells):
    """(N_lev [n_cells, atom levels of all species + molecular electronic
    states of all species], lev_on [n_species]) for the coefficient
    routines, or None without a CR model."""
    if cr is None:
        return None
    off = np.concatenate([[0], np.cumsum([len(s.level_E) for s in species])])
    eoff = off[-1] + np.concatenate([[0], np.cumsum([len(s.el_T) for s in species])])
    N_lev = np.zeros((cells.n, int(eoff[-1])))
    lev_on = np.zeros(len(species), np.int32)
    for rec, pop in zip(cr.species, cr_populations(cr, species, cells)):
        s = rec.species
        if species[s].kind == KIND_ATOM:
            N_lev[:, off[s]:off[s + 1]] = pop
        else:
            N_lev[:, eoff[s]:eoff[s + 1]] = pop
        lev_on[s] = 1
    return N_lev, lev_on


# ---------------------------------------------------------------------------
# eta / kappa (Sec. 2.2.1) for all cells at grid indices ks
# ---------------------------------------------------------------------------

def coeffs(species, lines, cells, grid, ks: Optional[np.ndarray] = None, threads: int = 0,
           E_ion=None, cr=None, line_levels=None):
    """Returns (eta [n_cells, n_k], kappa [n_cells, n_k], n_terms).  With a
    CR model and line_levels, the lines with levels take their populations
    from the QSS-CR solution."""
    if ks is None:
        ks = np.arange(grid.n_points, dtype=np.int64)
    ks = np.ascontiguousarray(ks, np.int64)
    st = SpeciesTable(species, E_ion)
    lt = LineTable(lines, line_levels if cr is not None else None)
    ct = CellTable(cells, cr_level_table(cr, species, cells))
    eta = np.zeros((cells.n, ks.size))
    kap = np.zeros((cells.n, ks.size))
    n = lib().orc_coeffs(C.byref(st.s), C.byref(lt.s), C.byref(ct.s), grid.nu_min, grid.nu_max,
                         grid.n_points, ks.size, _p(ks, _i64p), _p(eta), _p(kap), int(threads))
    return eta, kap, n


def knife_edges(species, lines, cells, grid, tol: float = 1e-9, near=None, E_ion=None,
                reach: float = 1000.0):
    """(cell, k) grid points next to a window bound that lies within tol grid
    steps of an integer grid index: a last-bit difference in the Voigt
    width may move such a bound by one point.  near: optional sorted grid
    indices; only lines within `reach` cm^-1 of one of them are scanned (the
    caller's bound on 100 Voigt HWHM)."""
    if near is not None and lines.n:
        h = grid_step(grid)
        nu = grid.nu_min + np.asarray(near, np.float64) * h
        lo = np.searchsorted(lines.nu0, nu - reach)
        hi = np.searchsorted(lines.nu0, nu + reach)
        keep = np.zeros(lines.n + 1, np.int64)
        np.add.at(keep, lo, 1)
        np.add.at(keep, hi, -1)
        lines = lines.subset(np.nonzero(np.cumsum(keep)[:-1] > 0)[0])
    st, lt, ct = SpeciesTable(species, E_ion), LineTable(lines), CellTable(cells)
    cap = 4096
    cc = np.zeros(cells.n * cap, np.int64)
    kk = np.zeros(cells.n * cap, np.int64)
    cnt = np.zeros(cells.n, np.int64)
    lib().orc_knife_edges(C.byref(st.s), C.byref(lt.s), C.byref(ct.s), grid.nu_min, grid.nu_max,
                          grid.n_points, tol, cap, _p(cc, _i64p), _p(kk, _i64p), _p(cnt, _i64p))
    sel = np.concatenate([np.arange(c * cap, c * cap + cnt[c]) for c in range(cells.n)]) \
        if cells.n else np.zeros(0, np.int64)
    return cc[sel].copy(), kk[sel].copy()


def saha_volume(T: float) -> float:
    return lib().orc_saha_volume(float(T))


def peach_ff(c, z: float, s: float, T: float) -> float:
    c = np.ascontiguousarray(c, np.float64)
    return lib().orc_peach_ff(_p(c), float(z), float(s), float(T))


def continuum(species, cells, grid, cont, ks: Optional[np.ndarray] = None, cr=None):
    """Atomic continuum (Sec. 2.2.1 bound-free and free-free) eta and kappa
    [n_cells, n_k] at grid points ks (default: all); with a CR model the
    bound-free absorption of its atoms uses the QSS-CR level populations."""
    if ks is None:
        ks = np.arange(grid.n_points, dtype=np.int64)
    ks = np.ascontiguousarray(ks, np.int64)
    st, ct = SpeciesTable(species), CellTable(cells, cr_level_table(cr, species, cells))
    keep = [(np.ascontiguousarray(r.sigma0, np.float64), np.ascontiguousarray(r.peach, np.float64))
            for r in cont]
    arr = (_Cont * max(1, len(cont)))()
    for j, (r, (s0, pc)) in enumerate(zip(cont, keep)):
        arr[j] = _Cont(int(r.species), int(r.ion), float(r.E_ion), float(r.Q_ion), _p(s0), _p(pc),
                       float(r.z))
    eta = np.zeros((cells.n, ks.size))
    kap = np.zeros((cells.n, ks.size))
    lib().orc_continuum(C.byref(st.s), C.byref(ct.s), len(cont), arr, float(grid.nu_min),
                        grid_step(grid), ks.size, _p(ks, _i64p), _p(eta), _p(kap))
    return eta, kap


def coeffs_bruteforce(species, lines, cells, grid, E_ion=None, cr=None, line_levels=None):
    st = SpeciesTable(species, E_ion)
    lt = LineTable(lines, line_levels if cr is not None else None)
    ct = CellTable(cells, cr_level_table(cr, species, cells))
    eta = np.zeros((cells.n, grid.n_points))
    kap = np.zeros((cells.n, grid.n_points))
    lib().orc_coeffs_bruteforce(C.byref(st.s), C.byref(lt.s), C.byref(ct.s), grid.nu_min,
                                grid.nu_max, grid.n_points, _p(eta), _p(kap))
    return eta, kap


# ---------------------------------------------------------------------------
# rays and quadrature (Sec. 2.2.3)
# ---------------------------------------------------------------------------

def gauss_legendre_01(n: int):
    """Gauss-Legendre nodes and weights on [0, 1] (weights sum to 1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def slab_rays(geom):
    """Rays of a 1-D slab seen from the wall: the wall-normal ray, then one
    ray per Gauss-Legendre node mu_i (path length dx / mu_i per cell).
    Returns (list of (cells, ds), mu, W) with cells ordered far -> wall."""
    n = geom.dx.shape[0]
    cells = np.arange(n, dtype=np.int64)
    rays = [(cells, np.asarray(geom.dx, np.float64).copy())]
    mu, W = (np.zeros(0), np.zeros(0))
    if geom.n_mu > 0:
        mu, W = gauss_legendre_01(geom.n_mu)
        for m in mu:
            rays.append((cells, np.asarray(geom.dx, np.float64) / m))
    return rays, mu, W


def axi_ray(geom, rw: float, mu: float, phi: float):
    cap = geom.nx + 2 * geom.nr + 8
    cell = np.zeros(cap, np.int64)
    ds = np.zeros(cap)
    n = lib().orc_axi_segments(geom.nx, geom.nr, geom.Lx, geom.R, rw, mu, phi, cap,
                               _p(cell, _i64p), _p(ds))
    if n < 0:
        raise RuntimeError("segment capacity exceeded")
    return cell[:n].copy(), ds[:n].copy()


def axi_rays(geom, wall_index: int):
    """Rays of one wall point: mu_i Gauss-Legendre on [0, 1] (outer),
    phi_j = (j + 1/2) 2 pi / n_phi (inner).  Returns (rays, weights) with
    weight W_i mu_i 2 pi / n_phi for the flux integral of I cos(theta) dOmega."""
    mu, W = gauss_legendre_01(geom.n_mu)
    rw = float(geom.wall_r[wall_index])
    rays, wts = [], []
    for i in range(geom.n_mu):
        for j in range(geom.n_phi):
            phi = (j + 0.5) * 2.0 * np.pi / geom.n_phi
            rays.append(axi_ray(geom, rw, mu[i], phi))
            wts.append(W[i] * mu[i] * 2.0 * np.pi / geom.n_phi)
    return rays, np.array(wts)


def march(cells_idx, ds, eta, kappa, I_far=None):
    """I at the target for every column of eta/kappa [n_cells, n_k]."""
    eta = np.ascontiguousarray(eta, np.float64)
    kappa = np.ascontiguousarray(kappa, np.float64)
    cells_idx = np.ascontiguousarray(cells_idx, np.int64)
    ds = np.ascontiguousarray(ds, np.float64)
    nk = eta.shape[1]
    out = np.zeros(nk)
    far = None if I_far is None else _p(np.ascontiguousarray(I_far, np.float64))
    lib().orc_march(cells_idx.size, _p(cells_idx, _i64p), _p(ds), nk, _p(eta), _p(kappa),
                    far, _p(out))
    return out


def linear_j_weights(t: float):
    """(W_far, W_near) of the linear-j segment (Sec. 2.2.3): the segment adds
    ds (W_far j_far + W_near j_near) to the attenuated intensity."""
    a, b = C.c_double(), C.c_double()
    lib().orc_linear_j_weights(float(t), C.byref(a), C.byref(b))
    return a.value, b.value


def midpoint_nodes(cells_idx, ds):
    """LOS nodes of a ray given as cell segments far -> target, for the
    linear-j march: the far end, the midpoint of every segment, the target.
    A node takes the state of the cell that contains it; spacings are
    ds_0/2, (ds_m + ds_m+1)/2, ..., ds_M-1/2."""
    cells_idx = np.asarray(cells_idx, np.int64)
    ds = np.asarray(ds, np.float64)
    node_cell = np.concatenate([cells_idx[:1], cells_idx, cells_idx[-1:]])
    dsn = np.concatenate([ds[:1] * 0.5, 0.5 * (ds[:-1] + ds[1:]), ds[-1:] * 0.5])
    return node_cell, dsn


def march_nodes(node_cell, dsn, eta, kappa, I_far=None):
    """Linear-j march over explicit nodes (Sec. 2.2.3): I at the last node for
    every column of eta/kappa [n_cells, n_k]."""
    eta = np.ascontiguousarray(eta, np.float64)
    kappa = np.ascontiguousarray(kappa, np.float64)
    node_cell = np.ascontiguousarray(node_cell, np.int64)
    dsn = np.ascontiguousarray(dsn, np.float64)
    nk = eta.shape[1]
    out = np.zeros(nk)
    far = None if I_far is None else _p(np.ascontiguousarray(I_far, np.float64))
    lib().orc_march_nodes(node_cell.size, _p(node_cell, _i64p), _p(dsn), nk, _p(eta), _p(kappa),
                          far, _p(out))
    return out


def march_linear(cells_idx, ds, eta, kappa, I_far=None):
    """Linear-j march of a cell-segment ray through its midpoint nodes."""
    nc, dsn = midpoint_nodes(cells_idx, ds)
    return march_nodes(nc, dsn, eta, kappa, I_far)


def planck_spectrum(grid, ks, T: float):
    """Blackbody intensity B(nu_k, T) (W cm^-2 sr^-1 per cm^-1) at grid points ks."""
    h = grid_step(grid)
    return np.array([lib().orc_planck(grid.nu_min + float(k) * h, float(T)) for k in ks])


def fibonacci_directions(n: int):
    """Fibonacci-sphere LOS directions (Sec. 2.2.3): for i = 1..n,
    w = 1 - 2 (i-1)/(n-1), r = sqrt(1 - w^2), a = (i-1)(sqrt 5 - 1) pi and the
    unit vector (r cos a, w, r sin a).  Returned in the wall frame: the polar
    component w along the wall normal (first coordinate), then (r cos a,
    r sin a)."""
    i = np.arange(1, n + 1, dtype=np.float64)
    w = 1.0 - 2.0 * (i - 1.0) / (n - 1.0)
    r = np.sqrt(np.maximum(0.0, 1.0 - w * w))
    a = (i - 1.0) * (np.sqrt(5.0) - 1.0) * np.pi
    return np.stack([w, r * np.cos(a), r * np.sin(a)], axis=1)


def fibonacci_quadrature(n_los: int, n_polar: int, n_azim: int):
    """Flux quadrature over the Fibonacci LOS seen from a wall (Sec. 2.2.3
    heat-flux sum): the LOS results are carried to the nodes of a uniform
    grid in polar angle phi_p = p (pi/2)/n_polar (from the wall normal) and
    azimuth theta_t = t 2 pi/n_azim by taking the nearest LOS direction, and
    every grid cell contributes the mean of its four corners times
    int sin(phi) cos(phi) dphi over the cell = (sin^2 phi_p+1 - sin^2 phi_p)/2,
    times the azimuth step.  Because the rule is linear in the LOS results it
    is a weight per LOS.  Returns (directions [m, 3] with positive normal
    component, weights [m])."""
    d = fibonacci_directions(n_los)
    keep = np.nonzero(d[:, 0] > 0.0)[0]
    d = d[keep]
    w = np.zeros(len(keep))
    phi = np.arange(n_polar + 1) * (0.5 * np.pi / n_polar)
    th = np.arange(n_azim + 1) * (2.0 * np.pi / n_azim)
    near = np.zeros((n_polar + 1, n_azim + 1), np.int64)
    for p in range(n_polar + 1):
        for t in range(n_azim + 1):
            nx_, ny_, nz_ = np.cos(phi[p]), np.sin(phi[p]) * np.cos(th[t]), np.sin(phi[p]) * np.sin(th[t])
            dots = d[:, 0] * nx_ + d[:, 1] * ny_ + d[:, 2] * nz_
            near[p, t] = int(np.argmax(dots))
    for p in range(n_polar):
        wp = 0.5 * (np.sin(phi[p + 1]) ** 2 - np.sin(phi[p]) ** 2)
        for t in range(n_azim):
            wc = 0.25 * wp * (th[t + 1] - th[t])
            for pp, tt in ((p, t), (p + 1, t), (p, t + 1), (p + 1, t + 1)):
                w[near[pp, tt]] += wc
    return d, w


def axi_rays_fibonacci(geom, wall_index: int, n_los: int, n_polar: int, n_azim: int):
    """Rays of one wall point along the Fibonacci LOS with a positive normal
    component, and their flux weights."""
    d, w = fibonacci_quadrature(n_los, n_polar, n_azim)
    rw = float(geom.wall_r[wall_index])
    rays = [axi_ray(geom, rw, float(v[0]), float(np.arctan2(v[2], v[1]))) for v in d]
    return rays, w


def trapezoid_weights(grid, ks=None):
    """Spectral trapezoid weights by global grid index: h/2 at both ends, h inside."""
    h = grid_step(grid)
    ks = np.arange(grid.n_points) if ks is None else np.asarray(ks)
    w = np.full(ks.shape, h)
    w[(ks == 0) | (ks == grid.n_points - 1)] = 0.5 * h
    return w


def solve_slab(wl, ks=None, threads: int = 0):
    """Whole path for a slab workload: eta/kappa at ks, I per ray, spectral
    integral per ray (trapezoid over ks; exact when ks is the full grid) and
    the tangent-slab flux q = 2 pi sum_i W_i mu_i I_int(mu_i)."""
    eta, kap, n_terms = coeffs(wl.species, wl.lines, wl.cells, wl.grid, ks, threads,
                               getattr(wl, "lorentz_E_ion", None), getattr(wl, "cr", None),
                               getattr(wl, "line_levels", None))
    rays, mu, W = slab_rays(wl.geometry)
    I = np.stack([march(c, d, eta, kap) for c, d in rays])
    w = trapezoid_weights(wl.grid, ks)
    I_int = I @ w
    q = 2.0 * np.pi * float(np.sum(W * mu * I_int[1:])) if len(mu) else None
    return dict(eta=eta, kappa=kap, I=I, I_int=I_int, q=q, n_terms=n_terms)


def solve_axi(wl, wall_indices: Sequence[int], ks=None, threads: int = 0):
    """Axisymmetric workload at the given wall points: per-point spectral
    flux q_k = sum_rays w_ray I_ray(k) and, over ks, q = sum_k w_k q_k."""
    eta, kap, n_terms = coeffs(wl.species, wl.lines, wl.cells, wl.grid, ks, threads,
                               getattr(wl, "lorentz_E_ion", None), getattr(wl, "cr", None),
                               getattr(wl, "line_levels", None))
    w = trapezoid_weights(wl.grid, ks)
    out = []
    for wi in wall_indices:
        rays, wts = axi_rays(wl.geometry, wi)
        qk = np.zeros(eta.shape[1])
        I_int = []
        for (c, d), wt in zip(rays, wts):
            I = march(c, d, eta, kap)
            qk += wt * I
            I_int.append(float(I @ w))
        out.append(dict(q_k=qk, q=float(qk @ w), I_int=np.array(I_int)))
    return dict(eta=eta, kappa=kap, walls=out, n_terms=n_terms)
