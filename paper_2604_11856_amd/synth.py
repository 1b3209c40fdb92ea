"""Seeded synthetic inputs: species tables, line lists, cell states, spectral
grids and ray geometry shaped like the workloads of the line-by-line +
ray-tracing radiation method (arXiv 2604.11856, Sec. 2.2 and Sec. 3.2).

This module draws random numbers and lays out data; it holds none of the
method's arithmetic (no populations, widths, profiles, march or quadrature).
The level energies of the synthetic rovibronic systems follow the term-value
forms of Sec. 2.2.2 (vibrational ladder, rigid-rotor J(J+1) rotation) because
those define what the synthetic line list *is*; the partition functions built
from these tables are computed elsewhere.

Both the oracle tests and the GPU path read inputs from here and nothing else
is shared between them.

Units: wavenumbers and energies in cm^-1, temperatures in K, number densities
in cm^-3, lengths in cm, masses in g/mol.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np

EV_CM = 8065.543937  # 1 eV in cm^-1 (CODATA)

# Species order used by every multi-species workload (11-species air).
AIR11 = ["N2", "O2", "NO", "N", "O", "N2+", "O2+", "NO+", "N+", "O+", "e-"]
AIR11_MASS = {"N2": 28.0, "O2": 32.0, "NO": 30.0, "N": 14.0, "O": 16.0,
              "N2+": 28.0, "O2+": 32.0, "NO+": 30.0, "N+": 14.0, "O+": 16.0,
              "e-": 5.48579909e-4}
ION_SPECIES = ["N2+", "O2+", "NO+", "N+", "O+"]

KIND_NONE, KIND_ATOM, KIND_MOLECULE = 0, 1, 2


@dataclasses.dataclass
class Species:
    """One species' level table.

    kind: KIND_ATOM (electronic levels only), KIND_MOLECULE (electronic x
    vibrational x rotational ladder) or KIND_NONE (no radiating levels).
    Atoms: level_E[n], level_g[n].
    Molecules: per electronic state e: el_T[e], el_g[e], el_nv[e] vibrational
    levels with term values vib_G and rotational constants vib_B, vib_D
    (concatenated over e, el_nv[e] entries each), J = 0..el_Jmax[e].
    """
    name: str
    kind: int
    mass: float
    level_E: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))
    level_g: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))
    el_T: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))
    el_g: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))
    el_nv: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int32))
    el_Jmax: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int32))
    vib_G: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))
    vib_B: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))
    vib_D: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))


@dataclasses.dataclass
class Lines:
    """Line list, SoA, sorted by nu0 ascending (stable)."""
    nu0: np.ndarray
    A: np.ndarray
    Eu_ev: np.ndarray
    Eu_rot: np.ndarray
    El_ev: np.ndarray
    El_rot: np.ndarray
    gu: np.ndarray
    gl: np.ndarray
    species: np.ndarray  # int32 index into the species table

    @property
    def n(self) -> int:
        return int(self.nu0.shape[0])

    def subset(self, idx) -> "Lines":
        return Lines(*(getattr(self, f.name)[idx] for f in dataclasses.fields(self)))


@dataclasses.dataclass
class Cells:
    T_tr: np.ndarray      # [n_cells]
    T_v: np.ndarray       # [n_cells]  (electron-electronic = vibrational temperature)
    N: np.ndarray         # [n_cells, n_species]
    n_e: np.ndarray       # [n_cells]

    @property
    def n(self) -> int:
        return int(self.T_tr.shape[0])


@dataclasses.dataclass
class Grid:
    nu_min: float
    nu_max: float
    n_points: int
    band_points: int

    @property
    def n_bands(self) -> int:
        return (self.n_points + self.band_points - 1) // self.band_points


@dataclasses.dataclass
class SlabGeometry:
    """1-D slab: cells ordered from the far (free) boundary to the wall."""
    dx: np.ndarray
    n_mu: int          # 0: only the wall-normal ray; else normal ray + n_mu Gauss-Legendre rays


@dataclasses.dataclass
class AxiGeometry:
    """Axisymmetric structured grid x in [0, Lx], r in [0, R], nx x nr uniform
    cells, cell index c = ix * nr + ir.  Wall is the plane x = 0, wall points at
    radii wall_r; rays leave the wall into x > 0.  Directions: n_mu
    Gauss-Legendre polar nodes x n_phi azimuths, or, when fib_los > 0, the
    Fibonacci-sphere LOS set of fib_los directions with its (fib_polar x
    fib_azim)-interval angular grid."""
    nx: int
    nr: int
    Lx: float
    R: float
    wall_r: np.ndarray
    n_mu: int
    n_phi: int
    fib_los: int = 0
    fib_polar: int = 0
    fib_azim: int = 0


@dataclasses.dataclass
class Continuum:
    """Atomic continuum data of one atom: bound-free absorption from each of
    its levels into the ground state of its singly charged ion, and free-free
    absorption of electrons in the field of that ion.
    sigma0[i]: photoionization cross section of level i at its threshold
    (E_ion - E_i), cm^2 (0: no bound-free from that level); peach: c1..c8 of
    the hydrogenic free-free fit, cm^5 (all 0: no free-free); z: ion charge."""
    species: int
    ion: int
    E_ion: float
    Q_ion: float
    sigma0: np.ndarray
    peach: np.ndarray
    z: float = 1.0


@dataclasses.dataclass
class CRSpecies:
    """Collisional-radiative data of one atom or diatomic molecule (Sec. 2.1
    CR model).  The states are the atom's table levels or the molecule's
    electronic states (energies E: level energies, electronic terms T_e);
    states 0..n_model-1 are solved for, the states above stay in Boltzmann
    ratio with state n_model-1.  Rate coefficients are Arrhenius triples
    (C in cm^3 mol^-1 s^-1 K^-n, n, E_a in K) of the forward processes:
      hpie[lo, hi], eie[lo, hi]: heavy-particle / electron impact excitation
        lo -> hi (lo < hi; other entries unused);
      A[hi, lo]: spontaneous emission hi -> lo, s^-1 (lo < hi);
    atoms only (ion < 0: the ion density is taken as 0):
      eii[i]: electron impact ionization of level i into the ion `ion`;
      ce[i]: charge exchange  atom(i) + partner_ion -> ion + partner
        (partner < 0: none);
    molecules only (diss_x < 0: none):
      hpid[i], eid[i]: heavy-particle / electron impact dissociation of
        state i into diss_x + diss_y, whose partition functions are the
        level sums of an atom, else the constants Q_x, Q_y; E_diss (cm^-1):
        energy of the separated products above the molecule's energy zero.
    Reverse rates follow from detailed balance.  texp[2m], texp[2m+1]: the
    forward and backward rates of mechanism m (HPIE, EIE, EII, CE, HPID,
    EID) are taken at T = T_tr^a T_v^(1-a) with a the entry.  Transitions
    above nu_cut (cm^-1, i.e. below 200 nm) are optically thick (no net
    radiative rate)."""
    species: int
    ion: int
    partner: int
    partner_ion: int
    n_model: int
    E_ion: float
    Q_ion: float
    partner_E_ion: float
    partner_Q_ion: float
    hpie: np.ndarray
    eie: np.ndarray
    A: np.ndarray
    eii: np.ndarray
    ce: np.ndarray
    texp: np.ndarray
    nu_cut: float = 50000.0
    diss_x: int = -1
    diss_y: int = -1
    Q_x: float = 0.0
    Q_y: float = 0.0
    E_diss: float = 0.0
    hpid: Optional[np.ndarray] = None
    eid: Optional[np.ndarray] = None


@dataclasses.dataclass
class CRModel:
    """QSS collisional-radiative populations for some atoms and molecules; collider_w[s]
    is the weight of species s among the heavy collision partners M (0 for
    electrons)."""
    species: List[CRSpecies]
    collider_w: np.ndarray


@dataclasses.dataclass
class BandSystem:
    """Molecular constants of one electronic band system (upper state u ->
    lower state l) of a diatomic radiator, the input of the rovibronic line
    generator: coupling case (0: Hund (a), 1: Hund (b) doublet), |Lambda| of
    each state, electronic terms T_e and degeneracy factors g_e (cm^-1, a
    level's degeneracy being g_e (2J + 1)), vibrational constants w_e,
    w_e x_e, w_e y_e, rotational constants B_e, alpha_e, D_e, beta_e and the
    spin-rotation constant gamma of each state (cm^-1), vibrational levels
    V = 0..nv-1 of each state, the rotational extent J_max, and per
    (V_u, V_l) band the squared rotationless transition moment Re'^2 (in
    units of e a0, row-major [nv_u][nv_l])."""
    species: int
    hund: int
    Lambda_u: int
    Lambda_l: int
    Te_u: float
    Te_l: float
    g_u: float
    g_l: float
    we_u: float
    wexe_u: float
    weye_u: float
    Be_u: float
    ae_u: float
    De_u: float
    be_u: float
    gamma_u: float
    we_l: float
    wexe_l: float
    weye_l: float
    Be_l: float
    ae_l: float
    De_l: float
    be_l: float
    gamma_l: float
    nv_u: int
    nv_l: int
    J_max: int
    Re2: np.ndarray


@dataclasses.dataclass
class Workload:
    name: str
    species: List[Species]
    lines: Lines
    cells: Cells
    grid: Grid
    geometry: object
    meta: Dict = dataclasses.field(default_factory=dict)
    continuum: Optional[List[Continuum]] = None
    # per-species ionization energies (cm^-1) giving atomic lines the full
    # Lorentz width (natural + per-line Stark + van der Waals); None: the
    # uniform Stark law for every line
    lorentz_E_ion: Optional[np.ndarray] = None
    # QSS collisional-radiative populations (None: Boltzmann for every level)
    # and, per line in list order, its (upper, lower) level in its atom's
    # level table (-1, -1: the line keeps Boltzmann populations)
    cr: Optional[CRModel] = None
    line_levels: Optional[np.ndarray] = None


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def atom_species(rng, name: str, n_levels: int = 20) -> Species:
    """Atom with a seeded level table: level 0 is the ground state (E = 0);
    the others have E ~ U(0.1, 14) eV.  Degeneracies g ~ U{2..12}."""
    E = np.empty(n_levels)
    E[0] = 0.0
    E[1:] = np.sort(rng.uniform(0.1, 14.0, n_levels - 1)) * EV_CM
    g = rng.integers(2, 13, n_levels).astype(np.float64)
    return Species(name, KIND_ATOM, AIR11_MASS.get(name, 14.0), level_E=E, level_g=g)


# Ionization energies of the ground states (cm^-1) and the ground-term
# degeneracies of the singly charged ions, used as their partition functions.
ION_ENERGY_CM = {"N": 117225.7, "O": 109837.02}
ION_Q = {"N+": 9.0, "O+": 4.0}
# Coefficients c1..c8 (cm^5) of the hydrogenic free-free fit for N and O, as
# printed in the paper's table of fitting parameters.
PEACH_FF = {"N": [0.006805, -0.00934, 0.000116, 0.508, 1.046, 5.77e-5, 1.85, 0.000343],
            "O": [0.001905, -0.005105, 8.176e-5, 0.4554, 1.0238, 5.329e-5, 1.7587, 0.003121]}


def air_continuum(species: List[Species], seed: int = 11862) -> List[Continuum]:
    """Continuum records of the radiating atoms N and O of a species list that
    also holds their ions N+ and O+ (found by name).  The photoionization cross
    sections are synthetic (the level-resolved data are not available):
    sigma0 ~ logU(1e-19, 1e-17) cm^2 per level, 0 for levels at or above the
    ionization energy."""
    rng = np.random.Generator(np.random.PCG64(seed))
    names = [sp.name for sp in species]
    out = []
    for atom in ("N", "O"):
        if atom not in names or atom + "+" not in names:
            continue
        a = names.index(atom)
        sp = species[a]
        if sp.kind != KIND_ATOM:
            continue
        s0 = 10.0 ** rng.uniform(-19.0, -17.0, sp.level_E.size)
        s0[sp.level_E >= ION_ENERGY_CM[atom]] = 0.0
        out.append(Continuum(a, names.index(atom + "+"), ION_ENERGY_CM[atom], ION_Q[atom + "+"],
                             s0, np.array(PEACH_FF[atom], np.float64), 1.0))
    return out


def air_ionization_energies(species: List[Species]) -> np.ndarray:
    """Per-species ionization energies for the full Lorentz width: the textbook
    values for the atoms N and O, 0 for every other species."""
    return np.array([ION_ENERGY_CM.get(sp.name, 0.0) if sp.kind == KIND_ATOM else 0.0
                     for sp in species], np.float64)


AVOGADRO = 6.02214076e23
C2_CM_K = 6.62607015e-27 * 2.99792458e10 / 1.380649e-16   # second radiation constant


def _arrhenius_triples(rng, n, k_lo, k_hi, n_lo, n_hi, Ea):
    """n Arrhenius triples whose rate at 1e4 K is k ~ logU(k_lo, k_hi) cm^3/s,
    with n ~ U(n_lo, n_hi) and the given activation temperatures."""
    k = _log_uniform(rng, k_lo, k_hi, n)
    ex = rng.uniform(n_lo, n_hi, n)
    return np.stack([k * AVOGADRO * 1e4 ** (-ex), ex, np.asarray(Ea, np.float64)], axis=-1)


# Dissociation energies D0 (cm^-1, from v = 0 of the ground state) of the
# synthetic diatomics: the textbook values of N2, O2, NO and N2+.
DISS_D0_CM = {"N2": 78714.0, "O2": 41260.0, "NO": 52400.0, "N2+": 70300.0}
DISS_PRODUCTS = {"N2": ("N", "N"), "O2": ("O", "O"), "NO": ("N", "O"), "N2+": ("N", "N+")}


def air_cr(species: List[Species], n_model: int = 18, seed: int = 11863,
           molecules: bool = True) -> CRModel:
    """Synthetic QSS-CR data for the atoms N and O of a species list (the
    paper's rate mechanism is not available); an atom whose ion is not in the
    list gets ion = -1 (no recombination source) and no charge exchange.  Per
    level pair lo < hi of the first n_model levels, with dE = E_hi - E_lo:
      EIE  k(1e4 K) ~ logU(1e-10, 1e-7) cm^3/s, n ~ U(-0.5, 0.5), E_a = c2 dE;
      HPIE k(1e4 K) ~ logU(1e-14, 1e-11) cm^3/s, n ~ U(0, 1),  E_a = c2 dE;
      A ~ logU(1e4, 1e8) s^-1 for half of the pairs (seeded), else 0;
    per level i: EII k ~ logU(1e-10, 1e-8), n ~ U(0, 0.5),
    E_a = c2 max(E_ion - E_i, 0); CE with the other atom (N(i) + O+ <-> N+ + O
    and O(i) + N+ <-> O+ + N) k ~ logU(1e-12, 1e-10), n ~ U(0, 0.5),
    E_a = c2 max(E_ion - E_i - E_ion', 0).  Temperatures: HPIE forward at
    sqrt(T_tr T_v), backward at T_tr; EIE and EII at T_v (= T_e); CE at T_tr.
    With molecules, every electronic state of N2, O2, NO and N2+ (seed + 1):
    HPIE and EIE between states as above with dE the term difference, the
    band's A ~ logU(1e5, 1e8) s^-1, and per state dissociation into the
    products of DISS_PRODUCTS (N+ with its ground-term degeneracy as partition
    function): HPID C ~ logU(1e21, 1e22), n = -1.6, EID C ~ logU(1e23, 1e25),
    n = -1.6, both with E_a = c2 (E_diss - T_e - G_e(0)) and E_diss = D0 +
    G_X(0) (the energy zero of the molecule's partition function is the
    bottom of the X well); HPID forward at sqrt(T_tr T_v), backward at T_tr,
    EID at T_v.  Heavy colliders: every species but e-, weight 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    names = [sp.name for sp in species]
    recs = []
    atoms = [a for a in ("N", "O") if a in names and species[names.index(a)].kind == KIND_ATOM]
    ion_of = lambda a: names.index(a + "+") if a + "+" in names else -1
    for a in atoms:
        other = [b for b in atoms if b != a]
        sp = species[names.index(a)]
        L = min(n_model, sp.level_E.size)
        E = sp.level_E[:L]
        dE = C2_CM_K * np.maximum(E[None, :] - E[:, None], 0.0)
        hpie = _arrhenius_triples(rng, L * L, 1e-14, 1e-11, 0.0, 1.0, dE.ravel()).reshape(L, L, 3)
        eie = _arrhenius_triples(rng, L * L, 1e-10, 1e-7, -0.5, 0.5, dE.ravel()).reshape(L, L, 3)
        A = np.zeros((L, L))
        for hi in range(L):
            for lo in range(hi):
                if rng.uniform() < 0.5:
                    A[hi, lo] = _log_uniform(rng, 1e4, 1e8, 1)[0]
        Ei = ION_ENERGY_CM[a]
        eii = _arrhenius_triples(rng, L, 1e-10, 1e-8, 0.0, 0.5, C2_CM_K * np.maximum(Ei - E, 0.0))
        if other and ion_of(a) >= 0 and ion_of(other[0]) >= 0:
            b = other[0]
            Eb = ION_ENERGY_CM[b]
            ce = _arrhenius_triples(rng, L, 1e-12, 1e-10, 0.0, 0.5,
                                    C2_CM_K * np.maximum(Ei - E - Eb, 0.0))
            partner, partner_ion, pE, pQ = names.index(b), ion_of(b), Eb, ION_Q[b + "+"]
        else:
            ce = np.zeros((L, 3))
            partner, partner_ion, pE, pQ = -1, -1, 0.0, 1.0
        recs.append(CRSpecies(names.index(a), ion_of(a), partner, partner_ion, L,
                              Ei, ION_Q[a + "+"], pE, pQ, hpie, eie, A, eii, ce,
                              np.array([0.5, 1.0, 0.0, 0.0, 0.0, 0.0, 1.0, 1.0,
                                        0.5, 1.0, 0.0, 0.0])))
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    for m in (("N2", "O2", "NO", "N2+") if molecules else ()):
        px, py = DISS_PRODUCTS[m]
        if m not in names or px not in names or py not in names:
            continue
        sp = species[names.index(m)]
        if sp.kind != KIND_MOLECULE:
            continue
        L = min(n_model, sp.el_T.size)
        T = sp.el_T[:L]
        dE = C2_CM_K * np.maximum(T[None, :] - T[:, None], 0.0)
        hpie = _arrhenius_triples(rng, L * L, 1e-14, 1e-11, 0.0, 1.0, dE.ravel()).reshape(L, L, 3)
        eie = _arrhenius_triples(rng, L * L, 1e-10, 1e-7, -0.5, 0.5, dE.ravel()).reshape(L, L, 3)
        A = np.zeros((L, L))
        for hi in range(1, L):
            for lo in range(hi):
                A[hi, lo] = _log_uniform(rng, 1e5, 1e8, 1)[0]
        off = np.concatenate([[0], np.cumsum(sp.el_nv)])
        G0 = np.array([sp.vib_G[off[e]] for e in range(sp.el_T.size)])
        E_diss = DISS_D0_CM[m] + G0[0]
        D = C2_CM_K * np.maximum(E_diss - T - G0[:L], 0.0)
        hpid = np.stack([_log_uniform(rng, 1e21, 1e22, L), np.full(L, -1.6), D], axis=-1)
        eid = np.stack([_log_uniform(rng, 1e23, 1e25, L), np.full(L, -1.6), D], axis=-1)
        qc = lambda p: ION_Q.get(p, 1.0) if species[names.index(p)].kind != KIND_ATOM else 0.0
        recs.append(CRSpecies(names.index(m), -1, -1, -1, L, 0.0, 0.0, 0.0, 0.0, hpie, eie, A,
                              np.zeros((L, 3)), np.zeros((L, 3)),
                              np.array([0.5, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0,
                                        0.5, 1.0, 0.0, 0.0]),
                              diss_x=names.index(px), diss_y=names.index(py), Q_x=qc(px),
                              Q_y=qc(py), E_diss=E_diss, hpid=hpid, eid=eid))
    w = np.array([0.0 if n == "e-" else 1.0 for n in names])
    return CRModel(recs, w)


def tie_lines_to_levels(lines: Lines, species: List[Species], cr: CRModel) -> np.ndarray:
    """(upper, lower) level of every line of a CR atom: the level of its
    atom nearest in energy to E_u and to E_l (ties: the lower level); the
    electronic states (1, 0) of the band system for the lines of a CR
    molecule; -1 for the lines of every other species.  [n_lines, 2] int32."""
    out = np.full((lines.n, 2), -1, np.int32)
    for rec in cr.species:
        sel = np.nonzero(lines.species == rec.species)[0]
        if species[rec.species].kind == KIND_MOLECULE:
            out[sel] = (1, 0)   # the band system: upper electronic state 1, lower 0
            continue
        E = species[rec.species].level_E
        for col, Ev in ((0, lines.Eu_ev[sel]), (1, lines.El_ev[sel])):
            out[sel, col] = np.argmin(np.abs(Ev[:, None] - E[None, :]), axis=1)
    return out


def lines_on_levels(lines: Lines, species: List[Species], cr: CRModel, grid: Grid,
                    seed: int = 11864, offset: float = 20.0):
    """Put the lines of the CR atoms on transitions between table levels: a
    line keeps its A and takes the level pair nearest in energy to its drawn
    E_u and E_l, with upper energy E_lev(u) + d_u, lower energy E_lev(l) + d_l
    (d ~ U(-offset, offset) cm^-1, a seeded fine-structure spread), nu0 their
    difference and the levels' degeneracies.  A line whose nearest pair is
    not upper above lower, or whose new centre leaves the grid, keeps its
    drawn values and no levels.  The rovibronic lines of a CR molecule keep
    their values and take the electronic states (1, 0) of their band system.  (A line far from the levels it is tied to
    would take its Boltzmann share of each level at T_v, so that in the
    cold-T_v cells behind the shock a line whose nu0 falls short of the gap
    between its levels reads an inversion of order e^{c2 (gap - nu0)/T_v}
    from populations that are not inverted.)  Returns the lines re-sorted by
    nu0 and their [n_lines, 2] levels."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = {f.name: getattr(lines, f.name).copy() for f in dataclasses.fields(lines)}
    lev = np.full((lines.n, 2), -1, np.int32)
    for rec in cr.species:
        sel = np.nonzero(lines.species == rec.species)[0]
        if species[rec.species].kind == KIND_MOLECULE:
            lev[sel] = (1, 0)   # rovibronic lines of the band system 1 -> 0
            continue
        E, g = species[rec.species].level_E, species[rec.species].level_g
        u = np.argmin(np.abs(lines.Eu_ev[sel][:, None] - E[None, :]), axis=1)
        l = np.argmin(np.abs(lines.El_ev[sel][:, None] - E[None, :]), axis=1)
        eu = E[u] + rng.uniform(-offset, offset, sel.size)
        el = E[l] + rng.uniform(-offset, offset, sel.size)
        nu = eu - el
        ok = (u > l) & (nu >= grid.nu_min) & (nu <= grid.nu_max)
        t = sel[ok]
        d["Eu_ev"][t], d["El_ev"][t], d["nu0"][t] = eu[ok], el[ok], nu[ok]
        d["gu"][t], d["gl"][t] = g[u[ok]], g[l[ok]]
        lev[t, 0], lev[t, 1] = u[ok], l[ok]
    order = np.argsort(d["nu0"], kind="stable")
    return (Lines(**{k: np.ascontiguousarray(v[order]) for k, v in d.items()}),
            np.ascontiguousarray(lev[order]))


def with_cr(wl: Workload, n_model: int = 18, seed: int = 11863) -> Workload:
    """The workload with QSS-CR populations for its atoms N and O, whose
    lines are put on transitions between their table levels
    (lines_on_levels)."""
    cr = air_cr(wl.species, n_model, seed)
    lines, lev = lines_on_levels(wl.lines, wl.species, cr, wl.grid)
    return dataclasses.replace(wl, cr=cr, lines=lines, line_levels=lev)


def none_species(name: str) -> Species:
    return Species(name, KIND_NONE, AIR11_MASS.get(name, 1.0))


def _vib_ladder(omega, omega_x, nv):
    v = np.arange(nv, dtype=np.float64)
    return omega * (v + 0.5) - omega_x * (v + 0.5) ** 2


def molecule_species(rng, name: str, n_v: int, J_max: int = 151) -> Species:
    """Diatomic with two electronic states (ground 'X' and one excited upper
    state), each with an n_v-level anharmonic vibrational ladder and one
    rigid-rotor constant B ~ U(1.5, 2.0) cm^-1 (D = 0)."""
    g_ground = {"N2": 1.0, "N2+": 2.0, "NO": 4.0, "O2": 3.0}.get(name, 1.0)
    T_up = rng.uniform(20000.0, 60000.0)
    g_up = float(rng.integers(1, 7))
    om = rng.uniform(1000.0, 2500.0, 2)
    G_lo = _vib_ladder(om[0], om[0] / 200.0, n_v)
    G_up = _vib_ladder(om[1], om[1] / 200.0, n_v)
    B = rng.uniform(1.5, 2.0, 2)
    return Species(
        name, KIND_MOLECULE, AIR11_MASS.get(name, 28.0),
        el_T=np.array([0.0, T_up]), el_g=np.array([g_ground, g_up]),
        el_nv=np.array([n_v, n_v], np.int32), el_Jmax=np.array([J_max, J_max], np.int32),
        vib_G=np.concatenate([G_lo, G_up]),
        vib_B=np.concatenate([np.full(n_v, B[0]), np.full(n_v, B[1])]),
        vib_D=np.zeros(2 * n_v))


def atomic_lines(rng, sp_index: int, n: int, nu_lo: float, nu_hi: float,
                 Eu_lo_ev: float = 10.0, Eu_hi_ev: float = 14.0) -> Dict[str, np.ndarray]:
    """n synthetic atomic lines: nu0 ~ U(nu_lo, nu_hi), A ~ logU(1e4, 1e9),
    E_u ~ U(10, 14) eV, E_l = E_u - nu0, g_u, g_l ~ U{2..12}.  A line whose
    E_l would be negative has its E_u redrawn from U(nu0, 14 eV)."""
    nu0 = rng.uniform(nu_lo, nu_hi, n)
    A = _log_uniform(rng, 1e4, 1e9, n)
    Eu = rng.uniform(Eu_lo_ev, Eu_hi_ev, n) * EV_CM
    bad = Eu - nu0 < 0.0
    if bad.any():
        Eu[bad] = rng.uniform(nu0[bad], Eu_hi_ev * EV_CM)
    El = Eu - nu0
    gu = rng.integers(2, 13, n).astype(np.float64)
    gl = rng.integers(2, 13, n).astype(np.float64)
    z = np.zeros(n)
    return dict(nu0=nu0, A=A, Eu_ev=Eu, Eu_rot=z.copy(), El_ev=El, El_rot=z.copy(),
                gu=gu, gl=gl, species=np.full(n, sp_index, np.int32))


def rovib_lines(rng, sp: Species, sp_index: int, n_target: int,
                nu_min: float, nu_max: float) -> Dict[str, np.ndarray]:
    """Synthetic rovibronic system upper(e=1) -> lower(e=0): P and R branches,
    J'' = 0..150, nu = nu_band(v', v'') + B'J'(J'+1) - B''J''(J''+1),
    A = A_band S / (2J'+1) with S_P = J'+1, S_R = J' (Sigma-Sigma column of
    the Hund (a) Hoenl-London table), A_band ~ logU(1e5, 1e8),
    g = g_el (2J+1).  Lines outside [nu_min, nu_max] are rejected; (v', v'')
    bands are added in a seeded order until n_target lines are collected."""
    nv = int(sp.el_nv[0])
    G_lo, G_up = sp.vib_G[:nv], sp.vib_G[nv:2 * nv]
    B_lo, B_up = float(sp.vib_B[0]), float(sp.vib_B[nv])
    T_up, g_lo_el, g_up_el = float(sp.el_T[1]), float(sp.el_g[0]), float(sp.el_g[1])
    Jpp = np.arange(0, 151)
    # P branch: J' = J'' - 1 (J'' >= 1); R branch: J' = J'' + 1
    Jl = np.concatenate([Jpp[1:], Jpp]).astype(np.float64)
    Ju = np.concatenate([Jpp[1:] - 1, Jpp + 1]).astype(np.float64)
    n_P = Jpp.size - 1
    S = np.where(np.arange(Ju.size) < n_P, Ju + 1.0, Ju)                 # P: J'+1 ; R: J'
    Eu_rot = B_up * Ju * (Ju + 1.0)
    El_rot = B_lo * Jl * (Jl + 1.0)
    out = {k: [] for k in ("nu0", "A", "Eu_ev", "Eu_rot", "El_ev", "El_rot", "gu", "gl")}
    pairs = [(a, b) for a in range(nv) for b in range(nv)]
    order = rng.permutation(len(pairs))
    count = 0
    for pi in order:
        vu, vl = pairs[pi]
        Eu_ev = T_up + G_up[vu]
        El_ev = G_lo[vl]
        nu0 = (Eu_ev - El_ev) + (Eu_rot - El_rot)
        keep = (nu0 >= nu_min) & (nu0 <= nu_max)
        m = int(keep.sum())
        if m == 0:
            continue
        A_band = _log_uniform(rng, 1e5, 1e8, 1)[0]
        out["nu0"].append(nu0[keep])
        out["A"].append(A_band * S[keep] / (2.0 * Ju[keep] + 1.0))
        out["Eu_ev"].append(np.full(m, Eu_ev))
        out["Eu_rot"].append(Eu_rot[keep])
        out["El_ev"].append(np.full(m, El_ev))
        out["El_rot"].append(El_rot[keep])
        out["gu"].append(g_up_el * (2.0 * Ju[keep] + 1.0))
        out["gl"].append(g_lo_el * (2.0 * Jl[keep] + 1.0))
        count += m
        if count >= n_target:
            break
    d = {k: np.concatenate(v)[:n_target] for k, v in out.items()}
    d["species"] = np.full(d["nu0"].shape[0], sp_index, np.int32)
    return d


def air_band_systems(seed: int = 11866, nv: int = 16, J_max: int = 150) -> List[BandSystem]:
    """Four seeded band systems, one per diatomic radiator of the air species
    list, near the magnitudes of the real ones: N2 (a Pi - Pi system, Hund
    (a)), N2+ (a doublet Sigma - Sigma system, Hund (b)), NO (a Sigma - Pi
    system, Hund (a), dLambda = -1) and O2 (a Sigma - Sigma system, Hund
    (a)).  Re'^2 ~ logU(1e-3, 1) per band."""
    rng = np.random.Generator(np.random.PCG64(seed))
    spec = [("N2", 0, 1, 1, 88000.0, 59600.0), ("N2+", 1, 0, 0, 25500.0, 0.0),
            ("NO", 0, 0, 1, 44000.0, 0.0), ("O2", 0, 0, 0, 49800.0, 0.0)]
    out = []
    for name, hund, lu, ll, Tu, Tl in spec:
        we = rng.uniform(1000.0, 2400.0, 2)
        Be = rng.uniform(1.4, 2.0, 2)
        out.append(BandSystem(
            species=AIR11.index(name), hund=hund, Lambda_u=lu, Lambda_l=ll, Te_u=Tu, Te_l=Tl,
            g_u=float(2 - (lu == 0)), g_l=float(2 - (ll == 0)),
            we_u=float(we[0]), wexe_u=float(we[0] / rng.uniform(60.0, 120.0)), weye_u=float(rng.uniform(-0.5, 0.5)),
            Be_u=float(Be[0]), ae_u=float(rng.uniform(0.01, 0.03)), De_u=float(rng.uniform(4e-6, 8e-6)),
            be_u=float(rng.uniform(-1e-7, 1e-7)), gamma_u=float(rng.uniform(0.005, 0.03) if hund else 0.0),
            we_l=float(we[1]), wexe_l=float(we[1] / rng.uniform(60.0, 120.0)), weye_l=float(rng.uniform(-0.5, 0.5)),
            Be_l=float(Be[1]), ae_l=float(rng.uniform(0.01, 0.03)), De_l=float(rng.uniform(4e-6, 8e-6)),
            be_l=float(rng.uniform(-1e-7, 1e-7)), gamma_l=float(rng.uniform(0.005, 0.03) if hund else 0.0),
            nv_u=nv, nv_l=nv, J_max=J_max, Re2=_log_uniform(rng, 1e-3, 1.0, nv * nv)))
    return out


def merge_sorted(parts: List[Dict[str, np.ndarray]]) -> Lines:
    d = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    order = np.argsort(d["nu0"], kind="stable")
    return Lines(**{k: np.ascontiguousarray(v[order]) for k, v in d.items()})


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def slab_equilibrium(n_cells=64, dx=0.05, n_lines_per_species=1000, n_points=200_000,
                     nu_min=5000.0, nu_max=80000.0, band_points=None, seed=11856,
                     identical_cells=False, n_mu=0) -> Workload:
    """Plain method, single 1-D tangent-slab line of sight: T_e = T_v = T_tr
    ~ U(6000, 12000) K per cell, N and O atoms logU(1e15, 1e17) cm^-3, n_e
    logU(1e15, 1e16) cm^-3; N and O lines with nu0 ~ U(5000, 80000) cm^-1;
    uniform grid; one wall-normal ray."""
    rng = np.random.Generator(np.random.PCG64(seed))
    species = [atom_species(rng, "N"), atom_species(rng, "O")]
    lines = merge_sorted([
        atomic_lines(rng, 0, n_lines_per_species, nu_min, nu_max),
        atomic_lines(rng, 1, n_lines_per_species, nu_min, nu_max)])
    nc = 1 if identical_cells else n_cells
    T = rng.uniform(6000.0, 12000.0, nc)
    N = _log_uniform(rng, 1e15, 1e17, (nc, 2))
    ne = _log_uniform(rng, 1e15, 1e16, nc)
    if identical_cells:
        T, N, ne = np.repeat(T, n_cells), np.repeat(N, n_cells, 0), np.repeat(ne, n_cells)
    cells = Cells(T_tr=T.copy(), T_v=T.copy(), N=np.ascontiguousarray(N), n_e=ne)
    grid = Grid(nu_min, nu_max, n_points, band_points or n_points)
    geom = SlabGeometry(dx=np.full(n_cells, dx), n_mu=n_mu)
    return Workload("slab-equilibrium", species, lines, cells, grid, geom,
                    dict(seed=seed))


def _air_species(rng, n_v: int, radiators=("N", "O", "N2", "N2+", "NO", "O2")) -> List[Species]:
    sp = []
    for name in AIR11:
        if name in ("N", "O") and name in radiators:
            sp.append(atom_species(rng, name))
        elif name in ("N2", "N2+", "NO", "O2") and name in radiators:
            sp.append(molecule_species(rng, name, n_v))
        else:
            sp.append(none_species(name))
    return sp


def _air_lines(rng, species, n_atomic, n_rovib, nu_min, nu_max) -> Lines:
    parts = []
    iN, iO = AIR11.index("N"), AIR11.index("O")
    parts.append(atomic_lines(rng, iN, n_atomic // 2, nu_min, nu_max))
    parts.append(atomic_lines(rng, iO, n_atomic - n_atomic // 2, nu_min, nu_max))
    mols = ["N2", "N2+", "NO", "O2"]
    for j, name in enumerate(mols):
        n_t = n_rovib // 4 + (1 if j < n_rovib % 4 else 0)
        if n_t:
            idx = AIR11.index(name)
            parts.append(rovib_lines(rng, species[idx], idx, n_t, nu_min, nu_max))
    return merge_sorted(parts)


def _fractions_to_N(f_mol, f_ion, N_tot):
    """Split total density into the 11 species from molecule / ion fractions."""
    n = f_mol.shape[0]
    N = np.zeros((n, 11))
    mol_split = {"N2": 0.70, "O2": 0.15, "NO": 0.12, "N2+": 0.02, "O2+": 0.005, "NO+": 0.005}
    ion_split = {"N+": 0.7, "O+": 0.3}
    f_atom = 1.0 - f_mol - f_ion
    for k, w in mol_split.items():
        N[:, AIR11.index(k)] = w * f_mol * N_tot
    for k, w in ion_split.items():
        N[:, AIR11.index(k)] = w * f_ion * N_tot
    N[:, AIR11.index("N")] = 0.78 * f_atom * N_tot
    N[:, AIR11.index("O")] = 0.22 * f_atom * N_tot
    ne = sum(N[:, AIR11.index(k)] for k in ION_SPECIES)
    N[:, AIR11.index("e-")] = ne
    return N, ne


def stagnation_line(n_cells=400, length=4.0, n_atomic=200_000, n_rovib=2_000_000,
                    n_points=1 << 21, nu_min=1000.0, nu_max=100000.0, band_points=None,
                    n_mu=16, n_v=50, seed=11857) -> Workload:
    """1-D stagnation-line nonequilibrium case: shock at x = 0 (far, free
    boundary), wall at x = length; T_tr = 1e4 + 2e4 exp(-x/0.4) relaxing,
    T_v = max(500, 1e4 - 9500 exp(-x/0.6)) lagging, +-1% seeded noise;
    11 species with molecules decaying and atoms/ions rising along x,
    N_tot 2e16..8e16; n_e = sum of ion densities."""
    rng = np.random.Generator(np.random.PCG64(seed))
    species = _air_species(rng, n_v)
    lines = _air_lines(rng, species, n_atomic, n_rovib, nu_min, nu_max)
    dx = length / n_cells
    x = (np.arange(n_cells) + 0.5) * dx * (4.0 / length)   # profile shape in 4 cm units
    noise = lambda: 1.0 + rng.uniform(-0.01, 0.01, n_cells)
    T_tr = (1e4 + 2e4 * np.exp(-x / 0.4)) * noise()
    T_v = np.maximum(500.0, 1e4 - 9500.0 * np.exp(-x / 0.6)) * noise()
    N_tot = 2e16 + 6e16 * (1.0 - np.exp(-x / 1.5))
    f_mol = 0.7 * np.exp(-x / 0.3) + 0.005
    f_ion = 1e-3 + 0.05 * (1.0 - np.exp(-x / 0.5))
    N, ne = _fractions_to_N(f_mol, f_ion, N_tot)
    cells = Cells(T_tr=T_tr, T_v=T_v, N=np.ascontiguousarray(N), n_e=ne)
    grid = Grid(nu_min, nu_max, n_points, band_points or n_points)
    geom = SlabGeometry(dx=np.full(n_cells, dx), n_mu=n_mu)
    return Workload("stagnation-line", species, lines, cells, grid, geom, dict(seed=seed))


def _smooth_field(rng, X, Rr, Lx, R, n_bumps=6):
    """Seeded smooth field in [0, 1] on the (x, r) plane: normalised sum of
    Gaussian bumps."""
    f = np.zeros_like(X)
    for _ in range(n_bumps):
        x0, r0 = rng.uniform(0, Lx), rng.uniform(0, R)
        sx, sr = rng.uniform(0.15, 0.5) * Lx, rng.uniform(0.15, 0.5) * R
        f += rng.uniform(0.3, 1.0) * np.exp(-((X - x0) / sx) ** 2 - ((Rr - r0) / sr) ** 2)
    f -= f.min()
    return f / max(f.max(), 1e-300)


def axisymmetric(nx=256, nr=128, Lx=100.0, R=50.0, n_atomic=250_000, n_rovib=750_000,
                 n_points=1 << 20, nu_min=1000.0, nu_max=100000.0, band_points=65536,
                 n_wall=64, wall_R=30.0, n_mu=16, n_phi=16, n_v=50, seed=11858) -> Workload:
    """2-D axisymmetric afterbody: structured nx x nr cells over
    [0, Lx] x [0, R] cm with smooth seeded T_tr in 3000..10000 K,
    T_v = T_tr (1 + 0.3 h) with smooth h in [0, 1] (T_v > T_tr in the wake),
    N, O 1e14..1e16, molecules 1e13..1e16, ions / e- 1e11..1e15 cm^-3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    species = _air_species(rng, n_v)
    lines = _air_lines(rng, species, n_atomic, n_rovib, nu_min, nu_max)
    xc = (np.arange(nx) + 0.5) * Lx / nx
    rc = (np.arange(nr) + 0.5) * R / nr
    X, Rr = np.meshgrid(xc, rc, indexing="ij")
    s1 = _smooth_field(rng, X, Rr, Lx, R)
    h = _smooth_field(rng, X, Rr, Lx, R)
    T_tr = 3000.0 + 7000.0 * s1
    T_v = T_tr * (1.0 + 0.3 * h)
    fa = _smooth_field(rng, X, Rr, Lx, R)
    fm = _smooth_field(rng, X, Rr, Lx, R)
    fi = _smooth_field(rng, X, Rr, Lx, R)
    N = np.zeros((nx * nr, 11))
    atoms = 10.0 ** (14.0 + 2.0 * fa.ravel())
    mols = 10.0 ** (13.0 + 3.0 * fm.ravel())
    ions = 10.0 ** (11.0 + 4.0 * fi.ravel())
    N[:, AIR11.index("N")] = 0.78 * atoms
    N[:, AIR11.index("O")] = 0.22 * atoms
    for k, w in {"N2": 0.6, "O2": 0.15, "NO": 0.2, "N2+": 0.05}.items():
        N[:, AIR11.index(k)] = w * mols
    for k, w in {"O2+": 0.05, "NO+": 0.15, "N+": 0.5, "O+": 0.3}.items():
        N[:, AIR11.index(k)] = w * ions
    ne = sum(N[:, AIR11.index(k)] for k in ION_SPECIES)
    N[:, AIR11.index("e-")] = ne
    cells = Cells(T_tr=T_tr.ravel().copy(), T_v=T_v.ravel().copy(),
                  N=np.ascontiguousarray(N), n_e=ne.copy())
    grid = Grid(nu_min, nu_max, n_points, band_points)
    wall_r = (np.arange(n_wall) + 0.5) * wall_R / n_wall
    geom = AxiGeometry(nx, nr, Lx, R, wall_r, n_mu, n_phi)
    return Workload("axisymmetric", species, lines, cells, grid, geom, dict(seed=seed))


# Named workloads at full size -------------------------------------------------

def config_slab() -> Workload:
    return slab_equilibrium()


def config_stagnation() -> Workload:
    return stagnation_line()


def config_axi() -> Workload:
    return axisymmetric()


def config_axi_large() -> Workload:
    return axisymmetric(nx=512, nr=256, n_atomic=1_000_000, n_rovib=3_000_000,
                        n_points=1 << 22, band_points=131072, n_wall=256,
                        n_mu=32, n_phi=32, seed=11860)


# Serving requests -------------------------------------------------------------

@dataclasses.dataclass
class LosRequest:
    cells: Cells
    ds: np.ndarray           # per-cell path length, far -> observer order
    k_first: int             # first grid index of the spectral window
    n_window: int            # number of grid points in the window
    species_mask: int        # bit s set: species s radiates in this request
    arrival: float = 0.0     # seconds from stream start


def serving_requests(n_requests: int, n_points: int, rate_hz: float = 0.0,
                     min_cells=16, max_cells=2048, min_win=10_000, max_win=1_000_000,
                     seed=11859) -> List[LosRequest]:
    """Line-of-sight requests: cell count logU[16, 2048], ds ~ U(0.01, 0.1) cm,
    T_tr ~ U(3000, 30000) and T_v ~ U(3000, 15000) K varying smoothly along the
    LOS, 11 species, a random non-empty radiating subset of
    {N, O, N2, O2, NO, N2+}, window length logU[1e4, 1e6] points at a uniform
    start; Poisson arrivals at rate_hz (0: all at t = 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    t = 0.0
    cand = [AIR11.index(s) for s in ("N", "O", "N2", "O2", "NO", "N2+")]
    for _ in range(n_requests):
        nc = int(np.round(_log_uniform(rng, min_cells, max_cells, 1)[0]))
        nw = int(np.round(_log_uniform(rng, min_win, max_win, 1)[0]))
        nw = min(nw, n_points)
        k0 = int(rng.integers(0, n_points - nw + 1))
        u = np.linspace(0.0, 1.0, nc)
        def smooth(lo, hi):
            a = rng.uniform(lo, hi, 3)
            return a[0] + (a[1] - a[0]) * u + (a[2] - 0.5 * (a[0] + a[1])) * 4 * u * (1 - u)
        T_tr = np.clip(smooth(3000.0, 30000.0), 3000.0, 30000.0)
        T_v = np.clip(smooth(3000.0, 15000.0), 3000.0, 15000.0)
        f_mol = np.clip(smooth(0.0, 0.7), 0.0, 0.7)
        f_ion = np.clip(smooth(1e-4, 0.05), 1e-4, 0.05)
        N_tot = np.clip(smooth(1e16, 1e17), 1e16, 1e17)
        N, ne = _fractions_to_N(f_mol, f_ion, N_tot)
        mask = 0
        while mask == 0:
            pick = rng.random(len(cand)) < 0.5
            for s, p in zip(cand, pick):
                if p:
                    mask |= 1 << s
        if rate_hz > 0:
            t += rng.exponential(1.0 / rate_hz)
        reqs.append(LosRequest(Cells(T_tr, T_v, np.ascontiguousarray(N), ne),
                               rng.uniform(0.01, 0.1, nc), k0, nw, mask, t))
    return reqs


def sample_points(grid: Grid, lines: Lines, n: int, seed: int = 7, cluster: int = 32) -> np.ndarray:
    """Seeded sorted unique grid indices for sampled comparisons: half in
    uniformly placed clusters of `cluster` consecutive points, half in
    clusters centred on the strongest (largest A) line centres."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = (grid.nu_max - grid.nu_min) / (grid.n_points - 1)
    n_cl = max(1, n // cluster)
    starts = list(rng.integers(0, max(1, grid.n_points - cluster), (n_cl + 1) // 2))
    strong = np.argsort(lines.A)[::-1][: max(1, n_cl // 2) * 4]
    pick = rng.choice(strong, size=n_cl // 2, replace=False) if n_cl // 2 else []
    for i in pick:
        kc = int(round((lines.nu0[i] - grid.nu_min) / h))
        starts.append(min(max(0, kc - cluster // 2), max(0, grid.n_points - cluster)))
    ks = np.unique(np.concatenate([np.arange(s, s + cluster) for s in starts]))
    return ks[(ks >= 0) & (ks < grid.n_points)].astype(np.int64)
