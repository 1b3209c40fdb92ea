"""Parity of the QSS collisional-radiative populations (Sec. 2.1 CR model:
R n = b with the ground-state closure, LU solve) through the C ABI with the
FP64 oracle, and of the line and continuum coefficients and the flux that use
them.  Bars: populations within 1e-12 relative per level; LRT_FP64
coefficients and fluxes within 1e-12, LRT_FP32_COMP within 1e-5 (normwise per
cell, relative for integrals and fluxes), knife-edge window bounds excluded."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2604_11856_amd import lrt, synth
from parity_util import edge_mask, normwise, say

pytestmark = pytest.mark.gpu

TOL = {lrt.LRT_FP64: 1e-12, lrt.LRT_FP32_COMP: 1e-5}
PRECS = [lrt.LRT_FP64, lrt.LRT_FP32_COMP]
POP_TOL = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch


def gpu_coeffs(ctx, band, prec, torch):
    eta, kap, esc = ctx.coeffs_torch(band, prec)
    torch.cuda.synchronize()
    if prec == lrt.LRT_FP32_COMP:
        return lrt.scaled_to_f64(eta, kap, esc)
    return eta.cpu().numpy(), kap.cpu().numpy()


def rel_err(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    zero = ref == 0.0
    assert np.all(got[zero] == 0.0)
    return float(np.max(np.abs(got[~zero] / ref[~zero] - 1.0))) if np.any(~zero) else 0.0


def check_populations(ctx, wl, label):
    ref = O.cr_populations(wl.cr, wl.species, wl.cells)
    worst = 0.0
    for a, (rec, r) in enumerate(zip(wl.cr.species, ref)):
        got = ctx.cr_populations(a, r.shape[1])
        worst = max(worst, rel_err(got, r))
    say("%s: populations max rel %.3e" % (label, worst))
    assert worst <= POP_TOL
    return ref


def cr_stagnation(n_cells=24, **kw):
    wl = synth.stagnation_line(n_cells=n_cells, **kw)
    return synth.with_cr(wl)


def test_cr_populations_stagnation_cells(torch_dev):
    """Nonequilibrium stagnation-line cells (T_tr up to 30,000 K, T_v from
    500 K), both atoms with ions and charge exchange; one cell without N
    atoms (all zero) and one with T_tr = T_v."""
    wl = cr_stagnation(n_cells=24, n_atomic=200, n_rovib=200, n_points=2000, band_points=2000)
    iN = [s.name for s in wl.species].index("N")
    wl.cells.N[3, iN] = 0.0
    wl.cells.T_v[7] = wl.cells.T_tr[7]
    ctx = lrt.Context(0).load(wl)
    ref = check_populations(ctx, wl, "stagnation cells")
    assert np.all(ref[0][3] == 0.0) and np.all(ref[0][np.arange(24) != 3] > 0.0)
    ctx.close()


@pytest.mark.parametrize("n_model", [2, 13, 20])
def test_cr_populations_model_sizes(n_model, torch_dev):
    """Smallest system (2 levels, long Boltzmann tail), a middle one and no
    tail at all (every level solved)."""
    wl = synth.stagnation_line(n_cells=10, n_atomic=100, n_rovib=100, n_points=1000, band_points=1000)
    wl = synth.with_cr(wl, n_model=n_model)
    ctx = lrt.Context(0).load(wl)
    check_populations(ctx, wl, "n_model %d" % n_model)
    ctx.close()


def test_cr_populations_largest_atom_no_ion(torch_dev):
    """An atom with the largest table (64 levels, all solved) in the
    two-species slab, which has no ions: no recombination source and no
    charge exchange."""
    wl = synth.slab_equilibrium(n_cells=8, n_lines_per_species=50, n_points=2000)
    rng = np.random.Generator(np.random.PCG64(17))
    wl.species[0] = synth.atom_species(rng, "N", n_levels=64)
    wl = synth.with_cr(wl, n_model=64)
    assert wl.cr.species[0].ion == -1 and wl.cr.species[0].partner == -1
    ctx = lrt.Context(0).load(wl)
    check_populations(ctx, wl, "64 levels, no ion")
    ctx.close()


def small_molecule(n_el, n_v=4, J_max=30):
    T_e = np.array([0.0, 30000.0, 45000.0, 52000.0][:n_el])
    G = []
    for e in range(n_el):
        om = 1500.0 + 200.0 * e
        v = np.arange(n_v) + 0.5
        G.append(om * v - om / 200.0 * v * v)
    return synth.Species("N2", synth.KIND_MOLECULE, 28.0, el_T=T_e,
                         el_g=np.array([1.0, 3.0, 2.0, 6.0][:n_el]),
                         el_nv=np.full(n_el, n_v, np.int32), el_Jmax=np.full(n_el, J_max, np.int32),
                         vib_G=np.concatenate(G), vib_B=np.repeat(np.linspace(1.6, 1.9, n_el), n_v),
                         vib_D=np.zeros(n_el * n_v))


def test_cr_molecule_with_tail_and_dissociation(torch_dev):
    """A four-state diatomic with three states solved (one in the two-
    temperature Boltzmann tail), dissociating into N + N, next to a CR atom;
    populations, and eta / kappa of its rovibronic lines (band 1 -> 0) and
    of the atom's lines, in nonequilibrium cells."""
    rng = np.random.Generator(np.random.PCG64(41))
    species = [small_molecule(4), synth.atom_species(rng, "N"), synth.none_species("N+"),
               synth.none_species("e-")]
    cr = synth.air_cr(species, n_model=3)
    assert [r.species for r in cr.species] == [1, 0] and cr.species[1].n_model == 3
    n_cells = 12
    Ttr = rng.uniform(6000.0, 25000.0, n_cells)
    Tv = rng.uniform(3000.0, 12000.0, n_cells)
    N = np.stack([10 ** rng.uniform(15, 17, n_cells), 10 ** rng.uniform(15, 17, n_cells),
                  10 ** rng.uniform(13, 15, n_cells), np.zeros(n_cells)], axis=1)
    N[:, 3] = N[:, 2]
    cells = synth.Cells(Ttr, Tv, N, N[:, 2].copy())
    parts = [synth.atomic_lines(rng, 1, 300, 15000.0, 40000.0),
             synth.rovib_lines(rng, species[0], 0, 600, 15000.0, 40000.0)]
    lines = synth.merge_sorted(parts)
    grid = synth.Grid(15000.0, 40000.0, 20001, 7000)
    wl = synth.Workload("molecule", species, lines, cells, grid, synth.SlabGeometry(np.full(n_cells, 0.1), 0))
    wl.cr = cr
    wl.lines, wl.line_levels = synth.lines_on_levels(lines, species, cr, grid)
    assert np.any(wl.line_levels[wl.lines.species == 0, 0] == 1)
    ctx = lrt.Context(0).load(wl)
    ref = check_populations(ctx, wl, "4-state molecule")
    assert np.all(ref[1] > 0)
    e_r, k_r, _ = O.coeffs(species, wl.lines, cells, grid, cr=cr, line_levels=wl.line_levels)
    for prec in PRECS:
        we = wk = 0.0
        for b in range(ctx.sizes()["n_bands"]):
            e, k = gpu_coeffs(ctx, b, prec, torch_dev)
            k0 = b * grid.band_points
            m = edge_mask(wl, k0, e.shape[1])
            we = max(we, normwise(e, e_r[:, k0:k0 + e.shape[1]], m))
            wk = max(wk, normwise(k, k_r[:, k0:k0 + e.shape[1]], m))
        say("4-state molecule coeffs prec %d: eta %.3e kappa %.3e" % (prec, we, wk))
        assert we <= TOL[prec] and wk <= TOL[prec]
    ctx.close()


def test_cr_coeffs_all_bands(torch_dev):
    """eta and kappa of the lines with levels (and the bound-free absorption)
    from the QSS-CR populations, over ragged bands, with and without the
    continuum; clearing the CR atoms gives the Boltzmann coefficients back."""
    wl = cr_stagnation(n_cells=12, n_atomic=2000, n_rovib=6000, n_points=30_000, band_points=11_000,
                       n_mu=2)
    e_r, k_r, _ = O.coeffs(wl.species, wl.lines, wl.cells, wl.grid, cr=wl.cr, line_levels=wl.line_levels)
    e_b, k_b, _ = O.coeffs(wl.species, wl.lines, wl.cells, wl.grid)
    assert normwise(e_r, e_b) > 1e-3   # the populations do change the result
    ctx = lrt.Context(0).load(wl)
    nb = ctx.sizes()["n_bands"]
    for prec in PRECS:
        we = wk = 0.0
        for b in range(nb):
            e, k = gpu_coeffs(ctx, b, prec, torch_dev)
            k0 = b * wl.grid.band_points
            sl = slice(k0, k0 + e.shape[1])
            m = edge_mask(wl, k0, e.shape[1])
            we = max(we, normwise(e, e_r[:, sl], m))
            wk = max(wk, normwise(k, k_r[:, sl], m))
        say("CR coeffs prec %d: eta %.3e kappa %.3e" % (prec, we, wk))
        assert we <= TOL[prec] and wk <= TOL[prec]
    # with the continuum: the bound-free absorption uses the CR populations
    wl.continuum = synth.air_continuum(wl.species)
    e_c, k_c = O.continuum(wl.species, wl.cells, wl.grid, wl.continuum, cr=wl.cr)
    ctx.set_continuum(wl.continuum)
    for prec in PRECS:
        e, k = gpu_coeffs(ctx, 0, prec, torch_dev)
        n = e.shape[1]
        m = edge_mask(wl, 0, n)
        we = normwise(e, e_r[:, :n] + e_c[:, :n], m)
        wk = normwise(k, k_r[:, :n] + k_c[:, :n], m)
        say("CR + continuum prec %d: eta %.3e kappa %.3e" % (prec, we, wk))
        assert we <= TOL[prec] and wk <= TOL[prec]
    ctx.set_continuum(None)
    ctx.set_cr(None)
    e, k = gpu_coeffs(ctx, 0, lrt.LRT_FP64, torch_dev)
    m = edge_mask(wl, 0, e.shape[1])
    assert normwise(e, e_b[:, :e.shape[1]], m) <= 1e-12
    assert normwise(k, k_b[:, :e.shape[1]], m) <= 1e-12
    ctx.close()


def test_cr_solve_slab(torch_dev):
    """Whole path with QSS-CR populations: wall intensities and flux."""
    wl = cr_stagnation(n_cells=16, n_atomic=1500, n_rovib=3000, n_points=16_384, band_points=5000, n_mu=4)
    ref = O.solve_slab(wl)
    ctx = lrt.Context(0).load(wl)
    for prec in PRECS:
        q, I_int, _ = ctx.solve(prec)
        eI = float(np.max(np.abs(I_int - ref["I_int"]) / np.abs(ref["I_int"])))
        eq = abs(q[0] - ref["q"]) / abs(ref["q"])
        say("CR solve prec %d: I_int %.3e q %.3e" % (prec, eI, eq))
        assert eI <= TOL[prec] and eq <= TOL[prec]
    ctx.close()


def test_cr_full_size_stagnation(torch_dev):
    """The 400-cell, 2.2M-line stagnation line with QSS-CR atoms, in the
    launch configuration the benchmark times: every population of every
    cell, and eta / kappa at sampled points of every cell in FP64 and the
    single-precision form."""
    wl = synth.with_cr(synth.config_stagnation())
    ctx = lrt.Context(0).load(wl)
    check_populations(ctx, wl, "stagnation full size")
    ks = synth.sample_points(wl.grid, wl.lines, 256, seed=29)
    e_r, k_r, _ = O.coeffs(wl.species, wl.lines, wl.cells, wl.grid, ks=ks, cr=wl.cr,
                           line_levels=wl.line_levels)
    cc, kk = O.knife_edges(wl.species, wl.lines, wl.cells, wl.grid, near=ks)
    mask = np.zeros((wl.cells.n, ks.size), bool)
    pos = {int(k): j for j, k in enumerate(ks)}
    for c_, k_ in zip(cc, kk):
        if int(k_) in pos:
            mask[c_, pos[int(k_)]] = True
    for prec in PRECS:
        e, k = gpu_coeffs(ctx, 0, prec, torch_dev)
        we = normwise(e[:, ks], e_r, mask)
        wk = normwise(k[:, ks], k_r, mask)
        say("CR full size prec %d: eta %.3e kappa %.3e" % (prec, we, wk))
        assert we <= TOL[prec] and wk <= TOL[prec]
    ctx.close()


def test_cr_arguments(torch_dev):
    wl = cr_stagnation(n_cells=2, n_atomic=10, n_rovib=10, n_points=1000, band_points=1000)
    cr = wl.cr
    names = [sp.name for sp in wl.species]
    ctx = lrt.Context(0)
    with pytest.raises(lrt.LrtError) as e:
        ctx.set_cr(cr)                           # no species yet
    assert e.value.status == 6
    ctx.set_species(wl.species)
    r0 = cr.species[0]

    def bad(**kw):
        with pytest.raises(lrt.LrtError) as e:
            ctx.set_cr(dataclasses.replace(cr, species=[dataclasses.replace(r0, **kw)]))
        assert e.value.status == 1

    bad(species=0)                               # N2 is a molecule: no ionization for it
    bad(diss_x=3, diss_y=3)                      # dissociation given to an atom
    m0 = [r for r in cr.species if r.diss_x >= 0][0]

    def bad_mol(**kw):
        with pytest.raises(lrt.LrtError) as e:
            ctx.set_cr(dataclasses.replace(cr, species=[dataclasses.replace(m0, **kw)]))
        assert e.value.status == 1

    bad_mol(diss_y=99)
    bad_mol(diss_y=names.index("N+"), Q_y=0.0)   # a non-atomic product needs Q > 0
    bad_mol(hpid=-m0.hpid)
    bad_mol(ion=names.index("N2+"))
    bad(n_model=1)
    bad(n_model=21)                              # the atom has 20 levels
    bad(ion=99)
    bad(partner=r0.species)                      # partner must be another atom
    bad(E_ion=0.0)
    bad(texp=np.array([0.5, 1.5, 0, 0, 0, 0, 1, 1]))
    h = r0.hpie.copy()
    h[0, 1, 0] = -1.0
    bad(hpie=h)
    A = r0.A.copy()
    A[3, 1] = np.nan
    bad(A=A)
    with pytest.raises(lrt.LrtError):
        ctx.set_cr(dataclasses.replace(cr, species=[r0, r0]))   # the same atom twice
    with pytest.raises(lrt.LrtError):
        ctx.set_cr(dataclasses.replace(cr, collider_w=-cr.collider_w))
    ctx.set_cr(cr)
    with pytest.raises(lrt.LrtError) as e:
        ctx.set_line_levels(wl.line_levels)      # no lines yet
    assert e.value.status == 6
    ctx.set_lines(wl.lines)
    with pytest.raises(lrt.LrtError):
        ctx.set_line_levels(wl.line_levels[:-1])
    lev = wl.line_levels.copy()
    names = [sp.name for sp in wl.species]
    mol = np.nonzero(wl.lines.species == names.index("N2"))[0][0]
    lev[mol] = (2, 0)                            # N2 has 2 electronic states
    with pytest.raises(lrt.LrtError):
        ctx.set_line_levels(lev)
    lev = wl.line_levels.copy()
    at = np.nonzero(lev[:, 0] >= 0)[0][0]
    lev[at] = (20, 0)                            # outside the 20-level table
    with pytest.raises(lrt.LrtError):
        ctx.set_line_levels(lev)
    lev[at] = (-1, 3)                            # only one level given
    with pytest.raises(lrt.LrtError):
        ctx.set_line_levels(lev)
    ctx.set_line_levels(wl.line_levels)
    with pytest.raises(lrt.LrtError):
        ctx.cr_populations(5, 20)                # no such record
    ctx.set_cr(None)
    with pytest.raises(lrt.LrtError) as e:
        ctx.cr_populations(0, 20)
    assert e.value.status == 6
    ctx.close()
