"""Parity of the full Lorentz width of atomic lines (Sec. 2.2.1: natural +
per-line Stark + van der Waals) through the C ABI with the FP64 oracle.  Bars
as for the line path (FP64 1e-12, FP32-comp 1e-5, normwise per cell; knife
edges of the window bounds excluded)."""
import numpy as np
import pytest

import oracle as O
from paper_2604_11856_amd import lrt, synth
from parity_util import normwise, say

pytestmark = pytest.mark.gpu

TOL = {lrt.LRT_FP64: 1e-12, lrt.LRT_FP32_COMP: 1e-5}
PRECS = [lrt.LRT_FP64, lrt.LRT_FP32_COMP]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch


def stark_workload(n_e):
    wl = synth.stagnation_line(n_cells=10, n_atomic=3000, n_rovib=3000, n_points=40_000,
                               band_points=15_000, n_mu=3, seed=7)
    wl.cells.n_e[:] = n_e
    wl.lorentz_E_ion = synth.air_ionization_energies(wl.species)
    return wl


@pytest.mark.parametrize("n_e", [1e15, 3e17])
def test_full_lorentz_coeffs(n_e, torch_dev):
    """eta / kappa over ragged bands with per-line Lorentz widths, at a low and
    a Stark-dominated electron density."""
    torch = torch_dev
    wl = stark_workload(n_e)
    E = wl.lorentz_E_ion
    e_ref, k_ref, n_ref = O.coeffs(wl.species, wl.lines, wl.cells, wl.grid, E_ion=E)
    cc, kk = O.knife_edges(wl.species, wl.lines, wl.cells, wl.grid, E_ion=E)
    ctx = lrt.Context(0).load(wl)
    nb = ctx.sizes()["n_bands"]
    n = sum(ctx.count_terms(b) for b in range(nb))
    say("n_e %g: terms gpu %d oracle %d knife edges %d" % (n_e, n, n_ref, cc.size))
    assert abs(n - n_ref) <= cc.size
    for prec in PRECS:
        we = wk = 0.0
        for b in range(nb):
            eta, kap, esc = ctx.coeffs_torch(b, prec)
            torch.cuda.synchronize()
            e, k = (lrt.scaled_to_f64(eta, kap, esc) if prec == lrt.LRT_FP32_COMP
                    else (eta.cpu().numpy(), kap.cpu().numpy()))
            k0 = b * wl.grid.band_points
            m = np.zeros(e.shape, bool)
            sel = (kk >= k0) & (kk < k0 + e.shape[1])
            m[cc[sel], kk[sel] - k0] = True
            we = max(we, normwise(e, e_ref[:, k0:k0 + e.shape[1]], m))
            wk = max(wk, normwise(k, k_ref[:, k0:k0 + e.shape[1]], m))
        say("  prec %d: eta %.3e kappa %.3e" % (prec, we, wk))
        assert we <= TOL[prec] and wk <= TOL[prec]
    # back to the uniform law
    ctx.set_lorentz(None)
    e_u, _, _ = O.coeffs(wl.species, wl.lines, wl.cells, wl.grid)
    eta, kap, _ = ctx.coeffs_torch(0, lrt.LRT_FP64)
    torch.cuda.synchronize()
    cu, ku = O.knife_edges(wl.species, wl.lines, wl.cells, wl.grid)
    m = np.zeros(eta.shape, bool)
    sel = ku < eta.shape[1]
    m[cu[sel], ku[sel]] = True
    assert normwise(eta.cpu().numpy(), e_u[:, :eta.shape[1]], m) <= 1e-12
    ctx.close()


def test_full_lorentz_solve(torch_dev):
    """Whole path with per-line widths: I_int per ray and the slab flux."""
    wl = stark_workload(5e16)
    ref = O.solve_slab(wl)
    ctx = lrt.Context(0).load(wl)
    for prec in PRECS:
        q, I_int, _ = ctx.solve(prec)
        eI = float(np.max(np.abs(I_int - ref["I_int"]) / np.abs(ref["I_int"])))
        eq = abs(q[0] - ref["q"]) / abs(ref["q"])
        say("full Lorentz solve prec %d: I_int %.3e q %.3e" % (prec, eI, eq))
        assert eI <= TOL[prec] and eq <= TOL[prec]
    ctx.close()


def test_lorentz_arguments(torch_dev):
    wl = stark_workload(1e16)
    ctx = lrt.Context(0)
    with pytest.raises(lrt.LrtError) as e:
        ctx.set_lorentz(wl.lorentz_E_ion)       # no species
    assert e.value.status == 6
    ctx.set_species(wl.species)
    bad = wl.lorentz_E_ion.copy()
    bad[3] = -5.0
    with pytest.raises(lrt.LrtError):
        ctx.set_lorentz(bad)
    ctx.set_lorentz(wl.lorentz_E_ion)
    ctx.close()
