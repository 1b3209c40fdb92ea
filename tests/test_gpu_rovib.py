"""Rovibronic line generation on the device (lrt_gen_rovib_lines, Sec. 2.2.2)
against the oracle's generator (oracle/rovib.py), through the C ABI:

  - the line list of the four air band systems at the size of the
    stagnation-line configuration (about 2M lines): the same lines in the same
    order, nu0 / A / energies within 1e-12 relative, degeneracies and species
    exact;
  - counting, capacity and argument errors;
  - the whole path run from generated lines (atomic lines from the host,
    molecular lines generated on the device, the list set from device
    memory): intensities and flux against the oracle run from its own
    generated lines (FP64 1e-12, FP32-comp 1e-5).
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from oracle import rovib as RV
from paper_2604_11856_amd import lrt, synth
from parity_util import say

pytestmark = pytest.mark.gpu

FIELDS = ("nu0", "A", "Eu_ev", "Eu_rot", "El_ev", "El_rot", "gu", "gl")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch


def _ctx_with_species():
    rng = np.random.Generator(np.random.PCG64(11857))
    species = synth._air_species(rng, 8)
    ctx = lrt.Context(0)
    ctx.set_species(species)
    return ctx, species


def _compare(gpu, ref):
    n = ref["nu0"].size
    assert gpu["nu0"].shape[0] == n, (gpu["nu0"].shape[0], n)
    for k in FIELDS:
        g = gpu[k].cpu().numpy()
        r = ref[k]
        scale = np.maximum(np.abs(r), 1.0 if k.startswith("E") else 0.0)
        err = float(np.max(np.abs(g - r) / np.where(scale > 0, scale, 1.0))) if n else 0.0
        say("    %-6s max rel err %.3e" % (k, err))
        assert err <= 1e-12, k
    assert np.array_equal(gpu["species"].cpu().numpy(), ref["species"])
    assert np.array_equal(gpu["gu"].cpu().numpy(), ref["gu"]) and np.array_equal(gpu["gl"].cpu().numpy(), ref["gl"])


def test_generated_lines_match_oracle_full_size(torch_dev):
    """Four band systems (Pi-Pi and Sigma-Sigma in Hund's case (a), Sigma-Pi
    with dLambda = -1, a doublet Sigma-Sigma in case (b)), 30 x 30 bands each,
    J up to 150, over 1000-100000 cm^-1."""
    ctx, species = _ctx_with_species()
    sy = synth.air_band_systems(nv=30, J_max=150)
    lo, hi = 1000.0, 100000.0
    ref = RV.rovib_lines(sy, lo, hi)
    # no line within 1e-9 of the window ends (else one rounding could flip it)
    assert np.all(np.abs(ref["nu0"] - lo) > 1e-9 * lo) and np.all(np.abs(ref["nu0"] - hi) > 1e-9 * hi)
    gpu = ctx.gen_rovib_lines(sy, lo, hi)
    say("generated %d lines (oracle %d)" % (gpu["nu0"].shape[0], ref["nu0"].size))
    assert ref["nu0"].size > 1_500_000
    _compare(gpu, ref)
    # a narrow window: the same lines as the oracle's cut
    ref2 = RV.rovib_lines(sy, 31000.0, 33000.0)
    _compare(ctx.gen_rovib_lines(sy, 31000.0, 33000.0), ref2)
    ctx.close()


def test_generator_edge_cases(torch_dev):
    torch = torch_dev
    ctx, species = _ctx_with_species()
    sy = synth.air_band_systems(nv=3, J_max=20)
    n = ctx.gen_rovib_lines(sy, 1000.0, 100000.0)["nu0"].shape[0]
    assert n == RV.rovib_lines(sy, 1000.0, 100000.0)["nu0"].size
    # an empty window
    assert ctx.gen_rovib_lines(sy, 500.0, 600.0)["nu0"].shape[0] == 0
    # capacity below the count: error, count reported
    import ctypes as C
    arr = (lrt._BandSystem * 1)()
    b = sy[0]
    re2 = np.ascontiguousarray(b.Re2, np.float64)
    vals = [float(getattr(b, k)) for k in ("Te_u", "Te_l", "g_u", "g_l", "we_u", "wexe_u", "weye_u", "Be_u",
                                           "ae_u", "De_u", "be_u", "gamma_u", "we_l", "wexe_l", "weye_l", "Be_l",
                                           "ae_l", "De_l", "be_l", "gamma_l")]
    arr[0] = lrt._BandSystem(b.species, b.hund, b.Lambda_u, b.Lambda_l, *vals, b.nv_u, b.nv_l, b.J_max,
                             re2.ctypes.data_as(C.POINTER(C.c_double)))
    out = {k: torch.empty(4, dtype=torch.float64, device="cuda:0") for k in FIELDS}
    sp = torch.empty(4, dtype=torch.int32, device="cuda:0")
    bufs = lrt._LineBuffers(*[C.cast(C.c_void_p(out[k].data_ptr()), C.POINTER(C.c_double)) for k in FIELDS],
                            C.cast(C.c_void_p(sp.data_ptr()), C.POINTER(C.c_int32)))
    cnt = C.c_int64()
    s = lrt.lib().lrt_gen_rovib_lines(ctx.h, 1, arr, 1000.0, 100000.0, 4, C.byref(bufs), C.byref(cnt), None)
    assert s == 1 and cnt.value > 4
    # invalid systems
    for kw in (dict(species=synth.AIR11.index("N")), dict(Lambda_u=3, Lambda_l=1), dict(nv_u=0),
               dict(hund=1, Lambda_u=1, Lambda_l=1), dict(Re2=-np.abs(b.Re2)), dict(g_u=0.5), dict(hund=7)):
        bad = dataclasses.replace(b, **kw)
        with pytest.raises((lrt.LrtError, ValueError)):
            ctx.gen_rovib_lines([bad], 1000.0, 100000.0)
    with pytest.raises(lrt.LrtError):
        ctx.gen_rovib_lines(sy, 2000.0, 1000.0)
    ctx.close()


def _stagnation_with(species, lines, seed=23):
    base = synth.stagnation_line(n_cells=40, n_atomic=2000, n_rovib=0, n_points=30000, band_points=12000,
                                 n_mu=3, n_v=8, seed=seed)
    return synth.Workload("stagnation-generated", species, lines, base.cells, base.grid, base.geometry)


def test_solve_from_generated_lines(torch_dev):
    """The whole path on a 40-cell stagnation line whose molecular lines are
    generated on the device and handed to the context from device memory,
    against the oracle run on its own generated lines."""
    torch = torch_dev
    base = synth.stagnation_line(n_cells=40, n_atomic=2000, n_rovib=0, n_points=30000, band_points=12000,
                                 n_mu=3, n_v=8, seed=23)
    sy = synth.air_band_systems(nv=8, J_max=80)
    lo, hi = base.grid.nu_min, base.grid.nu_max
    # the oracle's workload: host atomic lines + the oracle's generated lines
    ref_mol = RV.rovib_lines(sy, lo, hi)
    at = base.lines
    parts = [{k: np.asarray(getattr(at, k)) for k in FIELDS + ("species",)}, ref_mol]
    wl = synth.Workload("stagnation-generated", base.species, synth.merge_sorted(parts), base.cells, base.grid,
                        base.geometry)
    ref = O.solve_slab(wl)
    # the library: the atomic lines uploaded from the host into device tensors,
    # the molecular lines generated on the device, one device list
    ctx = lrt.Context(0)
    ctx.set_species(base.species)
    gen = ctx.gen_rovib_lines(sy, lo, hi)
    dev = {k: torch.cat([torch.as_tensor(np.asarray(getattr(at, k), np.float64), device="cuda:0"), gen[k]])
           for k in FIELDS}
    dev["species"] = torch.cat([torch.as_tensor(np.asarray(at.species, np.int32), device="cuda:0"), gen["species"]])
    ctx.set_lines_device(dev)
    ctx.set_grid(base.grid)
    ctx.set_cells(base.cells)
    ctx.set_rays(base.geometry)
    say("solve from generated lines: %d atomic + %d molecular" % (at.n, gen["nu0"].shape[0]))
    for prec, tol in ((lrt.LRT_FP64, 1e-12), (lrt.LRT_FP32_COMP, 1e-5)):
        q, I_int, _ = ctx.solve(prec)
        eI = float(np.max(np.abs(I_int - ref["I_int"]) / np.abs(ref["I_int"])))
        eq = abs(q[0] - ref["q"]) / abs(ref["q"])
        say("  prec %d: I_int %.3e  q %.3e" % (prec, eI, eq))
        assert eI <= tol and eq <= tol
    ctx.close()
