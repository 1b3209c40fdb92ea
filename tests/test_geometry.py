"""Host-side ray traversal of the library against the oracle's sorted-crossing
construction (no GPU): total path, path per cell and cell order, including
wall points on radial faces, exact x-plane / r-face ties and tangencies."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2604_11856_amd import lrt, synth


def _compare(geom, rw, mu, phi):
    c1, d1 = lrt.trace_axi_ray(geom.nx, geom.nr, geom.Lx, geom.R, rw, mu, phi)
    c2, d2 = O.axi_ray(geom, rw, mu, phi)
    tol = 1e-7 * geom.R   # near-tangent chords are conditioned like sqrt(eps) r
    assert d1.sum() == pytest.approx(d2.sum(), rel=1e-13)
    n = geom.nx * geom.nr
    np.testing.assert_allclose(np.bincount(c1, d1, n), np.bincount(c2, d2, n), rtol=1e-10, atol=2 * tol)

    def seq(cs, dd):
        out = []
        for c, d in zip(cs, dd):
            if d > tol and (not out or out[-1] != c):
                out.append(int(c))
        return out
    assert seq(c1, d1) == seq(c2, d2)


def test_traversal_faces_ties_tangencies():
    rng = np.random.default_rng(0)
    geom = synth.AxiGeometry(64, 32, 10.0, 8.0, np.concatenate([np.arange(32) * 0.25,
                                                                rng.uniform(0, 7.99, 12)]), 7, 6)
    mus = list(O.gauss_legendre_01(7)[0]) + [0.5, 0.8, 0.6, 1 / math.sqrt(2), 0.999999, 1.0]
    phis = list(rng.uniform(0, 2 * math.pi, 6)) + [(j + 0.5) * math.pi / 3 for j in range(6)] + \
        [0.0, math.pi / 2, math.pi, 3 * math.pi / 2]
    for rw in geom.wall_r:
        for mu in mus:
            for phi in phis:
                _compare(geom, float(rw), mu, phi)


def test_traversal_axisymmetric_workload_rays():
    g = synth.AxiGeometry(256, 128, 100.0, 50.0, (np.arange(64) + 0.5) * 30.0 / 64, 16, 16)
    mu, _ = O.gauss_legendre_01(16)
    for rw in g.wall_r[::7]:
        for m in mu[::3]:
            for j in range(8):
                _compare(g, float(rw), float(m), (j + 0.5) * 2 * math.pi / 16)


def test_trace_rejects_bad_arguments():
    with pytest.raises(lrt.LrtError):
        lrt.trace_axi_ray(4, 4, 1.0, 1.0, 2.0, 0.5, 0.0)     # rw outside [0, R)
    with pytest.raises(lrt.LrtError):
        lrt.trace_axi_ray(4, 4, 1.0, 1.0, 0.5, 0.0, 0.0)     # mu = 0 never leaves the wall


def test_fibonacci_rule_matches_oracle():
    """The library's Fibonacci LOS directions and flux weights (host-only
    entry point) equal the oracle's, written independently from the same
    passage."""
    for n, p, a in ((400, 20, 40), (100, 8, 16), (1600, 32, 64), (7, 3, 5), (61, 6, 12)):
        d1, w1 = lrt.fibonacci_quadrature(n, p, a)
        d0, w0 = O.fibonacci_quadrature(n, p, a)
        assert d1.shape == d0.shape
        np.testing.assert_allclose(d1, d0, rtol=0, atol=1e-15)
        np.testing.assert_allclose(w1, w0, rtol=1e-14, atol=0)


@pytest.mark.parametrize("R,nr", [(0.3, 20), (0.7, 10), (50.0 / 3.0, 30), (1.0, 7)])
def test_traversal_wall_points_on_faces_non_dyadic(R, nr):
    """Wall points at k R / nr on grids whose radial step is not a power of
    two: the start cell must agree with the face products (r_k = k dr), or an
    outward ray misses its first face.  Checked against the oracle's sorted
    crossings for every face, polar node and azimuth.  (A ray along the wall
    normal from a face point runs on the face itself, where either adjacent
    cell is correct; it is checked for its length only.)"""
    g = synth.AxiGeometry(16, nr, 1.0, R, np.arange(nr) * R / nr, 4, 4)
    mus = list(O.gauss_legendre_01(5)[0]) + [0.3, 0.95]
    phis = [0.2, 1.3, 2.9, math.pi, 4.0, 5.5, 0.0, math.pi / 2]
    for rw in g.wall_r:
        for mu in mus:
            for phi in phis:
                _compare(g, float(rw), float(mu), phi)
        c1, d1 = lrt.trace_axi_ray(g.nx, g.nr, g.Lx, g.R, float(rw), 1.0, 0.0)
        assert d1.sum() == pytest.approx(g.Lx, rel=1e-14) and np.all(np.diff(c1 // nr) == -1)
