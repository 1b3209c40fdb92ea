"""Error metrics shared by the GPU parity tests (not a test module).

normwise(): max over rows (cells or rays) of max|got - ref| / max|ref|, the
bar of every eta / kappa / I comparison.  Each call also prints, for
information, the pointwise relative error over the points whose reference is
at least 1e-3 of its row's maximum, and enforces the cap on the knife-edge
exclusion: the points a mask drops (window bounds within 1e-9 grid steps of
an integer index, flagged by the oracle) may be at most MASK_FRACTION_MAX of
the points compared.
"""
import numpy as np

import oracle as O

MASK_FRACTION_MAX = 1e-5


def say(*a):
    print(*a, flush=True)


def pointwise(got, ref, mask=None, floor=1e-3):
    """max |got - ref| / |ref| over points with |ref| >= floor * max|ref| of
    their row (masked points left out)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    big = np.abs(ref) >= floor * np.max(np.abs(ref), axis=-1, keepdims=True)
    big &= np.abs(ref) > 0
    if mask is not None:
        big &= ~mask
    if not np.any(big):
        return 0.0
    return float(np.max(np.abs(got - ref)[big] / np.abs(ref)[big]))


def normwise(got, ref, mask=None, label=""):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    d = np.abs(got - ref)
    n_masked = 0
    if mask is not None:
        mask = np.broadcast_to(mask, d.shape)
        n_masked = int(mask.sum())
        assert n_masked <= MASK_FRACTION_MAX * d.size, \
            "knife-edge exclusion drops %d of %d points" % (n_masked, d.size)
        d = np.where(mask, 0.0, d)
    den = np.max(np.abs(ref), axis=-1)
    num = np.max(d, axis=-1)
    zero = den == 0
    assert np.all(num[zero] == 0), "nonzero values where the oracle has none"
    e = float(np.max(num[~zero] / den[~zero])) if np.any(~zero) else 0.0
    say("    %snormwise %.3e  pointwise(|ref| >= 1e-3 max) %.3e  knife-edge points dropped %d of %d"
        % (label + " " if label else "", e, pointwise(got, ref, mask), n_masked, d.size))
    return e


def edge_mask(wl, k_first, n, cells=None, E_ion=None):
    """[n_cells, n] mask of the knife-edge points of grid indices
    k_first..k_first+n-1."""
    cells = wl.cells if cells is None else cells
    cc, kk = O.knife_edges(wl.species, wl.lines, cells, wl.grid, E_ion=E_ion)
    m = np.zeros((cells.n, n), bool)
    sel = (kk >= k_first) & (kk < k_first + n)
    m[cc[sel], kk[sel] - k_first] = True
    return m


def knife_mask(wl, cells, ks, E_ion=None, reach=1000.0):
    """[n_cells, ks.size] mask of the knife-edge points among sampled grid
    indices ks (sorted); reach bounds 100 Voigt HWHM in cm^-1."""
    cc, kk = O.knife_edges(wl.species, wl.lines, cells, wl.grid, near=ks, E_ion=E_ion, reach=reach)
    pos = {int(k): j for j, k in enumerate(ks)}
    m = np.zeros((cells.n, ks.size), bool)
    for c, k in zip(cc, kk):
        if int(k) in pos:
            m[c, pos[int(k)]] = True
    return m
