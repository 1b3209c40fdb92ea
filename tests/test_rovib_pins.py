"""Pins of the oracle's rovibronic line generator (oracle/rovib.py; Sec. 2.2.2
vibrational and rotational terms, Hoenl-London tables for Hund's cases (a)
and (b), molecular Einstein coefficient) against what spectroscopy fixes
independently of the generator's own formulas:

  - the Hoenl-London sum rules (the factors of all branches from one level
    add up to 2J + 1), which a mistyped factor of either table breaks;
  - the vibrational spacing in its own closed form;
  - the rotational combination differences of a Sigma-Sigma band (the
    textbook relations that isolate B and D of one state);
  - the case (b) spin-rotation doubling gamma (N + 1/2);
  - the Einstein coefficient against the textbook value
    A = 3.1361891e-7 nu^3 |mu|^2 / (2J_u + 1) * S (nu in cm^-1, mu in debye),
    e a0 = 2.541746 D, and J-independence of a level's total decay;
  - enumeration: line counts, degeneracies, the grid cut.
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import rovib as RV
from paper_2604_11856_amd import synth


def _system(**kw):
    base = dict(species=0, hund=0, Lambda_u=0, Lambda_l=0, Te_u=20000.0, Te_l=0.0, g_u=1.0, g_l=1.0,
                we_u=1500.0, wexe_u=12.0, weye_u=0.05, Be_u=1.7, ae_u=0.02, De_u=6e-6, be_u=2e-8, gamma_u=0.0,
                we_l=2000.0, wexe_l=15.0, weye_l=-0.02, Be_l=1.9, ae_l=0.018, De_l=5.5e-6, be_l=-1e-8,
                gamma_l=0.0, nv_u=3, nv_l=4, J_max=60, Re2=np.full(12, 0.3))
    base.update(kw)
    return synth.BandSystem(**base)


@pytest.mark.parametrize("lu,ll", [(0, 0), (1, 1), (2, 2), (1, 0), (0, 1), (2, 1), (1, 2), (3, 2)])
def test_hund_a_sum_rule(lu, ll):
    """Table for Hund (a): P + Q + R from one upper level J_u = 2 J_u + 1."""
    for J in range(max(lu, ll) + 1, 80):
        tot = sum(float(RV.honl_london_a(b, J, lu, ll)) for b in (RV.P_BRANCH, RV.Q_BRANCH, RV.R_BRANCH))
        assert abs(tot - (2 * J + 1)) <= 1e-12 * (2 * J + 1), (lu, ll, J, tot)
        for b in (RV.P_BRANCH, RV.Q_BRANCH, RV.R_BRANCH):
            assert float(RV.honl_london_a(b, J, lu, ll)) >= 0.0


def test_hund_a_limits():
    """Sigma-Sigma: no Q branch, P = J_u + 1, R = J_u; Pi-Pi Q branch falls as
    Lambda^2 (2J+1)/(J(J+1)); the dLambda = +-1 tables mirror each other
    (upper and lower signs) for Lambda_u = 1 against Lambda_u = 0."""
    assert float(RV.honl_london_a(RV.Q_BRANCH, 7, 0, 0)) == 0.0
    assert float(RV.honl_london_a(RV.P_BRANCH, 7, 0, 0)) == 8.0
    assert float(RV.honl_london_a(RV.R_BRANCH, 7, 0, 0)) == 7.0
    q = float(RV.honl_london_a(RV.Q_BRANCH, 50, 1, 1))
    assert abs(q - 101.0 / 2550.0) <= 1e-15
    # Pi (u) -> Sigma (l), J_u = 1: the R line needs J_l = 0 >= 0 and has (1 + 1)(0 + 1)/2 = 1
    assert float(RV.honl_london_a(RV.R_BRANCH, 1, 1, 0)) == 1.0
    # Sigma (u) -> Pi (l): P = (J + 2)/2, Q = (2J + 1)/2, R = (J - 1)/2
    for J in (1, 5, 40):
        assert float(RV.honl_london_a(RV.P_BRANCH, J, 0, 1)) == pytest.approx((J + 2) / 2, rel=1e-15)
        assert float(RV.honl_london_a(RV.Q_BRANCH, J, 0, 1)) == pytest.approx((2 * J + 1) / 2, rel=1e-15)
        assert float(RV.honl_london_a(RV.R_BRANCH, J, 0, 1)) == pytest.approx((J - 1) / 2, rel=1e-15)


def test_hund_b_sum_rule():
    """Table for Hund (b): P + Q + R into one lower level J_l = 2 J_l + 1,
    Q the weak satellite (2J+1)/(4J(J+1))."""
    for J in np.arange(0.5, 90.0, 1.0):
        tot = sum(float(RV.honl_london_b(b, J)) for b in (RV.P_BRANCH, RV.Q_BRANCH, RV.R_BRANCH))
        assert abs(tot - (2 * J + 1)) <= 1e-12 * (2 * J + 1), (J, tot)
    assert float(RV.honl_london_b(RV.P_BRANCH, 0.5)) == 0.0
    assert float(RV.honl_london_b(RV.Q_BRANCH, 10.5)) == pytest.approx(22.0 / 483.0, rel=1e-15)


def test_vibrational_spacing_closed_form():
    """E_V(v+1) - E_V(v) = w_e - w_e x_e (2x + 1) + w_e y_e (3x^2 + 3x + 1),
    x = v + 1/2, and E_V(0) = w_e/2 - w_e x_e/4 + w_e y_e/8."""
    we, wexe, weye = 2358.5, 14.3, -0.0075
    v = np.arange(0, 40)
    d = RV.vib_term(we, wexe, weye, v + 1) - RV.vib_term(we, wexe, weye, v)
    x = v + 0.5
    np.testing.assert_allclose(d, we - wexe * (2 * x + 1) + weye * (3 * x * x + 3 * x + 1), rtol=1e-12)
    assert float(RV.vib_term(we, wexe, weye, 0)) == pytest.approx(we / 2 - wexe / 4 + weye / 8, rel=1e-15)


def test_sigma_sigma_combination_differences():
    """Hund (a) Sigma-Sigma band: R(J-1) - P(J+1) = (4B'' - 6D'')(J + 1/2) -
    8D''(J + 1/2)^3 (lower state) and R(J) - P(J) the same in B', D' (upper
    state), J = J_l; the band origin from R(0) and P(1)."""
    s = _system(nv_u=1, nv_l=1, Re2=np.array([0.5]))
    d = RV.rovib_lines([s], 1.0, 1e6)
    # order: J_u, then P, R (no Q); key by (J_u, J_l)
    Ju = (d["gu"] / s.g_u - 1) / 2
    Jl = (d["gl"] / s.g_l - 1) / 2
    nu = {(int(a), int(b)): x for a, b, x in zip(Ju, Jl, d["nu0"])}
    Bu, Du = RV.rot_constants(s.Be_u, s.ae_u, s.De_u, s.be_u, 0)
    Bl, Dl = RV.rot_constants(s.Be_l, s.ae_l, s.De_l, s.be_l, 0)
    for J in range(1, 55):
        R_Jm1, P_Jp1 = nu[(J, J - 1)], nu[(J, J + 1)]          # R(J-1): J_u = J; P(J+1): J_u = J
        x = J + 0.5
        assert R_Jm1 - P_Jp1 == pytest.approx((4 * Bl - 6 * Dl) * x - 8 * Dl * x ** 3, rel=1e-10)
        R_J, P_J = nu[(J + 1, J)], nu[(J - 1, J)]
        assert R_J - P_J == pytest.approx((4 * Bu - 6 * Du) * x - 8 * Du * x ** 3, rel=1e-10)


def test_hund_b_spin_doubling():
    """E(N, +1/2) - E(N, -1/2) = gamma (N + 1/2) at the same N."""
    B, D, g = 1.92, 6e-6, 0.0237
    for N in range(0, 60):
        Ep = float(RV.rot_term_b(B, D, g, N + 0.5, 0.5))
        Em = float(RV.rot_term_b(B, D, g, N - 0.5, -0.5))
        assert Ep - Em == pytest.approx(g * (N + 0.5), rel=1e-10, abs=1e-12)


def test_einstein_coefficient_textbook():
    """A = 3.1361891e-7 nu^3 |mu|^2 S / (2J_u + 1) s^-1 with mu in debye and
    nu in cm^-1 (electric-dipole emission), mu = e a0 Re' and e a0 =
    2.5417464 D."""
    for nu, Re2, S, J in ((20000.0, 0.3, 11.0, 5), (3000.0, 1.0, 1.0, 0), (95000.0, 2e-3, 40.5, 40)):
        mu2 = Re2 * 2.5417464 ** 2
        ref = 3.1361891e-7 * nu ** 3 * mu2 * S / (2 * J + 1)
        assert float(RV.einstein_A(nu, Re2, S, J)) == pytest.approx(ref, rel=2e-7)


def test_level_decay_independent_of_rotation():
    """With B and D negligible every line of a band has the band origin's
    wavenumber, and the Hoenl-London sum rule makes the total decay rate of
    each upper level independent of J: sum_branches A = 64 pi^4 nu^3 (e a0)^2
    Re'^2 / (3h), for every J_u and every coupling case."""
    for lu, ll in ((0, 0), (1, 1), (1, 0), (0, 1)):
        s = _system(Lambda_u=lu, Lambda_l=ll, nv_u=1, nv_l=1, Re2=np.array([0.7]), Be_u=1e-9, Be_l=1e-9,
                    ae_u=0.0, ae_l=0.0, De_u=0.0, De_l=0.0, be_u=0.0, be_l=0.0, J_max=40)
        d = RV.rovib_lines([s], 1.0, 1e6)
        Ju = np.round((d["gu"] / s.g_u - 1) / 2).astype(int)
        nu0 = d["nu0"][0]
        A0 = float(RV.einstein_A(nu0, 0.7, 1.0, 0.0))   # S/(2J+1) = 1
        for J in range(max(lu, ll) + 1, 40):
            tot = d["A"][Ju == J].sum()
            assert tot == pytest.approx(A0, rel=1e-6), (lu, ll, J)


def test_enumeration_and_grid_cut():
    """Line counts of one band: Sigma-Sigma Hund (a) has P for J_u = 0..J_max
    and R for J_u = 1..J_max; Pi-Pi adds Q for J_u >= 1 and starts at J >= 1;
    the Hund (b) doublet has 6 lines per lower N (fewer at N = 0); the grid
    cut keeps exactly the lines inside [nu_min, nu_max]; degeneracies are
    g_e (2J + 1)."""
    s = _system(nv_u=1, nv_l=1, Re2=np.array([0.5]), J_max=30)
    assert RV.rovib_lines([s], 1.0, 1e6)["nu0"].size == 31 + 30
    s = _system(Lambda_u=1, Lambda_l=1, nv_u=1, nv_l=1, Re2=np.array([0.5]), J_max=30, g_u=2.0, g_l=2.0)
    d = RV.rovib_lines([s], 1.0, 1e6)
    assert d["nu0"].size == 30 + 30 + 29                 # P: J_u 1..30, Q: 1..30, R: J_u 2..30
    assert np.all(d["gu"] % 2 == 0) and d["gu"].min() == 2 * 3
    s = _system(hund=1, gamma_u=0.02, gamma_l=0.03, nv_u=1, nv_l=1, Re2=np.array([0.5]), J_max=30)
    d = RV.rovib_lines([s], 1.0, 1e6)
    # N_l = 0: only S_l = +1/2 (J_l = 1/2): R and Q (its P would need J_u = -1/2);
    # N_l >= 1, S_l = +1/2: P, Q, R; S_l = -1/2: Q needs N_u = N_l - 1, P needs J_u >= 1/2
    n = 2 + 3 * 30 + sum(3 if N >= 2 else 2 for N in range(1, 31))
    assert d["nu0"].size == n
    full = RV.rovib_lines(synth.air_band_systems(nv=4, J_max=40), 1.0, 1e6)
    cut = RV.rovib_lines(synth.air_band_systems(nv=4, J_max=40), 30000.0, 40000.0)
    inside = (full["nu0"] >= 30000.0) & (full["nu0"] <= 40000.0)
    np.testing.assert_array_equal(cut["nu0"], full["nu0"][inside])
    np.testing.assert_array_equal(cut["A"], full["A"][inside])


def test_rotational_constant_falls_with_vibration():
    """The lower-state combination differences of the (0, 0) and (0, 1) bands
    give B'' of V'' = 0 and 1 (D'' = 0): they differ by alpha_e, the larger
    for V'' = 0 (B_v = B_e - alpha_e (V + 1/2), alpha_e > 0 by convention)."""
    s = _system(nv_u=1, nv_l=2, Re2=np.array([0.5, 0.5]), De_l=0.0, be_l=0.0, J_max=30)
    d = RV.rovib_lines([s], 1.0, 1e6)
    Ju = np.round((d["gu"] / s.g_u - 1) / 2).astype(int)
    Jl = np.round((d["gl"] / s.g_l - 1) / 2).astype(int)
    n_band = d["nu0"].size // 2
    B = []
    for b in range(2):
        sl = slice(b * n_band, (b + 1) * n_band)
        nu = {(a, c): x for a, c, x in zip(Ju[sl], Jl[sl], d["nu0"][sl])}
        J = 10
        B.append((nu[(J, J - 1)] - nu[(J, J + 1)]) / (4 * J + 2))   # R(J-1) - P(J+1) = 4B''(J + 1/2)
    assert B[0] - B[1] == pytest.approx(s.ae_l, rel=1e-9)
    assert B[0] == pytest.approx(s.Be_l - 0.5 * s.ae_l, rel=1e-12)
