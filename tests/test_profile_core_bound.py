"""The single-precision accumulation evaluates the two exponential terms of the
Whiting profile (Sec. 2.2.1) only within 12 gamma_V of a line centre
(x = |dnu| / (2 gamma_V) <= 6).  Beyond it the oracle's full profile must
equal its rational part to within 2^-30 relative, for every Lorentz fraction
r = gamma_L / gamma_V the kernel stages (r >= 2^-40) and up to the window's
edge at 100 gamma_V.  CPU only: the oracle against the profile with its
exponential terms taken out."""
import numpy as np
import pytest

import oracle as O

CORE_X = 6.0


def rational_part(delta, gV, gL):
    r = gL / gV
    x = abs(delta) / (2.0 * gV)
    x225 = x ** 2.25
    shape = r / (1.0 + 4.0 * x * x) - 0.016 * r * (1.0 - r) / (1.0 + 0.1 * x225)
    return shape / (2.0 * gV * (1.065 + 0.447 * r + 0.058 * r * r))


@pytest.mark.parametrize("r", [2.0 ** -40, 1e-9, 1e-4, 0.01, 0.3, 0.7, 0.99, 1.0 - 1e-9])
def test_exponentials_negligible_beyond_core(r):
    gV = 0.37
    gL = r * gV
    worst = 0.0
    for x in np.concatenate([np.linspace(CORE_X, 8.0, 41), np.linspace(8.0, 50.0, 43)]):
        delta = 2.0 * x * gV
        for d in (delta, -delta):
            full = O.voigt_profile(d, gV, gL)
            rat = rational_part(d, gV, gL)
            assert rat > 0.0
            worst = max(worst, abs(full - rat) / rat)
    assert worst <= 2.0 ** -30, worst


def test_exponentials_matter_inside_core():
    """The bound is not slack by orders of magnitude: at x = 5 the second
    exponential term is still above single-precision rounding of the term for a
    line with equal Lorentz and Gaussian shares."""
    gV, r = 0.37, 0.5
    d = 2.0 * 5.0 * gV
    rel = abs(O.voigt_profile(d, gV, r * gV) - rational_part(d, gV, r * gV)) / rational_part(d, gV, r * gV)
    assert rel > 2.0 ** -24
