"""Printed data of the paper against the generators that feed the oracle and
the library (CPU).  Each fixture under tests/golden/ states the passage it is
taken from."""
import os

import numpy as np

from paper_2604_11856_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    out = {}
    for ln in open(os.path.join(GOLDEN, name)):
        ln = ln.strip()
        if not ln or ln.startswith("#"):
            continue
        f = ln.split()
        out[f[0]] = np.array([float(x) for x in f[1:]], np.float64)
    return out


def test_free_free_fit_matches_the_printed_table():
    """The free-free coefficients the continuum records carry are the printed
    table, digit for digit, for both atoms."""
    table = _rows("free_free_fit_N_O.txt")
    assert sorted(table) == ["N", "O"]
    for atom, c in table.items():
        assert c.shape == (8,)
        assert np.array_equal(np.array(synth.PEACH_FF[atom], np.float64), c), atom


def test_free_free_fit_reaches_the_continuum_records():
    """air_continuum hands exactly those coefficients to the N and O records."""
    table = _rows("free_free_fit_N_O.txt")
    sp = synth.stagnation_line(n_cells=4, n_atomic=64, n_rovib=0, n_points=4096, n_mu=0).species
    recs = synth.air_continuum(sp)
    names = {r.species: sp[r.species].name for r in recs}
    assert sorted(names.values()) == ["N", "O"]
    for r in recs:
        assert np.array_equal(np.asarray(r.peach, np.float64), table[names[r.species]])
