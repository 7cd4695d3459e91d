"""Values the paper prints, stored as small cited text fixtures under
tests/golden/, checked against the oracle."""
import os

import numpy as np

import workloads
from oracle import forcing
from oracle.grid import Grid
from oracle.step import SCHEMES

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_time_scheme_coefficients():
    for scheme, s, gamma, rho, alpha in _rows("time_schemes.txt"):
        g_, r_ = SCHEMES[scheme][int(s) - 1]
        assert (g_, r_) == (float(gamma), float(rho))
        assert g_ + r_ == float(alpha)


def test_uniform_grid_probe_length():
    (delta, ratio), = _rows("probe_length.txt")
    n = 8
    L = float(delta) * n
    g = Grid(n, n, n, L, L, workloads.uniform_faces(n, -L / 2, L / 2))
    for c in range(3):
        assert np.isclose(forcing.probe_length(g, c, 3) / float(delta), float(ratio),
                          rtol=1e-15)
