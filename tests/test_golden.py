"""The oracle's single-source signals against the closed-form solutions printed in Appendix A,
stored under tests/golden/ (written by tests/golden/make_golden.py from those formulas)."""
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
# fixture: (kernel, trunc, nu) of the model that stands for it
CASES = {"gaussian": (0, 6.0, 1.0), "exponential": (1, 12.0, 1.0), "power_nu2": (2, 12.0, 2.0),
         "uniform": (3, 1.0, 1.0)}


def load(name):
    path = os.path.join(GOLDEN, "point_source_%s.txt" % name)
    head = [l for l in open(path) if l.startswith("#")]
    vals = dict(kv.split(" = ") for kv in head[1][2:].strip().split(", "))
    c = float(vals["c"].split()[0])
    fs = float(vals["fs"].split()[0])
    r = float(vals["r"].split()[0])
    w = float(vals["width w"].split()[0])
    rows = np.loadtxt(path, comments="#")
    return c, fs, r, w, rows[:, 0].astype(int), rows[:, 2], rows[:, 3]


@pytest.mark.parametrize("name", list(CASES))
def test_point_source_matches_closed_form(name):
    """One voxel of unit value at the origin seen from 10 mm: inside the window the model
    equals the outgoing term of the closed-form pressure to rounding; outside it is zero; and
    it differs from the full solution by the inward term, which the far-field form drops, and
    by what the window cuts off."""
    kernel, trunc, nu = CASES[name]
    c, fs, r, w, k, p_full, p_out = load(name)
    grid = O.Grid(1, 1, 1, (0.0, 0.0, 0.0), 1e-4)
    poses = np.array([[1.0, 0, 0, 0, 1.0, 0, 0, 0, 1.0, 0, 0, 0]])
    elem = np.array([[0.0, 0.0, r]])
    samp = O.Sampling(c, fs, int(k.max()) + 1, w, trunc, kernel, nu)
    s = O.grid_forward(grid, np.ones((1, 1, 1)), poses, elem, samp)[0, 0][k]
    inside = np.abs(r - c * k / fs) <= trunc * w
    assert inside.sum() >= 5
    peak = np.abs(p_out).max()
    np.testing.assert_allclose(s[inside], p_out[inside], rtol=1e-12, atol=1e-15 * peak)
    assert np.all(s[~inside] == 0.0)
    cut = np.abs(p_out[~inside]).max() if (~inside).any() else 0.0
    assert np.abs(s - p_full).max() <= np.abs(p_full - p_out).max() + cut + 1e-15 * peak
