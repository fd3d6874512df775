"""The moment form of the Gaussian dL/dp0 adjoint, checked on the CPU.

The GPU kernel replaces the window sum of one (voxel, element) pair by a Taylor expansion about
the pair's nearest sample: with d = (kc + x) delta, |x| <= 1/2 and Delta = delta / sigma,

    phi((x - j) delta) = sigma psi((x - j) Delta) ~ sum_{n < 8} x^n D_n(j),
    D_n(j) = -sigma Delta^n He_{n+1}(j Delta) exp(-(j Delta)^2 / 2) / n!,

and admits the form only where 1.791 (Delta/2)^8 sqrt(9 / 8!) <= 1e-6 of the kernel's peak.
These tests evaluate the expansion with numpy's own Hermite series (not the kernel's recurrence),
check the error bound the kernel relies on, and bound the terms the whole-row window adds.
"""
import math

import numpy as np
from numpy.polynomial import hermite_e as He

NMOM = 8
C, FS = 1540.0, 40e6
DELTA = C / FS


def psi(y):
    return y * np.exp(-0.5 * y * y)


def coef(n, j, dd):
    """D_n(j) / sigma from the probabilists' Hermite series of numpy."""
    c = np.zeros(n + 2)
    c[n + 1] = 1.0
    y = j * dd
    return -(dd ** n) * He.hermeval(y, c) * np.exp(-0.5 * y * y) / math.factorial(n)


def bound(dd):
    return 1.791 * (0.5 * dd) ** NMOM * math.sqrt((NMOM + 1) / math.factorial(NMOM))


def largest_admitted_ratio():
    lo, hi = 0.1, 2.0                       # bound() is increasing in delta / sigma
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if bound(mid) <= 1e-6 else (lo, mid)
    return lo


def expansion_error(dd, jt):
    x = np.linspace(-0.5, 0.5, 2001)
    peak = psi(1.0)
    worst = 0.0
    for j in range(-jt, jt + 1):
        approx = sum(x ** n * coef(n, j, dd) for n in range(NMOM))
        worst = max(worst, np.max(np.abs(approx - psi((x - j) * dd))) / peak)
    return worst


def test_expansion_matches_kernel_and_meets_bound():
    """Sweep (C1, sigma 0.1 mm), freehand sweep (sigma 0.08 mm) and the largest admitted
    delta/sigma: the 8-term expansion stays within the bound the host checks.  A sign slip in
    D_n, a wrong Hermite index or a missing 1/n! breaks the first assertion by orders of
    magnitude."""
    for sigma in (1e-4, 8e-5, DELTA / largest_admitted_ratio()):
        dd = DELTA / sigma
        jt = int(math.floor(6.0 / dd + 0.5))
        err = expansion_error(dd, jt)
        assert err <= bound(dd), (sigma, err, bound(dd))
        assert bound(dd) <= 1e-6 * (1 + 1e-9)


def test_bound_is_not_loose_by_orders():
    """The bound is a real bound and not vacuous: at the freehand sweep's sigma the observed error
    is within two orders of it."""
    dd = DELTA / 8e-5
    err = expansion_error(dd, 12)
    assert bound(dd) / 100 <= err <= bound(dd)


def test_whole_rows_add_only_edge_terms():
    """Rows |j| <= JT about the nearest sample hold every term of the 6 sigma window, and the
    terms they add beyond it are below psi(6) of the peak (1.5e-7)."""
    for sigma in (1e-4, 8e-5):
        dd = DELTA / sigma
        jt = int(math.floor(6.0 / dd + 0.5))
        x = np.linspace(-0.5, 0.5, 4001)
        # every in-window offset is a whole row
        for j in range(-jt - 3, jt + 4):
            inside = np.abs((x - j) * dd) <= 6.0
            if abs(j) > jt:
                assert not inside.any()
        # the extra terms of the whole rows
        extra = 0.0
        for j in (-jt, jt):
            u = np.abs((x - j) * dd)
            out = u > 6.0
            if out.any():
                extra = max(extra, np.max(np.abs(psi(u[out]))))
        assert extra / psi(1.0) <= psi(6.0) / psi(1.0) + 1e-15
        assert psi(6.0) / psi(1.0) < 1.6e-7
