"""Writes the fixtures of this directory: the closed-form single-source pressures printed in
Appendix A ("Analytical Solutions for Typical Initial Distributions"), evaluated at sample
times of a 40 MHz record for a source of unit peak 10 mm from the sensor.

Each profile's solution is p(r, t) = [(r + c t) p0(r + c t) + (r - c t) p0(|r - c t|)] / (2 r)
(the spherically symmetric solution of the same appendix); the second term is the outgoing
wave that the far-field model keeps.  Columns: k, t_k [s], p (both terms), p_out (outgoing
term only).  Run from the repository root: python tests/golden/make_golden.py
"""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
C, FS, R, W = 1540.0, 40e6, 10e-3, 0.1e-3
PROFILES = {
    # name: (p0(rho) with p0(0) = 1, half-width of the listed samples in widths, citation)
    "gaussian": (lambda x: np.exp(-x * x / (2 * W * W)), 8.0,
                 "Appendix A, Gaussian distribution (the kernel of Eq. (A13)), p_c = 1, sigma = w"),
    "exponential": (lambda x: np.exp(-x / W), 14.0, "Appendix A, exponential distribution, p_c = 1, a = w"),
    "power_nu2": (lambda x: (1.0 + (x / W) ** 2) ** -2.0, 14.0,
                  "Appendix A, power-law distribution, nu = 2, A = a^(2 nu) (peak 1), a = w"),
    "uniform": (lambda x: (x <= W).astype(float), 1.5, "Appendix A, uniform spherical source, p_0 = 1, a_0 = w"),
}


def main():
    k0 = int(round(R / C * FS))
    for name, (prof, half, cite) in PROFILES.items():
        n = int(np.ceil(half * W / (C / FS)))
        k = np.arange(k0 - n, k0 + n + 1)
        t = k / FS
        ct = C * t
        out = (R - ct) * prof(np.abs(R - ct)) / (2 * R)
        inward = (R + ct) * prof(R + ct) / (2 * R)
        path = os.path.join(HERE, "point_source_%s.txt" % name)
        with open(path, "w") as f:
            f.write("# %s\n" % cite)
            f.write("# c = %.1f m/s, fs = %.0f Hz, r = %.4g m, width w = %.4g m\n" % (C, FS, R, W))
            f.write("# columns: k  t_k[s]  p(r,t_k) (both terms)  p_out (outgoing term)\n")
            for kk, tt, pf, po in zip(k, t, out + inward, out):
                f.write("%d %.17g %.17g %.17g\n" % (kk, tt, pf, po))


if __name__ == "__main__":
    main()
