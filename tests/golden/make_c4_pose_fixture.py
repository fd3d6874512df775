"""Writes c4_subarray_pose.txt: the oracle's element gradients and rigid-pose gradient of one
frame of the 256^3 matrix-array configuration, for a 16 x 8 block of the 32 x 32 array.

The model is Eq. (1) with the kernel of Eq. (A13); the element gradient is dL/dx_e for a
given dL/ds = r, and the pose gradient is its Stage 4 rigid chain (dL/dR = sum_m g_e e_m^T,
dL/dt = sum_m g_e).  Every voxel of the 256^3 volume contributes to every element, so the
pose gradient sums about 16.7 million terms per element, the reduction that the GPU path
carries out in FP64.  The oracle needs a few minutes for it, too long for a test, so its
values are stored here.  Only the seeded input generators and the oracle are called.

Run from the repository root: python tests/golden/make_c4_pose_fixture.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O                   # noqa: E402
from paper_2604_09643_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "c4_subarray_pose.txt")
FRAME = 0
R_SEED = 17


def subarray():
    """Element indices m = 32 i + j of the block i in [8, 24), j in [12, 20) of the 32 x 32 array."""
    return np.array([32 * i + j for i in range(8, 24) for j in range(12, 20)])


def inputs():
    """(workload, element template of the block, pose of the frame, residual r [1, 128, K])."""
    w = W.c4()
    elem = np.ascontiguousarray(w.elem[subarray()])
    poses = np.ascontiguousarray(w.poses[FRAME:FRAME + 1])
    r = np.random.default_rng(R_SEED).normal(size=(1, elem.shape[0], w.K)).astype(np.float32)
    return w, elem, poses, r


def main():
    w, elem, poses, r = inputs()
    og = O.Grid(*w.shape, w.origin, w.spacing)
    os_ = O.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)
    p0 = w.p0.astype(np.float32).astype(np.float64)
    ge = O.grid_adjoint_elem(og, p0, poses, elem, os_, r.astype(np.float64))
    gp = O.pose_grad(elem, ge)
    with open(OUT, "w") as f:
        f.write("# oracle dL/dx_e and (dL/dR, dL/dt) of frame %d of the 256^3 / 32x32 matrix-array "
                "configuration,\n" % FRAME)
        f.write("# elements m = 32 i + j, i in [8, 24), j in [12, 20) (128 elements, in that order); "
                "dL/ds = r ~ N(0, 1) float32, numpy default_rng(%d), shape [1, 128, K]\n" % R_SEED)
        f.write("# Eq. (1) with the kernel of Eq. (A13); rigid chain of Stage 4.  "
                "Written by tests/golden/make_c4_pose_fixture.py (oracle only).\n")
        f.write("# first 128 lines: g_e (x, y, z); last line: dL/dR row-major (9), dL/dt (3)\n")
        for row in ge[0]:
            f.write("%.17e %.17e %.17e\n" % tuple(row))
        f.write(" ".join("%.17e" % v for v in gp[0]) + "\n")


def load():
    """(g_e [128, 3], grad_pose [12]) from the fixture."""
    a = [list(map(float, ln.split())) for ln in open(OUT) if not ln.startswith("#")]
    return np.array(a[:-1]), np.array(a[-1])


if __name__ == "__main__":
    main()
