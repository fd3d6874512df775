"""Shared helpers for the GPU parity tests: descriptors for both sides, tolerances."""
import numpy as np

from oracle import oracle as O
from paper_2604_09643_amd import workloads as W

# Tolerances of the parity bar (relative L2 against the FP64 oracle).
TOL_SIGNAL = 1e-5
TOL_GRAD = 1e-4


def rel_l2(got, ref) -> float:
    """Relative L2 error; against an all-zero reference, 0 if the result is all zero too, else inf."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    nr = np.linalg.norm(ref)
    if nr == 0.0:
        return 0.0 if np.linalg.norm(got) == 0.0 else float("inf")
    return float(np.linalg.norm(got - ref) / nr)


def oracle_desc(w: W.Workload):
    return O.Grid(*w.shape, w.origin, w.spacing), O.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)


def gpu_desc(w: W.Workload):
    from paper_2604_09643_amd import _lib as L
    return L.Grid(*w.shape, tuple(w.origin), w.spacing), L.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)


def to_gpu(w: W.Workload):
    import torch
    dev = torch.device("cuda:0")
    p0 = torch.tensor(w.p0.astype(np.float32), device=dev).contiguous()
    elem = torch.tensor(w.elem, dtype=torch.float64, device=dev).contiguous()
    poses = torch.tensor(w.poses, dtype=torch.float64, device=dev).contiguous()
    return p0, elem, poses


def announce(msg: str):
    print("[gpu-case] " + msg, flush=True)


def edge_value(kernel, x, w, nu):
    """|phi| and |phi'| bounds at the window edge x = trunc*sigma of a source profile (K(0) = 1)."""
    k = {1: np.exp(-x / w), 2: (1.0 + (x / w) ** 2) ** -nu, 3: 1.0}[kernel]
    dk = {1: abs(1 - x / w), 2: abs(1 - 2 * nu * x * x / (w * w + x * x)), 3: 1.0}[kernel]
    return x * k, dk * k
