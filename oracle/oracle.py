"""FP64 CPU oracle of the PA-SFM differentiable acoustic radiation model.

TEST INFRASTRUCTURE ONLY.  The product library never imports this module; only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
use it.  It wraps ``radiate_oracle.c`` (plain C, double precision) through
ctypes and adds the voxel-grid bookkeeping that the C code leaves to callers.

Every function states the passage of the paper it follows; the C source holds
the arithmetic.  Conventions (readings of what the paper leaves open):

* voxel (i, j, k) sits at ``origin + (i, j, k) * spacing`` and the volume is
  stored C-order ``[nx][ny][nz]`` (z fastest);
* sample k is taken at ``t_k = k / fs`` for ``k = 0..K-1``;
* a term is kept iff ``|d - c t_k| <= trunc * sigma`` (inclusive);
* a posed array has element coordinates ``R e_m + t`` (Stage 4), poses are
  ``[F][12]`` = R row-major then t.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "radiate_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle into ``oracle/_liboracle.so`` (gcc, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        D = ctypes.POINTER(ctypes.c_double)
        L, I, F64 = ctypes.c_long, ctypes.c_int, ctypes.c_double
        lib.or_num_threads.restype = I
        lib.or_set_threads.argtypes = [I]
        lib.or_set_threads.restype = None
        lib.or_element_positions.argtypes = [I, D, I, D, D]
        for name in ("or_forward", "or_forward_dense"):
            getattr(lib, name).argtypes = [L, D, D, L, D, F64, F64, I, F64, F64, I, F64, D]
        lib.or_adjoint_amp.argtypes = [L, D, L, D, F64, F64, I, F64, F64, I, F64, D, D]
        lib.or_adjoint_elem.argtypes = [L, D, D, L, D, F64, F64, I, F64, F64, I, F64, D, D]
        lib.or_count_updates.argtypes = [L, D, L, D, F64, F64, I, F64, F64, I, F64]
        lib.or_count_updates.restype = ctypes.c_longlong
        lib.or_loss_residual.argtypes = [L, D, D, D]
        lib.or_loss_residual.restype = F64
        lib.or_pose_grad.argtypes = [I, I, D, D, D]
        lib.or_rodrigues.argtypes = [D, D]
        lib.or_rodrigues_vjp.argtypes = [D, D, D]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def num_threads() -> int:
    return _load().or_num_threads()


def set_threads(n: int):
    """Thread count of the oracle's parallel loops (timing only; results do not depend on it)."""
    _load().or_set_threads(int(n))


@dataclass(frozen=True)
class Sampling:
    """Acquisition: speed of sound c [m/s], rate fs [Hz], K samples, kernel width sigma [m],
    truncation at trunc*sigma; kernel: 0 Gaussian (Eq. (A13)), 1 exponential, 2 power law
    with exponent nu, 3 uniform sphere (the source profiles of Appendix A, normalised to
    K(0) = 1 with width sigma)."""
    c: float
    fs: float
    K: int
    sigma: float
    trunc: float = 6.0
    kernel: int = 0
    nu: float = 1.0

    def args(self):
        return (float(self.c), float(self.fs), int(self.K), float(self.sigma), float(self.trunc),
                int(self.kernel), float(self.nu))


# ----------------------------------------------------------------------------------------------
# point-source form of the model (sources at arbitrary positions)
# ----------------------------------------------------------------------------------------------

def forward(src, amp, xe, samp: Sampling, dense: bool = False) -> np.ndarray:
    """Eq. (1) with the far-field Gaussian kernel of Eq. (A13): s[e, k] for sources ``src`` [N,3]
    of amplitude ``amp`` [N] seen by elements ``xe`` [E,3].  ``dense`` visits every sample."""
    src, amp, xe = _f64(src).reshape(-1, 3), _f64(amp).reshape(-1), _f64(xe).reshape(-1, 3)
    s = np.zeros((xe.shape[0], samp.K))
    fn = _load().or_forward_dense if dense else _load().or_forward
    fn(src.shape[0], _p(src), _p(amp), xe.shape[0], _p(xe), *samp.args(), _p(s))
    return s


def adjoint_amp(src, xe, samp: Sampling, r) -> np.ndarray:
    """Back-projection A^T r: gradient of <s, r> with respect to each source amplitude."""
    src, xe, r = _f64(src).reshape(-1, 3), _f64(xe).reshape(-1, 3), _f64(r)
    assert r.shape == (xe.shape[0], samp.K)
    g = np.zeros(src.shape[0])
    _load().or_adjoint_amp(src.shape[0], _p(src), xe.shape[0], _p(xe), *samp.args(), _p(r), _p(g))
    return g


def adjoint_elem(src, amp, xe, samp: Sampling, r) -> np.ndarray:
    """Gradient of <s, r> with respect to each element coordinate, [E,3]."""
    src, amp = _f64(src).reshape(-1, 3), _f64(amp).reshape(-1)
    xe, r = _f64(xe).reshape(-1, 3), _f64(r)
    assert r.shape == (xe.shape[0], samp.K)
    ge = np.zeros((xe.shape[0], 3))
    _load().or_adjoint_elem(src.shape[0], _p(src), _p(amp), xe.shape[0], _p(xe), *samp.args(),
                            _p(r), _p(ge))
    return ge


def count_updates(src, xe, samp: Sampling) -> int:
    """Exact number of in-window (source, element, sample) triples."""
    src, xe = _f64(src).reshape(-1, 3), _f64(xe).reshape(-1, 3)
    return int(_load().or_count_updates(src.shape[0], _p(src), xe.shape[0], _p(xe), *samp.args()))


def loss_residual(s, y):
    """Stage 1 objective without regulariser: L = sum (s - y)^2, r = 2 (s - y)."""
    s, y = _f64(s), _f64(y)
    r = np.zeros_like(s)
    L = _load().or_loss_residual(s.size, _p(s), _p(y), _p(r))
    return L, r


def nc_loss_residual(s, y, weight=None):
    """Stage 2 negative correlation, per row (one element's K samples): L_e = -Cov(s_e, y_e) /
    (sigma_sim sigma_meas), the statistics taken over the row's samples (population form; the
    normalisation cancels in the ratio).  A row where either signal has zero spread gets
    L_e = 0 and zero gradient.  With per-row weights w_e (the inlier mask of Stage 4; default
    1), returns (L_e [rows], dL/ds [rows, K]) for L = sum_e w_e L_e."""
    s, y = _f64(s), _f64(y)
    shape = s.shape
    s2, y2 = s.reshape(-1, shape[-1]), y.reshape(-1, shape[-1])
    K = s2.shape[1]
    ds = s2 - s2.mean(axis=1, keepdims=True)
    dy = y2 - y2.mean(axis=1, keepdims=True)
    C = (ds * dy).mean(axis=1)
    vs, vy = (ds * ds).mean(axis=1), (dy * dy).mean(axis=1)
    ok = (vs > 0) & (vy > 0)
    ss, sy = np.sqrt(np.where(ok, vs, 1.0)), np.sqrt(np.where(ok, vy, 1.0))
    L = np.where(ok, -C / (ss * sy), 0.0)
    # d rho / d s_k = (y_k - ybar) / (K ss sy) - C (s_k - sbar) / (K ss^3 sy), and L = -rho
    g = -(dy / (K * ss * sy)[:, None] - (C / (K * ss ** 3 * sy))[:, None] * ds)
    g[~ok] = 0.0
    w = np.ones(s2.shape[0]) if weight is None else _f64(weight).reshape(-1)
    return L.reshape(shape[:-1]), (g * w[:, None]).reshape(shape)


# ----------------------------------------------------------------------------------------------
# rigid array poses (Stage 4: X = R X_template + t)
# ----------------------------------------------------------------------------------------------

def element_positions(poses, elem) -> np.ndarray:
    """x[f, m] = R_f e_m + t_f; poses [F,12], elem [M,3] -> [F,M,3]."""
    poses, elem = _f64(poses).reshape(-1, 12), _f64(elem).reshape(-1, 3)
    F, M = poses.shape[0], elem.shape[0]
    xe = np.zeros((F, M, 3))
    _load().or_element_positions(F, _p(poses), M, _p(elem), _p(xe))
    return xe


def pose_grad(elem, ge) -> np.ndarray:
    """[F,12] = (dL/dR row-major, dL/dt) from element gradients ge [F,M,3]."""
    elem = _f64(elem).reshape(-1, 3)
    ge = _f64(ge)
    F, M = ge.shape[0], ge.shape[1]
    assert M == elem.shape[0]
    g = np.zeros((F, 12))
    _load().or_pose_grad(F, M, _p(elem), _p(ge), _p(g))
    return g


def rodrigues(w) -> np.ndarray:
    """R = exp([w]x) for an axis-angle vector w."""
    w = _f64(w).reshape(3)
    R = np.zeros(9)
    _load().or_rodrigues(_p(w), _p(R))
    return R.reshape(3, 3)


def rodrigues_vjp(w, gR) -> np.ndarray:
    """dL/dw from dL/dR for R = exp([w]x)."""
    w, gR = _f64(w).reshape(3), _f64(gR).reshape(9)
    gw = np.zeros(3)
    _load().or_rodrigues_vjp(_p(w), _p(gR), _p(gw))
    return gw


def poses_from_pose6(pose6) -> np.ndarray:
    """[F,6] (axis-angle w, translation t) -> [F,12] (R row-major, t)."""
    pose6 = _f64(pose6).reshape(-1, 6)
    out = np.zeros((pose6.shape[0], 12))
    for f in range(pose6.shape[0]):
        out[f, :9] = rodrigues(pose6[f, :3]).reshape(9)
        out[f, 9:] = pose6[f, 3:]
    return out


def pose6_grad(pose6, gpose12) -> np.ndarray:
    """Chain [F,12] (dL/dR, dL/dt) to [F,6] (dL/dw, dL/dt)."""
    pose6, gpose12 = _f64(pose6).reshape(-1, 6), _f64(gpose12).reshape(-1, 12)
    out = np.zeros_like(pose6)
    for f in range(pose6.shape[0]):
        out[f, :3] = rodrigues_vjp(pose6[f, :3], gpose12[f, :9])
        out[f, 3:] = gpose12[f, 9:]
    return out


def _axis_rotations(a):
    """Elementary rotations about x, y, z by angles a[0], a[1], a[2] and their derivatives."""
    out = []
    for i, t in enumerate(a):
        c, s = np.cos(t), np.sin(t)
        R = np.eye(3)
        D = np.zeros((3, 3))
        j, k = [(1, 2), (0, 2), (0, 1)][i]
        sg = -1.0 if i == 1 else 1.0           # about y the sine terms swap sign
        R[j, j], R[j, k], R[k, j], R[k, k] = c, -sg * s, sg * s, c
        D[j, j], D[j, k], D[k, j], D[k, k] = -s, -sg * c, sg * c, -s
        out.append((R, D))
    return out


def euler_rotation(a) -> np.ndarray:
    """Stage 4 Euler-angle parameterisation (reading: extrinsic x, then y, then z):
    R = Rz(a2) Ry(a1) Rx(a0)."""
    (Rx, _), (Ry, _), (Rz, _) = _axis_rotations(_f64(a).reshape(3))
    return Rz @ Ry @ Rx


def euler_vjp(a, gR) -> np.ndarray:
    """dL/da from G = dL/dR (row-major 9): <G, dR/da_i> by the product rule."""
    (Rx, Dx), (Ry, Dy), (Rz, Dz) = _axis_rotations(_f64(a).reshape(3))
    G = _f64(gR).reshape(3, 3)
    return np.array([np.sum(G * (Rz @ Ry @ Dx)), np.sum(G * (Rz @ Dy @ Rx)), np.sum(G * (Dz @ Ry @ Rx))])


def poses_from_euler6(pose6) -> np.ndarray:
    """[F,6] (Euler angles a, translation t) -> [F,12] (R row-major, t)."""
    pose6 = _f64(pose6).reshape(-1, 6)
    out = np.zeros((pose6.shape[0], 12))
    for f in range(pose6.shape[0]):
        out[f, :9] = euler_rotation(pose6[f, :3]).reshape(9)
        out[f, 9:] = pose6[f, 3:]
    return out


def euler6_grad(pose6, gpose12) -> np.ndarray:
    """Chain [F,12] (dL/dR, dL/dt) to [F,6] (dL/da, dL/dt)."""
    pose6, gpose12 = _f64(pose6).reshape(-1, 6), _f64(gpose12).reshape(-1, 12)
    out = np.zeros_like(pose6)
    for f in range(pose6.shape[0]):
        out[f, :3] = euler_vjp(pose6[f, :3], gpose12[f, :9])
        out[f, 3:] = gpose12[f, 9:]
    return out


# ----------------------------------------------------------------------------------------------
# voxel-grid form: each voxel is a Gaussian blob of width sigma at its centre (Eq. (A13))
# ----------------------------------------------------------------------------------------------

@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    origin: tuple
    spacing: float

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    @property
    def n(self):
        return self.nx * self.ny * self.nz


def voxel_centres(grid: Grid, index=None) -> np.ndarray:
    """Centres of all voxels (C-order, z fastest), or of the flat voxel indices ``index``."""
    if index is None:
        index = np.arange(grid.n)
    index = np.asarray(index, dtype=np.int64)
    i = index // (grid.ny * grid.nz)
    j = (index // grid.nz) % grid.ny
    k = index % grid.nz
    o = np.asarray(grid.origin, dtype=np.float64)
    return np.stack([o[0] + i * grid.spacing, o[1] + j * grid.spacing,
                     o[2] + k * grid.spacing], axis=1)


def grid_forward(grid: Grid, p0, poses, elem, samp: Sampling, elements=None) -> np.ndarray:
    """s[f, m, k] for the volume p0 [nx,ny,nz] and posed array; ``elements`` restricts the
    output to a list of flat (f*M + m) indices (returned as [len, K])."""
    xe = element_positions(poses, elem).reshape(-1, 3)
    src = voxel_centres(grid)
    amp = _f64(p0).reshape(-1)
    if elements is not None:
        return forward(src, amp, xe[np.asarray(elements)], samp)
    F, M = _f64(poses).reshape(-1, 12).shape[0], _f64(elem).reshape(-1, 3).shape[0]
    return forward(src, amp, xe, samp).reshape(F, M, samp.K)


def grid_adjoint_p0(grid: Grid, poses, elem, samp: Sampling, r, voxels=None) -> np.ndarray:
    """dL/dp0 for dL/ds = r [F,M,K]; ``voxels`` restricts to flat voxel indices."""
    xe = element_positions(poses, elem).reshape(-1, 3)
    src = voxel_centres(grid, voxels)
    g = adjoint_amp(src, xe, samp, _f64(r).reshape(xe.shape[0], samp.K))
    return g if voxels is not None else g.reshape(grid.shape)


def grid_adjoint_elem(grid: Grid, p0, poses, elem, samp: Sampling, r, elements=None) -> np.ndarray:
    """dL/dx_e [F,M,3] (or [len,3] for flat ``elements``) for dL/ds = r."""
    poses_a = _f64(poses).reshape(-1, 12)
    elem_a = _f64(elem).reshape(-1, 3)
    F, M = poses_a.shape[0], elem_a.shape[0]
    xe = element_positions(poses_a, elem_a).reshape(-1, 3)
    r = _f64(r).reshape(F * M, samp.K)
    src, amp = voxel_centres(grid), _f64(p0).reshape(-1)
    if elements is not None:
        idx = np.asarray(elements)
        return adjoint_elem(src, amp, xe[idx], samp, np.ascontiguousarray(r[idx]))
    return adjoint_elem(src, amp, xe, samp, r).reshape(F, M, 3)


def grid_count_updates(grid: Grid, poses, elem, samp: Sampling, elements=None) -> int:
    xe = element_positions(poses, elem).reshape(-1, 3)
    if elements is not None:
        xe = xe[np.asarray(elements)]
    return count_updates(voxel_centres(grid), xe, samp)


def grid_nc_loss_and_grad(grid: Grid, p0, poses, elem, samp: Sampling, y, weight=None):
    """Stage 2/4 objective on a posed array: per-element NC losses L_e [F,M], the element
    gradients of sum_e w_e L_e [F,M,3] and the pose gradient [F,12] (rigid chain of Stage 4)."""
    s = grid_forward(grid, p0, poses, elem, samp)
    L, r = nc_loss_residual(s, y, weight)
    ge = grid_adjoint_elem(grid, p0, poses, elem, samp, r)
    return L, ge, pose_grad(elem, ge)


# ----------------------------------------------------------------------------------------------
# TGV regulariser of the Stage 1 / Stage 5 objectives (second order, auxiliary field w)
# ----------------------------------------------------------------------------------------------

def _dplus(u, a):
    """Forward difference along axis a, zero at the last index."""
    d = np.zeros_like(u)
    sl_hi = [slice(None)] * 3
    sl_lo = [slice(None)] * 3
    sl_hi[a], sl_lo[a] = slice(1, None), slice(0, -1)
    d[tuple(sl_lo)] = u[tuple(sl_hi)] - u[tuple(sl_lo)]
    return d


def _dminus(u, a):
    """Backward difference along axis a, zero at the first index."""
    d = np.zeros_like(u)
    sl_hi = [slice(None)] * 3
    sl_lo = [slice(None)] * 3
    sl_hi[a], sl_lo[a] = slice(1, None), slice(0, -1)
    d[tuple(sl_hi)] = u[tuple(sl_hi)] - u[tuple(sl_lo)]
    return d


def tgv_value(u, w, alpha0, alpha1, eps):
    """Second-order total generalised variation with its auxiliary field written out:
    alpha1 sum_v |D+ u - w|_eps + alpha0 sum_v |E(w)|_eps, with D+ the forward-difference
    gradient, E(w)_ab = (D-_a w_b + D-_b w_a)/2 the symmetrised backward-difference gradient
    (Frobenius norm), and |x|_eps = sqrt(|x|^2 + eps^2) - eps.  u [nx,ny,nz]; w [3,nx,ny,nz]."""
    u, w = _f64(u), _f64(w)
    g = np.stack([_dplus(u, a) for a in range(3)]) - w
    n1 = np.sqrt((g * g).sum(0) + eps * eps) - eps
    D = [[_dminus(w[b], a) for b in range(3)] for a in range(3)]
    E2 = sum(((D[a][b] + D[b][a]) / 2) ** 2 for a in range(3) for b in range(3))
    n0 = np.sqrt(E2 + eps * eps) - eps
    return alpha1 * n1.sum() + alpha0 * n0.sum()


def tgv_grad(u, w, alpha0, alpha1, eps):
    """Gradients (dTGV/du [nx,ny,nz], dTGV/dw [3,nx,ny,nz]) of tgv_value: the adjoints of the
    two difference operators applied to the normalised fields."""
    u, w = _f64(u), _f64(w)
    g = np.stack([_dplus(u, a) for a in range(3)]) - w
    q = alpha1 * g / np.sqrt((g * g).sum(0) + eps * eps)
    D = [[_dminus(w[b], a) for b in range(3)] for a in range(3)]
    E = [[(D[a][b] + D[b][a]) / 2 for b in range(3)] for a in range(3)]
    nrm = np.sqrt(sum(E[a][b] ** 2 for a in range(3) for b in range(3)) + eps * eps)
    Q = [[alpha0 * E[a][b] / nrm for b in range(3)] for a in range(3)]
    gu = np.zeros_like(u)
    gw = -q.copy()
    for a in range(3):
        # adjoint of D+_a (zero at the last index): -(q(v) - q(v - e_a)) with the ends handled
        qa = q[a].copy()
        idx_last = [slice(None)] * 3
        idx_last[a] = -1
        qa[tuple(idx_last)] = 0.0
        gu += _dminus_full(qa, a)
        for b in range(3):
            # adjoint of D-_a (zero at the first index) applied to Q_ab for w_b
            gw[b] += _dplus_adj(Q[a][b], a)
    return gu, gw


def _dminus_full(x, a):
    """-(D+)^T x for D+ zero at the last index: x(v - e_a) - x(v), with x(-1) = 0 (x is zero
    at the last index on entry)."""
    y = -x.copy()
    sl_hi = [slice(None)] * 3
    sl_lo = [slice(None)] * 3
    sl_hi[a], sl_lo[a] = slice(1, None), slice(0, -1)
    y[tuple(sl_hi)] += x[tuple(sl_lo)]
    return y


def _dplus_adj(x, a):
    """(D-)^T x for D- zero at the first index: x(v) [v_a >= 1] - x(v + e_a) [v_a + 1 <= n-1]."""
    y = x.copy()
    sl0 = [slice(None)] * 3
    sl0[a] = 0
    y[tuple(sl0)] = 0.0
    sl_hi = [slice(None)] * 3
    sl_lo = [slice(None)] * 3
    sl_hi[a], sl_lo[a] = slice(1, None), slice(0, -1)
    y[tuple(sl_lo)] -= x[tuple(sl_hi)]
    return y
