"""Seeded synthetic inputs: grids, array templates, poses, vessel phantoms, residuals.

This module only draws inputs.  It contains none of the radiation model's
arithmetic, and both the GPU path and the CPU oracle take their inputs from it.
Rotation matrices for the generated poses come from
``scipy.spatial.transform.Rotation``.

The paper's data are not available (the phantom liver of the simulation
study and the in-vivo rat kidney recordings), so the configurations below use
phantoms with the stated statistics:

* ``C1``: a 32^3 grid at 0.2 mm centred 10 mm below a 64-element linear
  array (pitch 0.3 mm), one identity frame, K=512, sigma=0.1 mm, three
  random-walk tubes (radius U(0.2,0.5) mm, value U(0.5,1)), residual N(0,1);
* ``C2``: a 128x128x64 grid at 0.1 mm, a 128-element linear array, 64
  frames stepping 0.2 mm in y with 0.3 mm / 1.5 deg jitter, K=1024,
  sigma=0.08 mm, a 40-branch vessel tree (radii 0.08-0.6 mm, values
  U(0.3,1)) plus N(0, 0.01^2) on every voxel;
* ``C3``: a 256x256x128 grid at 0.08 mm, 128 elements, 256 frames stepping
  0.08 mm, K=2048, sigma=0.08 mm, initial poses perturbed by N(0, 0.5 mm)
  and N(0, 2 deg);
* ``C4``: a 256^3 grid at 0.1 mm whose top plane is 2 mm below a 32x32
  matrix array (pitch 0.5 mm), 8 frames with 0.3 mm / 1 deg jitter,
  K=2048, sigma=0.1 mm, a 120-branch tree.

All use c = 1540 m/s, fs = 40 MHz and truncation at 6 sigma.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation

C_SOUND = 1540.0
FS = 40e6
TRUNC = 6.0
MM = 1e-3


@dataclass
class Workload:
    name: str
    shape: tuple            # (nx, ny, nz)
    origin: tuple           # metres, centre of voxel (0,0,0)
    spacing: float          # metres
    c: float
    fs: float
    K: int
    sigma: float
    trunc: float
    elem: np.ndarray        # [M,3] float64, probe frame
    pose6: np.ndarray       # [F,6] float64 (axis-angle, translation)
    poses: np.ndarray       # [F,12] float64 (R row-major, t)
    p0: np.ndarray          # [nx,ny,nz] float64
    extra: dict = field(default_factory=dict)

    @property
    def F(self):
        return self.poses.shape[0]

    @property
    def M(self):
        return self.elem.shape[0]

    @property
    def n_voxels(self):
        return int(np.prod(self.shape))


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(seed).spawn(stream + 1)[stream])


def centred_origin(shape, spacing, centre):
    return tuple(float(centre[a] - 0.5 * (shape[a] - 1) * spacing) for a in range(3))


def linear_array(M: int, pitch: float) -> np.ndarray:
    x = (np.arange(M) - 0.5 * (M - 1)) * pitch
    return np.stack([x, np.zeros(M), np.zeros(M)], axis=1)


def matrix_array(n: int, pitch: float) -> np.ndarray:
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x = (i.reshape(-1) - 0.5 * (n - 1)) * pitch
    y = (j.reshape(-1) - 0.5 * (n - 1)) * pitch
    return np.stack([x, y, np.zeros(n * n)], axis=1)


def poses_from_pose6(pose6: np.ndarray) -> np.ndarray:
    pose6 = np.asarray(pose6, dtype=np.float64).reshape(-1, 6)
    R = Rotation.from_rotvec(pose6[:, :3]).as_matrix().reshape(-1, 9)
    return np.ascontiguousarray(np.concatenate([R, pose6[:, 3:]], axis=1))


def sweep_pose6(F: int, step: float, jitter_t: float, jitter_deg: float, rng) -> np.ndarray:
    """Frames stepping along y, plus Gaussian translation and axis-angle jitter."""
    pose6 = np.zeros((F, 6))
    pose6[:, 4] = (np.arange(F) - 0.5 * (F - 1)) * step
    pose6[:, 3:] += rng.normal(0.0, jitter_t, size=(F, 3))
    pose6[:, :3] += rng.normal(0.0, np.deg2rad(jitter_deg), size=(F, 3))
    return pose6


# ----------------------------------------------------------------------------------------------
# phantoms
# ----------------------------------------------------------------------------------------------

def _paint_segment(vol, origin, h, a, b, radius, value):
    """Set voxels whose centre lies within ``radius`` of segment ab to max(vol, value)."""
    lo = np.minimum(a, b) - radius
    hi = np.maximum(a, b) + radius
    o = np.asarray(origin)
    i0 = np.maximum(np.floor((lo - o) / h).astype(int), 0)
    i1 = np.minimum(np.ceil((hi - o) / h).astype(int) + 1, np.array(vol.shape))
    if np.any(i1 <= i0):
        return
    gx = o[0] + np.arange(i0[0], i1[0]) * h
    gy = o[1] + np.arange(i0[1], i1[1]) * h
    gz = o[2] + np.arange(i0[2], i1[2]) * h
    X, Y, Z = np.meshgrid(gx, gy, gz, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1)
    ab = b - a
    L2 = float(ab @ ab)
    t = np.clip(((P - a) @ ab) / L2, 0.0, 1.0) if L2 > 0 else np.zeros(P.shape[:-1])
    near = P - (a + t[..., None] * ab)
    inside = np.einsum("...i,...i->...", near, near) <= radius * radius
    sub = vol[i0[0]:i1[0], i0[1]:i1[1], i0[2]:i1[2]]
    np.maximum(sub, np.where(inside, value, 0.0), out=sub)


def _random_walk(rng, start, direction, n_steps, step, turn):
    pts = [np.asarray(start, dtype=np.float64)]
    d = np.asarray(direction, dtype=np.float64)
    d /= np.linalg.norm(d)
    for _ in range(n_steps):
        d = d + rng.normal(0.0, turn, size=3)
        d /= np.linalg.norm(d)
        pts.append(pts[-1] + step * d)
    return np.array(pts)


def random_tubes(shape, origin, h, n_tubes, r_lo, r_hi, v_lo, v_hi, rng):
    vol = np.zeros(shape)
    o = np.asarray(origin)
    ext = np.asarray(shape) * h
    for _ in range(n_tubes):
        start = o + rng.uniform(0.2, 0.8, size=3) * ext
        walk = _random_walk(rng, start, rng.normal(size=3), 24, 2.0 * h, 0.35)
        radius = rng.uniform(r_lo, r_hi)
        value = rng.uniform(v_lo, v_hi)
        for a, b in zip(walk[:-1], walk[1:]):
            _paint_segment(vol, origin, h, a, b, radius, value)
    return vol


def vessel_tree(shape, origin, h, n_branches, r_max, r_min, v_lo, v_hi, rng):
    """Branching random-walk vessels: a root crossing the volume, children spawned from
    points of earlier branches with radius shrinking by U(0.6, 0.85) down to r_min."""
    vol = np.zeros(shape)
    o = np.asarray(origin)
    ext = np.asarray(shape) * h
    step = max(2.0 * h, 0.25 * MM)
    branches = []
    start = o + np.array([0.05, 0.5, 0.5]) * ext
    root = _random_walk(rng, start, [1.0, 0.0, 0.0], int(0.9 * ext[0] / step), step, 0.15)
    branches.append((root, r_max))
    while len(branches) < n_branches:
        parent, pr = branches[rng.integers(len(branches))]
        p = parent[rng.integers(len(parent))]
        radius = max(r_min, pr * rng.uniform(0.6, 0.85))
        n_steps = int(rng.integers(8, 24))
        branches.append((_random_walk(rng, p, rng.normal(size=3), n_steps, step, 0.3), radius))
    for walk, radius in branches:
        value = rng.uniform(v_lo, v_hi)
        for a, b in zip(walk[:-1], walk[1:]):
            _paint_segment(vol, origin, h, a, b, radius, value)
    return vol


# ----------------------------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------------------------

def c1(seed: int = 0) -> Workload:
    shape, h = (32, 32, 32), 0.2 * MM
    origin = centred_origin(shape, h, (0.0, 0.0, 10 * MM))
    elem = linear_array(64, 0.3 * MM)
    pose6 = np.zeros((1, 6))
    p0 = random_tubes(shape, origin, h, 3, 0.2 * MM, 0.5 * MM, 0.5, 1.0, np.random.default_rng(seed))
    r = np.random.default_rng(seed + 1).normal(size=(1, 64, 512))
    return Workload("C1", shape, origin, h, C_SOUND, FS, 512, 0.1 * MM, TRUNC, elem, pose6,
                    poses_from_pose6(pose6), p0, {"r": r})


def c2(seed: int = 0, background: bool = True) -> Workload:
    shape, h = (128, 128, 64), 0.1 * MM
    origin = centred_origin(shape, h, (0.0, 0.0, 10 * MM))
    elem = linear_array(128, 0.3 * MM)
    pose6 = sweep_pose6(64, 0.2 * MM, 0.3 * MM, 1.5, _rng(seed, 0))
    p0 = vessel_tree(shape, origin, h, 40, 0.6 * MM, 0.08 * MM, 0.3, 1.0, _rng(seed, 1))
    if background:
        p0 = p0 + _rng(seed, 2).normal(0.0, 0.01, size=shape)
    return Workload("C2", shape, origin, h, C_SOUND, FS, 1024, 0.08 * MM, TRUNC, elem, pose6,
                    poses_from_pose6(pose6), p0)


def c3(seed: int = 0, frames: int = 256) -> Workload:
    shape, h = (256, 256, 128), 0.08 * MM
    origin = centred_origin(shape, h, (0.0, 0.0, 10 * MM))
    elem = linear_array(128, 0.3 * MM)
    true6 = sweep_pose6(frames, 0.08 * MM, 0.3 * MM, 1.5, _rng(seed, 0))
    init6 = true6.copy()
    rng = _rng(seed, 3)
    init6[:, 3:] += rng.normal(0.0, 0.5 * MM, size=(frames, 3))
    init6[:, :3] += rng.normal(0.0, np.deg2rad(2.0), size=(frames, 3))
    p0 = vessel_tree(shape, origin, h, 60, 0.6 * MM, 0.08 * MM, 0.3, 1.0, _rng(seed, 1))
    return Workload("C3", shape, origin, h, C_SOUND, FS, 2048, 0.08 * MM, TRUNC, elem, true6,
                    poses_from_pose6(true6), p0, {"init_pose6": init6})


def c4(seed: int = 0) -> Workload:
    shape, h = (256, 256, 256), 0.1 * MM
    origin = (-0.5 * (shape[0] - 1) * h, -0.5 * (shape[1] - 1) * h, 2.0 * MM)
    elem = matrix_array(32, 0.5 * MM)
    pose6 = sweep_pose6(8, 0.0, 0.3 * MM, 1.0, _rng(seed, 0))
    p0 = vessel_tree(shape, origin, h, 120, 0.6 * MM, 0.08 * MM, 0.3, 1.0, _rng(seed, 1))
    return Workload("C4", shape, origin, h, C_SOUND, FS, 2048, 0.1 * MM, TRUNC, elem, pose6,
                    poses_from_pose6(pose6), p0)


def fibonacci_cap(M: int, radius: float, half_angle: float) -> np.ndarray:
    """M points spread evenly (golden-angle spiral) over the cap of a sphere of `radius`
    centred at the origin, within `half_angle` of the -z axis: elements below a volume that
    sits around the sphere's centre, each facing it."""
    k = np.arange(M) + 0.5
    cos_t = 1.0 - (1.0 - np.cos(half_angle)) * k / M          # uniform in area over the cap
    sin_t = np.sqrt(1.0 - cos_t ** 2)
    phi = k * np.pi * (3.0 - np.sqrt(5.0))
    return radius * np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), -cos_t], axis=1)


def cap33(seed: int = 0) -> Workload:
    """The simulation setup of the paper's multi-view experiment: a 33-element sparse array on a
    spherical cap (here radius 40 mm, half-angle 35 degrees; sizes not stated) around a 256^3
    grid at 0.1 mm; three views (the reference pose and two translated and rotated ones)."""
    shape, h = (256, 256, 256), 0.1 * MM
    origin = centred_origin(shape, h, (0.0, 0.0, 0.0))
    elem = fibonacci_cap(33, 40 * MM, np.deg2rad(35.0))
    pose6 = np.array([[0.0, 0.0, 0.0, 0.0, 0.0, 0.0],
                      [0.12, -0.05, 0.3, 1.5 * MM, -1.0 * MM, 0.5 * MM],
                      [-0.08, 0.1, -0.25, -1.0 * MM, 2.0 * MM, -0.5 * MM]])
    p0 = vessel_tree(shape, origin, h, 120, 0.6 * MM, 0.08 * MM, 0.3, 1.0, _rng(seed, 1))
    return Workload("cap33", shape, origin, h, C_SOUND, FS, 2048, 0.1 * MM, TRUNC, elem, pose6,
                    poses_from_pose6(pose6), p0)


def hemisphere1024(seed: int = 0, view: int = 0) -> Workload:
    """The in-vivo system's geometry: 1024 elements on a hemisphere of radius 60 mm, split into
    two views of 512 by azimuth (view 0: the 512 of smallest azimuth), around a 256^3 grid at
    0.1 mm centred at the sphere's centre."""
    shape, h = (256, 256, 256), 0.1 * MM
    origin = centred_origin(shape, h, (0.0, 0.0, 0.0))
    full = fibonacci_cap(1024, 60 * MM, np.pi / 2)
    order = np.argsort(np.mod(np.arctan2(full[:, 1], full[:, 0]), 2 * np.pi), kind="stable")
    elem = full[np.sort(order[:512] if view == 0 else order[512:])]
    pose6 = np.zeros((1, 6))
    p0 = vessel_tree(shape, origin, h, 120, 0.6 * MM, 0.08 * MM, 0.3, 1.0, _rng(seed, 1))
    return Workload("hemi1024v%d" % view, shape, origin, h, C_SOUND, FS, 2560, 0.1 * MM, TRUNC, elem, pose6,
                    poses_from_pose6(pose6), p0)


def small(seed: int = 0, shape=(9, 7, 5), h=0.2 * MM, M=5, F=2, K=400, sigma=0.1 * MM) -> Workload:
    """A tiny jittered configuration for brute-force checks."""
    origin = centred_origin(shape, h, (0.0, 0.0, 8 * MM))
    elem = linear_array(M, 0.7 * MM)
    pose6 = sweep_pose6(F, 0.5 * MM, 0.3 * MM, 3.0, _rng(seed, 0))
    p0 = _rng(seed, 1).uniform(-0.5, 1.0, size=shape)
    r = _rng(seed, 2).normal(size=(F, M, K))
    return Workload("small", shape, origin, h, C_SOUND, FS, K, sigma, TRUNC, elem, pose6,
                    poses_from_pose6(pose6), p0, {"r": r})


def serving_volume(seed: int = 0, n: int = 256, h: float = 0.1 * MM, branches: int = 60):
    """Resident volume for the serving workload: n^3 voxels whose top plane is 2 mm deep."""
    shape = (n, n, n)
    origin = (-0.5 * (n - 1) * h, -0.5 * (n - 1) * h, 2.0 * MM)
    p0 = vessel_tree(shape, origin, h, branches, 0.6 * MM, 0.08 * MM, 0.3, 1.0, _rng(seed, 5))
    return shape, origin, h, p0


@dataclass
class RequestSpec:
    rid: int
    kind: int                # 0 pose refinement, 1 volume update
    arrival: float           # seconds from the start of the stream
    box: tuple               # (i0, j0, k0, nx, ny, nz) voxels of the resident volume
    M: int
    K: int
    elem: np.ndarray         # [M,3] linear array, pitch 0.3 mm
    true6: np.ndarray        # pose that generated the measured signals
    init6: np.ndarray        # starting pose (pose requests); equals true6 for volume requests
    steps: int


def serving_stream(n_requests: int, rate: float, shape, origin, h, seed: int = 0, frac_pose: float = 0.7,
                   Ms=(64, 128, 256), Ks=(512, 1024, 2048), side=(64, 160), depth: float = 10 * MM,
                   pose_steps: int = 10, jitter_t: float = 0.1 * MM, jitter_deg: float = 0.5):
    """Poisson arrivals of mixed requests.  Each request has a box of side U{side} of the
    resident volume and a linear array `depth` above the box centre, rotated about z by a
    random angle; pose requests start from the true pose plus Gaussian jitter."""
    rng = _rng(seed, 6)
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate)
        kind = 0 if rng.uniform() < frac_pose else 1
        n = int(rng.integers(side[0], side[1] + 1))
        n = min(n, *shape)
        i0 = int(rng.integers(0, shape[0] - n + 1))
        j0 = int(rng.integers(0, shape[1] - n + 1))
        k0 = int(rng.integers(0, max(1, shape[2] - n + 1)))
        cz = origin[2] + (k0 + 0.5 * (n - 1)) * h
        cx = origin[0] + (i0 + 0.5 * (n - 1)) * h
        cy = origin[1] + (j0 + 0.5 * (n - 1)) * h
        M = int(rng.choice(Ms))
        K = int(rng.choice(Ks))
        true6 = np.array([0.0, 0.0, rng.uniform(-np.pi, np.pi), cx, cy, cz - depth])
        init6 = true6.copy()
        if kind == 0:
            init6[:3] += rng.normal(0.0, np.deg2rad(jitter_deg), 3)
            init6[3:] += rng.normal(0.0, jitter_t, 3)
        out.append(RequestSpec(rid, kind, t, (i0, j0, k0, n, n, n), M, K, linear_array(M, 0.3 * MM), true6,
                               init6, pose_steps if kind == 0 else 1))
    return out


def residual(F: int, M: int, K: int, seed: int = 1) -> np.ndarray:
    return np.random.default_rng(seed).normal(size=(F, M, K))


CONFIGS = {"C1": c1, "C2": c2, "C3": c3, "C4": c4}
