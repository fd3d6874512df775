"""The seeded input generators on the CPU: determinism per seed, the geometric preconditions the
configurations rely on (elements outside the grid by more than the library's 10 sigma check, every
window inside [0, K)), rigid poses, phantom statistics and the serving stream's statistics."""
import numpy as np
import pytest

from paper_2604_09643_amd import workloads as W

GEOMETRIES = [W.c1, W.c2, W.c3, W.c4, W.cap33, lambda: W.hemisphere1024(view=0),
              lambda: W.hemisphere1024(view=1)]


def element_positions(w):
    R = w.poses[:, :9].reshape(-1, 3, 3)
    return np.einsum("fij,mj->fmi", R, w.elem) + w.poses[:, None, 9:]


def grid_box(w):
    lo = np.asarray(w.origin, dtype=np.float64)
    return lo, lo + (np.asarray(w.shape) - 1) * w.spacing


def test_seeded_determinism():
    a, b, c = W.c1(0), W.c1(0), W.c1(1)
    assert np.array_equal(a.p0, b.p0) and np.array_equal(a.poses, b.poses) and np.array_equal(a.extra["r"],
                                                                                                b.extra["r"])
    assert not np.array_equal(a.p0, c.p0)
    a, b = W.c2(0), W.c2(0)
    assert np.array_equal(a.p0, b.p0) and np.array_equal(a.poses, b.poses)
    assert not np.array_equal(a.poses, W.c2(1).poses)
    s1 = W.serving_stream(50, 20.0, (256,) * 3, (0.0, 0.0, 0.0), 1e-4, seed=3)
    s2 = W.serving_stream(50, 20.0, (256,) * 3, (0.0, 0.0, 0.0), 1e-4, seed=3)
    assert [(r.arrival, r.box, r.M, r.K, r.kind) for r in s1] == [(r.arrival, r.box, r.M, r.K, r.kind) for r in s2]


@pytest.mark.parametrize("make", GEOMETRIES)
def test_geometry_preconditions(make):
    """Elements stay more than 10 sigma from the grid box (closer ones make the library report
    RA_EGEOM), and every voxel-element distance d has its whole window inside the record:
    d - 6 sigma >= 0 and d + 6 sigma <= (K - 1) c / fs."""
    w = make()
    xe = element_positions(w).reshape(-1, 3)
    lo, hi = grid_box(w)
    d_box = np.linalg.norm(xe - np.clip(xe, lo, hi), axis=1).min()
    corners = np.array([[x, y, z] for x in (lo[0], hi[0]) for y in (lo[1], hi[1]) for z in (lo[2], hi[2])])
    d_max = np.linalg.norm(xe[:, None, :] - corners[None], axis=2).max()   # a convex box's farthest point
    assert d_box > 10.0 * w.sigma, (w.name, d_box / w.sigma)
    assert d_box - w.trunc * w.sigma >= 0.0
    assert d_max + w.trunc * w.sigma <= (w.K - 1) * w.c / w.fs, (w.name, d_max)


@pytest.mark.parametrize("make", GEOMETRIES)
def test_poses_are_rigid(make):
    w = make()
    R = w.poses[:, :9].reshape(-1, 3, 3)
    assert np.allclose(R @ R.transpose(0, 2, 1), np.eye(3), atol=1e-12)
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-12)


def test_sweep_frames_step_along_y():
    """The sweep's 64 frames step 0.2 mm in y with 0.3 mm jitter: the mean step over the sweep is
    0.2 mm to within the jitter's contribution (2 x 0.3 mm / 63)."""
    w = W.c2()
    ty = w.poses[:, 10]
    assert abs((ty[-1] - ty[0]) / (w.F - 1) - 0.2e-3) <= 2 * 3 * 0.3e-3 / (w.F - 1)


def test_phantom_statistics():
    """C1: three tubes with values in [0.5, 1] and zero elsewhere; the sweep: a vessel tree with
    values in [0.3, 1] and zero elsewhere, plus N(0, 0.01^2) on every voxel; both occupy a few
    percent of the volume."""
    w = W.c1()
    v = w.p0[w.p0 != 0]
    assert v.min() >= 0.5 and v.max() <= 1.0
    assert 0.005 <= v.size / w.p0.size <= 0.1
    t = W.c2(background=False).p0
    v = t[t != 0]
    assert v.min() >= 0.3 and v.max() <= 1.0
    assert 0.005 <= v.size / t.size <= 0.1
    bg = W.c2().p0 - t
    assert abs(bg.mean()) <= 5 * 0.01 / np.sqrt(bg.size)
    assert abs(bg.std() / 0.01 - 1.0) <= 0.01


def test_serving_stream_statistics():
    """Poisson arrivals at the offered rate, 70% pose requests, boxes inside the resident volume,
    sizes from the stated sets, and each array 10 mm above its box centre."""
    shape, origin, h = (256, 256, 256), (-12.75e-3, -12.75e-3, 2e-3), 1e-4
    rate, n = 50.0, 4000
    reqs = W.serving_stream(n, rate, shape, origin, h, seed=9)
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() * rate - 1.0) <= 4.0 / np.sqrt(n)          # exponential gaps: sd = mean
    frac_pose = np.mean([r.kind == 0 for r in reqs])
    assert abs(frac_pose - 0.7) <= 4.0 * np.sqrt(0.21 / n)
    for r in reqs:
        i0, j0, k0, nx, ny, nz = r.box
        assert 64 <= nx <= 160 and nx == ny == nz
        assert 0 <= i0 and i0 + nx <= shape[0] and 0 <= j0 and j0 + ny <= shape[1] and 0 <= k0
        assert k0 + nz <= shape[2]
        assert r.M in (64, 128, 256) and r.K in (512, 1024, 2048) and r.elem.shape == (r.M, 3)
        cz = origin[2] + (k0 + 0.5 * (nz - 1)) * h
        assert abs(r.true6[5] - (cz - 10e-3)) <= 1e-12
        assert r.steps == (10 if r.kind == 0 else 1)
        if r.kind == 1:
            assert np.array_equal(r.init6, r.true6)
