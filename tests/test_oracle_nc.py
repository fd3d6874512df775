"""Pins of the oracle's Stage 2 negative-correlation loss and its gradients (CPU)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2604_09643_amd import workloads as W


def rows(seed, n=6, K=200):
    rng = np.random.default_rng(seed)
    s = rng.normal(size=(n, K)) + np.sin(np.linspace(0, 9, K))
    y = 0.4 * s + rng.normal(size=(n, K))
    return s, y


def test_loss_is_minus_pearson_r():
    """Against numpy's Pearson correlation coefficient, row by row."""
    s, y = rows(0)
    L, _ = O.nc_loss_residual(s, y)
    ref = np.array([-np.corrcoef(a, b)[0, 1] for a, b in zip(s, y)])
    np.testing.assert_allclose(L, ref, rtol=0, atol=1e-14)


def test_special_values_and_invariance():
    s, y = rows(1, n=1)
    assert O.nc_loss_residual(s, s)[0][0] == pytest.approx(-1.0, abs=1e-15)
    assert O.nc_loss_residual(-2.0 * s + 3.0, s)[0][0] == pytest.approx(1.0, abs=1e-15)
    L0 = O.nc_loss_residual(s, y)[0]
    L1 = O.nc_loss_residual(7.5 * s - 2.0, y)[0]
    L2 = O.nc_loss_residual(s, 0.1 * y + 4.0)[0]
    np.testing.assert_allclose([L1, L2], [L0, L0], rtol=0, atol=1e-14)
    assert np.all(np.abs(O.nc_loss_residual(*rows(2))[0]) <= 1.0)


def test_gradient_finite_differences():
    s, y = rows(3, n=3, K=60)
    _, g = O.nc_loss_residual(s, y)
    h = 1e-6
    fd = np.zeros_like(s)
    for i in range(s.shape[0]):
        for k in range(s.shape[1]):
            sp, sm = s.copy(), s.copy()
            sp[i, k] += h
            sm[i, k] -= h
            fd[i, k] = (O.nc_loss_residual(sp, y)[0][i] - O.nc_loss_residual(sm, y)[0][i]) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-8 * np.max(np.abs(g))


def test_gradient_orthogonal_to_shift_and_scale():
    """Shift and scale invariance: the gradient sums to zero and is orthogonal to s."""
    s, y = rows(4)
    _, g = O.nc_loss_residual(s, y)
    scale = np.abs(g).sum(axis=1)
    assert np.all(np.abs(g.sum(axis=1)) <= 1e-14 * scale * s.shape[1])
    assert np.all(np.abs((g * s).sum(axis=1)) <= 1e-12 * (np.abs(g * s)).sum(axis=1))


def test_flat_rows_and_weights():
    s, y = rows(5, n=3)
    s[1] = 2.0                                  # no spread: loss and gradient are zero
    L, g = O.nc_loss_residual(s, y, weight=[1.0, 1.0, 0.0])
    assert L[1] == 0.0 and np.all(g[1] == 0.0)
    assert np.all(g[2] == 0.0) and L[2] != 0.0   # weight 0 masks the gradient, not the loss
    L1, g1 = O.nc_loss_residual(s[:1], y[:1])
    np.testing.assert_array_equal(g[0], g1[0])


def test_element_gradient_finite_differences():
    """The composite Stage 2 gradient d(sum_e L_e)/dx_e against central differences of the
    forward model plus the loss, moving one element at a time."""
    w = W.small(shape=(7, 6, 5), M=4, F=1, K=400)
    og = O.Grid(*w.shape, w.origin, w.spacing)
    os_ = O.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)
    # measured signals: the same volume seen from slightly shifted elements
    elem_true = w.elem + np.array([[30e-6, -20e-6, 40e-6]])
    y = O.grid_forward(og, w.p0, w.poses, elem_true, os_)
    L, ge, gpose = O.grid_nc_loss_and_grad(og, w.p0, w.poses, w.elem, os_, y)
    R = w.poses[0, :9].reshape(3, 3)
    gtemplate = ge[0] @ R                       # d/de_m = R^T dL/dx_m
    h = 1e-7
    for m in range(w.M):
        for a in range(3):
            ep, em = w.elem.copy(), w.elem.copy()
            ep[m, a] += h
            em[m, a] -= h
            Lp = O.nc_loss_residual(O.grid_forward(og, w.p0, w.poses, ep, os_), y)[0].sum()
            Lm = O.nc_loss_residual(O.grid_forward(og, w.p0, w.poses, em, os_), y)[0].sum()
            fd = (Lp - Lm) / (2 * h)
            assert abs(gtemplate[m, a] - fd) <= 2e-4 * np.abs(gtemplate).max(), (m, a, gtemplate[m, a], fd)


def test_euler_rotation_against_scipy():
    """Stage 4 Euler angles: R = Rz(a2) Ry(a1) Rx(a0), i.e. scipy's extrinsic 'xyz'."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(11)
    for a in rng.uniform(-3.0, 3.0, size=(20, 3)):
        np.testing.assert_allclose(O.euler_rotation(a), Rotation.from_euler("xyz", a).as_matrix(),
                                   rtol=0, atol=1e-15)


def test_euler_vjp_finite_differences():
    rng = np.random.default_rng(12)
    for a in rng.uniform(-2.0, 2.0, size=(5, 3)):
        G = rng.normal(size=(3, 3))
        g = O.euler_vjp(a, G)
        fd = np.zeros(3)
        for i in range(3):
            ap, am = a.copy(), a.copy()
            ap[i] += 1e-6
            am[i] -= 1e-6
            fd[i] = np.sum(G * (O.euler_rotation(ap) - O.euler_rotation(am))) / 2e-6
        np.testing.assert_allclose(g, fd, rtol=0, atol=1e-8 * np.abs(G).sum())
