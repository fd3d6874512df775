"""Pins of the oracle's second-order TGV regulariser (CPU)."""
import numpy as np

from oracle import oracle as O

A0, A1 = 0.7, 1.3


def test_constant_volume_costs_nothing():
    u = np.full((5, 4, 6), 2.5)
    w = np.zeros((3, 5, 4, 6))
    assert O.tgv_value(u, w, A0, A1, 1e-3) == 0.0


def test_step_is_its_jump_area():
    """u jumps by c across one x-plane, w = 0: only that plane of forward differences is
    nonzero, so TGV = alpha1 * ny * nz * |c|_eps."""
    u = np.zeros((6, 4, 5))
    u[3:] = 2.0
    eps = 1e-2
    val = O.tgv_value(u, np.zeros((3,) + u.shape), A0, A1, eps)
    assert abs(val - A1 * 4 * 5 * (np.sqrt(4.0 + eps ** 2) - eps)) <= 1e-12


def test_affine_field_in_the_kernel_of_the_second_term():
    """w linear along one axis has a constant symmetrised gradient: |E|_F^2 = beta^2 / 2 on
    every voxel past the first plane of that axis; a constant w has E = 0."""
    u = np.zeros((5, 6, 4))
    x = np.arange(6, dtype=float)[None, :, None] * np.ones(u.shape)
    w = np.zeros((3,) + u.shape)
    w[2] = 0.3 * x                               # w_z grows along y
    eps = 1e-3
    val = O.tgv_value(u, w, A0, 0.0, eps)
    assert abs(val - A0 * 5 * 5 * 4 * (np.sqrt(0.09 / 2 + eps ** 2) - eps)) <= 1e-12
    w_const = np.ones((3,) + u.shape) * np.array([0.2, -0.1, 0.4])[:, None, None, None]
    assert O.tgv_value(u, w_const, A0, 0.0, eps) == 0.0


def test_positive_homogeneity_without_smoothing():
    rng = np.random.default_rng(0)
    u, w = rng.normal(size=(4, 5, 3)), rng.normal(size=(3, 4, 5, 3))
    v1 = O.tgv_value(u, w, A0, A1, 0.0)
    v2 = O.tgv_value(2.5 * u, 2.5 * w, A0, A1, 0.0)
    assert abs(v2 - 2.5 * v1) <= 1e-12 * v2


def test_gradients_finite_differences():
    rng = np.random.default_rng(1)
    u, w = rng.normal(size=(4, 3, 5)), 0.5 * rng.normal(size=(3, 4, 3, 5))
    eps = 0.05
    gu, gw = O.tgv_grad(u, w, A0, A1, eps)
    h = 1e-6
    fu = np.zeros_like(u)
    for i in np.ndindex(u.shape):
        up, um = u.copy(), u.copy()
        up[i] += h
        um[i] -= h
        fu[i] = (O.tgv_value(up, w, A0, A1, eps) - O.tgv_value(um, w, A0, A1, eps)) / (2 * h)
    fw = np.zeros_like(w)
    for i in np.ndindex(w.shape):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fw[i] = (O.tgv_value(u, wp, A0, A1, eps) - O.tgv_value(u, wm, A0, A1, eps)) / (2 * h)
    assert np.max(np.abs(gu - fu)) <= 1e-7 * np.max(np.abs(gu))
    assert np.max(np.abs(gw - fw)) <= 1e-7 * np.max(np.abs(gw))
