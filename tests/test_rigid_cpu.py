"""Host logic of Stages 3 and 4: Kabsch, the RANSAC with its geometric pre-check, and the
Euler-angle extraction (CPU)."""
import numpy as np
from scipy.spatial.transform import Rotation

from oracle import oracle as O
from paper_2604_09643_amd import rigid
from paper_2604_09643_amd import workloads as W


def test_kabsch_exact_and_weighted():
    rng = np.random.default_rng(0)
    P = rng.normal(size=(20, 3))
    R = Rotation.random(random_state=1).as_matrix()
    t = np.array([0.3, -1.0, 2.0])
    Q = P @ R.T + t
    R1, t1 = rigid.kabsch(P, Q)
    np.testing.assert_allclose(R1, R, atol=1e-12)
    np.testing.assert_allclose(t1, t, atol=1e-12)
    Q2 = Q.copy()
    Q2[:5] += 10.0                             # zero weight: ignored entirely
    w = np.ones(20)
    w[:5] = 0.0
    R2, t2 = rigid.kabsch(P, Q2, w)
    np.testing.assert_allclose(R2, R, atol=1e-12)
    np.testing.assert_allclose(t2, t, atol=1e-12)


def test_kabsch_never_returns_a_reflection():
    rng = np.random.default_rng(2)
    P = rng.normal(size=(10, 3))
    Q = P * np.array([1.0, 1.0, -1.0])         # a mirror image: best proper rotation, det = +1
    R, _ = rigid.kabsch(P, Q)
    assert abs(np.linalg.det(R) - 1.0) < 1e-12


def test_euler_round_trip():
    rng = np.random.default_rng(3)
    for a in rng.uniform([-3, -1.4, -3], [3, 1.4, 3], size=(20, 3)):
        np.testing.assert_allclose(rigid.euler_from_matrix(O.euler_rotation(a)), a, atol=1e-12)


def test_ransac_with_outliers():
    """8x8 matrix array, 40% of the positions replaced by gross errors, 10 um noise on the rest.
    (A linear array leaves the roll about its own axis to the small off-axis spread: a
    2-D array fixes all three angles.)"""
    rng = np.random.default_rng(4)
    tmpl = W.matrix_array(8, 0.5e-3)
    R = Rotation.from_euler("xyz", [0.05, -0.08, 0.3]).as_matrix()
    t = np.array([1e-3, -2e-3, 0.5e-3])
    obs = tmpl @ R.T + t + rng.normal(scale=10e-6, size=(64, 3))
    bad = rng.choice(64, size=26, replace=False)
    obs[bad] += rng.normal(scale=1e-3, size=(26, 3))
    R1, t1, inl, fitted = rigid.ransac_rigid(tmpl, obs, threshold=60e-6, iterations=500, seed=5)
    truth = np.ones(64, bool)
    truth[bad] = False
    assert np.array_equal(inl, truth)
    assert np.linalg.norm(Rotation.from_matrix(R1 @ R.T).as_rotvec()) < 2e-3
    assert np.linalg.norm(tmpl @ R1.T + t1 - (tmpl @ R.T + t), axis=1).max() < 20e-6
    assert fitted < 500                         # the edge-length check rejected samples before any SVD
