"""Stages 3 and 4 on the GPU: the Euler-angle maps against the oracle, the inlier-masked
fine-tuning of a rigid array, and the Stage 2 -> 3 -> 4 pipeline end to end."""
import numpy as np
import pytest

from gpu_helpers import announce, gpu_desc, to_gpu
from oracle import oracle as O
from paper_2604_09643_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_09643_amd import _lib as L
    L.load()
    w = W.c2()
    g, s = gpu_desc(w)
    p0, _, _ = to_gpu(w)
    return torch, L, w, g, s, p0


def test_euler_maps(env):
    torch, L, *_ = env
    rng = np.random.default_rng(6)
    pose6 = np.concatenate([rng.uniform(-2.5, 2.5, size=(8, 3)), rng.normal(scale=1e-3, size=(8, 3))], 1)
    gpose = rng.normal(size=(8, 12))
    t6 = torch.tensor(pose6, device="cuda:0")
    announce("euler maps")
    P = L.pose_from_euler(t6).cpu().numpy()
    G = L.pose_grad_euler(t6, torch.tensor(gpose, device="cuda:0")).cpu().numpy()
    np.testing.assert_allclose(P, O.poses_from_euler6(pose6), rtol=0, atol=1e-14)
    np.testing.assert_allclose(G, O.euler6_grad(pose6, gpose), rtol=0, atol=1e-12)


def scene(env, seed, n_bad):
    """A 8x8 matrix array (0.5 mm pitch) under the vessel-tree volume at a rotated and shifted
    pose; measured signals with 1% noise, `n_bad` rows replaced by noise (outliers)."""
    torch, L, w, g, s, p0 = env
    rng = np.random.default_rng(seed)
    tmpl = W.matrix_array(8, 0.5e-3)
    true6 = np.array([0.03, -0.02, 0.1, 0.2e-3, -0.3e-3, 0.1e-3])
    poses = L.pose_from_euler(torch.tensor(true6[None], device="cuda:0"))
    y = L.radiate_forward(g, p0, torch.tensor(tmpl, device="cuda:0"), poses, s)[0]
    y = y + torch.randn_like(y) * 0.01 * float(y.abs().max())
    bad = rng.choice(64, size=n_bad, replace=False)
    y[torch.as_tensor(bad, device="cuda:0")] = torch.randn((n_bad, s.K), device="cuda:0") * float(y.std())
    true_x = O.element_positions(O.poses_from_euler6(true6), tmpl)[0]
    return tmpl, true6, y.contiguous(), bad, true_x


def test_finetune_from_perturbed_pose(env):
    torch, L, w, g, s, p0 = env
    from paper_2604_09643_amd import rigid
    tmpl, true6, y, bad, true_x = scene(env, 1, 8)
    inl = np.ones(64, bool)
    inl[bad] = False
    init6 = true6 + np.array([0.01, -0.008, 0.012, 80e-6, -60e-6, 70e-6])
    announce("stage 4 fine-tuning")
    hist = []
    p6 = rigid.finetune(g, p0, s, y, tmpl, init6, inl, steps=120, lr_angle=1e-3, lr_t=1e-5, history=hist)
    x = O.element_positions(O.poses_from_euler6(p6.cpu().numpy()), tmpl)[0]
    x0 = O.element_positions(O.poses_from_euler6(init6), tmpl)[0]
    err, err0 = np.linalg.norm(x - true_x, axis=1), np.linalg.norm(x0 - true_x, axis=1)
    print("[rigid] fine-tuning: element error max %.1f um (start %.1f um), loss %.4f -> %.4f"
          % (1e6 * err.max(), 1e6 * err0.max(), hist[0], hist[-1]), flush=True)
    assert err.max() <= 10e-6 and hist[-1] < hist[0]


def test_pipeline_stage2_to_4(env):
    """Per-element localisation (coarse search + annealed refinement), RANSAC with the
    edge-length pre-check, then inlier-masked fine-tuning: every element, outliers included,
    ends within a few um of the truth, and the corrupted rows are not inliers."""
    torch, L, w, g, s, p0 = env
    from dataclasses import replace
    from paper_2604_09643_amd import localise as Z
    from paper_2604_09643_amd import rigid
    tmpl, true6, y, bad, true_x = scene(env, 2, 8)
    announce("stage 2-4 pipeline")
    sigmas = [1.5 * w.sigma, 1.25 * w.sigma, w.sigma]
    top, _ = Z.coarse_search(g, p0, replace(s, sigma=sigmas[0]), y, tmpl, half_width=0.4e-3, n_per_axis=9)
    x2 = Z.refine(g, p0, s, y, top[:, 0, :], sigmas, steps_per_sigma=20, lr=2e-5).cpu().numpy()
    R, t, inl, fitted = rigid.ransac_rigid(tmpl, x2, threshold=50e-6, iterations=400, seed=3)
    init6 = np.concatenate([rigid.euler_from_matrix(R), t])
    p6 = rigid.finetune(g, p0, s, y, tmpl, init6, inl, steps=80, lr_angle=3e-4, lr_t=3e-6)
    x = O.element_positions(O.poses_from_euler6(p6.cpu().numpy()), tmpl)[0]
    e2 = np.linalg.norm(x2 - true_x, axis=1)
    e3 = np.linalg.norm(tmpl @ R.T + t - true_x, axis=1)
    e4 = np.linalg.norm(x - true_x, axis=1)
    print("[rigid] stage 2 median %.1f um (max %.0f); stage 3 max %.1f um, %d inliers, %d Kabsch fits; "
          "stage 4 max %.1f um" % (1e6 * np.median(e2), 1e6 * e2.max(), 1e6 * e3.max(), inl.sum(), fitted,
                                   1e6 * e4.max()), flush=True)
    assert not np.any(inl[bad])
    assert e4.max() <= 10e-6
