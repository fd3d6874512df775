"""Stages 3 and 4 of PA-SFM: robust rigid-array estimation and global differentiable
fine-tuning.

Stage 3 fits the array template to the noisy per-element positions of Stage 2 with a RANSAC
whose samples first pass a geometric consistency check (their pairwise distances must match
the template's) before the Kabsch fit; it returns the rigid pose and the inlier set.  This is
host logic on a few hundred 3-D points (SVDs of 3x3 matrices).

Stage 4 refines the pose, parameterised by Euler angles and a translation, against the
measured signals of the inliers only: the loss is the negative correlation summed over the
inlier elements (``nc_loss_and_grad`` with 0/1 weights), and its gradient reaches the six pose
parameters through the rigid chain (``grad_pose``) and the Euler map, both in the library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L


def kabsch(P, Q, w=None):
    """Rotation R and translation t minimising sum_i w_i |R P_i + t - Q_i|^2 (P, Q: [n, 3]),
    by the SVD of the weighted cross-covariance with the reflection excluded."""
    P, Q = np.asarray(P, dtype=np.float64), np.asarray(Q, dtype=np.float64)
    w = np.ones(len(P)) if w is None else np.asarray(w, dtype=np.float64)
    ws = w.sum()
    cp, cq = (w[:, None] * P).sum(0) / ws, (w[:, None] * Q).sum(0) / ws
    H = (w[:, None] * (P - cp)).T @ (Q - cq)
    U, _, Vt = np.linalg.svd(H)
    d = np.sign(np.linalg.det(Vt.T @ U.T))
    R = Vt.T @ np.diag([1.0, 1.0, d]) @ U.T
    return R, cq - R @ cp


def ransac_rigid(template, observed, threshold: float, iterations: int = 2000, sample: int = 3,
                 edge_tol: float = None, seed: int = 0):
    """Stage 3: RANSAC fit of `template` [M,3] onto `observed` [M,3].  A random sample of
    `sample` elements is kept only if every pairwise distance of its observed points is within
    `edge_tol` (default: threshold) of the template's; survivors are fitted by Kabsch and scored
    by the number of elements within `threshold` of the fitted template.  The best consensus is
    refitted on its inliers.  Returns (R, t, inlier mask, number of samples that reached Kabsch)."""
    template, observed = np.asarray(template, np.float64), np.asarray(observed, np.float64)
    M = len(template)
    tol = threshold if edge_tol is None else edge_tol
    rng = np.random.default_rng(seed)
    best, fitted = None, 0
    for _ in range(iterations):
        idx = rng.choice(M, size=sample, replace=False)
        a, b = np.triu_indices(sample, 1)
        dt = np.linalg.norm(template[idx[a]] - template[idx[b]], axis=1)
        do = np.linalg.norm(observed[idx[a]] - observed[idx[b]], axis=1)
        if np.any(np.abs(dt - do) > tol):
            continue
        fitted += 1
        R, t = kabsch(template[idx], observed[idx])
        inl = np.linalg.norm(template @ R.T + t - observed, axis=1) < threshold
        if best is None or inl.sum() > best.sum():
            best = inl
    if best is None or best.sum() < 3:
        raise RuntimeError("RANSAC found no consistent sample")
    for _ in range(2):                      # refit on the consensus, then re-select once
        R, t = kabsch(template[best], observed[best])
        best = np.linalg.norm(template @ R.T + t - observed, axis=1) < threshold
    R, t = kabsch(template[best], observed[best])
    return R, t, best, fitted


def euler_from_matrix(R) -> np.ndarray:
    """Angles a with R = Rz(a2) Ry(a1) Rx(a0) (away from a1 = +-pi/2)."""
    R = np.asarray(R, dtype=np.float64)
    a1 = -np.arcsin(np.clip(R[2, 0], -1.0, 1.0))
    a0 = np.arctan2(R[2, 1], R[2, 2])
    a2 = np.arctan2(R[1, 0], R[0, 0])
    return np.array([a0, a1, a2])


def finetune(grid: L.Grid, p0, samp: L.Sampling, y, template, euler6, inliers, steps: int = 100,
             lr_angle: float = 1e-3, lr_t: float = 1e-5, ctx: L.Context = None, history=None):
    """Stage 4: Adam on (Euler angles, translation) of one array pose against the measured
    signals y [M, K] (float32), with the NC loss masked to the inlier elements.  Returns the
    refined pose6 (float64 [6], device)."""
    dev = p0.device
    M = template.shape[0]
    elem = torch.as_tensor(template, dtype=torch.float64, device=dev).contiguous()
    wt = torch.as_tensor(np.asarray(inliers, dtype=np.float32), device=dev).reshape(1, M).contiguous()
    yb = y.reshape(1, M, samp.K).contiguous()
    a = torch.as_tensor(np.asarray(euler6[:3]), dtype=torch.float64, device=dev).clone().requires_grad_(True)
    t = torch.as_tensor(np.asarray(euler6[3:]), dtype=torch.float64, device=dev).clone().requires_grad_(True)
    opt = torch.optim.Adam([{"params": [a], "lr": lr_angle}, {"params": [t], "lr": lr_t}])
    gpose = torch.empty((1, 12), dtype=torch.float64, device=dev)
    for _ in range(steps):
        p6 = torch.cat([a.detach(), t.detach()]).reshape(1, 6).contiguous()
        poses = L.pose_from_euler(p6, ctx=ctx)
        loss = L.nc_loss_and_grad(grid, p0, elem, poses, samp, yb, weight=wt, grad_pose=gpose, ctx=ctx)
        g6 = L.pose_grad_euler(p6, gpose, ctx=ctx)[0]
        a.grad, t.grad = g6[:3].clone(), g6[3:].clone()
        opt.step()
        if history is not None:
            history.append(loss)
    return torch.cat([a.detach(), t.detach()])
