"""Stage 2 of PA-SFM: differentiable single-element localisation against a fixed volume.

Each element of the unknown pose is placed on its own: a global coarse search scores the
positions of a lattice around a starting guess by the negative-correlation (NC) loss and keeps
the best, then gradient refinement moves every element along dL_NC/dx while the Gaussian
kernel width sigma of Eq. (1) is lowered step by step (dynamic smoothing).  All model
arithmetic (forward model, NC statistics, element adjoint) runs in the library through
``nc_loss_and_grad``; this module lays out candidates, ranks their losses on the host and
applies the optimiser step.

Elements are passed as one frame with the identity pose, so the element gradient of the
library is the gradient with respect to each element's own coordinates.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np
import torch

from . import _lib as L


def _identity(device):
    return torch.tensor([[1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0]], dtype=torch.float64,
                        device=device)


def nc_scores(grid: L.Grid, p0, samp: L.Sampling, y_rows, positions, chunk: int = 8192,
              ctx: L.Context = None):
    """L_NC of every candidate position against the measured row it stands for.
    positions float64 [N, 3]; y_rows float32 [N, K] (row n is the signal the element at
    positions[n] should explain).  Returns float64 [N] (host)."""
    dev = p0.device
    N = positions.shape[0]
    out = torch.empty(N, dtype=torch.float64, device=dev)
    ident = _identity(dev)
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        L.nc_loss_and_grad(grid, p0, positions[a:b].contiguous(), ident, samp,
                           y_rows[a:b].reshape(1, b - a, samp.K).contiguous(), want_loss=False,
                           loss_elem=out[a:b].view(1, b - a), ctx=ctx)
    return out.cpu().numpy()


def coarse_search(grid: L.Grid, p0, samp: L.Sampling, y, centres, half_width: float, n_per_axis: int,
                  top_k: int = 1, ctx: L.Context = None):
    """Global coarse search: for element m, the n^3 lattice of half-width `half_width` around
    centres[m] is scored by L_NC against y[m]; returns the top_k positions per element, best
    first (float64 [M, top_k, 3], device) and their losses (numpy [M, top_k])."""
    dev = p0.device
    M, K = y.shape[0], samp.K
    ax = np.linspace(-half_width, half_width, n_per_axis) if n_per_axis > 1 else np.zeros(1)
    offs = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    C = offs.shape[0]
    cand = (torch.as_tensor(centres, dtype=torch.float64, device=dev)[:, None, :]
            + torch.as_tensor(offs, dtype=torch.float64, device=dev)[None]).reshape(M * C, 3)
    y_rep = y.reshape(M, 1, K).expand(M, C, K).reshape(M * C, K)
    scores = nc_scores(grid, p0, samp, y_rep, cand, ctx=ctx).reshape(M, C)
    order = np.argsort(scores, axis=1, kind="stable")[:, :top_k]
    best = torch.as_tensor(order, device=dev)
    pos = cand.reshape(M, C, 3)[torch.arange(M, device=dev)[:, None], best]
    return pos, np.take_along_axis(scores, order, axis=1)


def refine(grid: L.Grid, p0, samp: L.Sampling, y, x0, sigmas, steps_per_sigma: int = 5, lr: float = 2e-5,
           weight=None, ctx: L.Context = None, history=None):
    """Gradient refinement with dynamic smoothing: for each kernel width in `sigmas` (largest
    first), `steps_per_sigma` Adam steps of every element's (x, y, z) on sum_m w_m L_NC,m, the
    step size scaled with the kernel width (lr at sigmas[0]).
    y float32 [M, K]; x0 float64 [M, 3]; returns the refined positions [M, 3]."""
    dev = p0.device
    M = x0.shape[0]
    x = x0.detach().clone().to(torch.float64).requires_grad_(True)
    opt = torch.optim.Adam([x], lr=lr)
    ident = _identity(dev)
    yb = y.reshape(1, M, samp.K).contiguous()
    ge = torch.empty((1, M, 3), dtype=torch.float64, device=dev)
    for sg in sigmas:
        s_k = replace(samp, sigma=float(sg))
        for grp in opt.param_groups:
            grp["lr"] = lr * float(sg) / float(sigmas[0])
        for _ in range(steps_per_sigma):
            loss = L.nc_loss_and_grad(grid, p0, x.detach().contiguous(), ident, s_k, yb, weight=weight,
                                      grad_elem=ge, ctx=ctx)
            x.grad = ge[0].clone()
            opt.step()
            if history is not None:
                history.append((float(sg), loss))
    return x.detach()


def localise(grid: L.Grid, p0, samp: L.Sampling, y, centres, half_width: float, n_per_axis: int,
             sigmas, steps_per_sigma: int = 5, lr: float = 2e-5, ctx: L.Context = None):
    """Stage 2 end to end: the best lattice candidate of each element, then refinement."""
    top, _ = coarse_search(grid, p0, replace(samp, sigma=float(sigmas[0])), y, centres, half_width,
                           n_per_axis, top_k=1, ctx=ctx)
    return refine(grid, p0, samp, y, top[:, 0, :], sigmas, steps_per_sigma, lr, ctx=ctx)
