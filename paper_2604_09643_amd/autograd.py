"""torch.autograd integration of the radiation library.

The paper wraps its forward and backward kernels in a ``torch.autograd.Function``
so that gradients flow to both the source intensity and the sensor coordinates
(section "Differentiable Acoustic Radiation").  Here the parameters are the
volume p0 and one 6-DoF pose per frame (axis-angle w, translation t; the array
is rigid, Stage 4).  Every arithmetic step runs in the library:
``ra_pose_from_axis_angle`` builds R from w, ``radiate_forward`` and
``radiate_adjoint`` / ``loss_and_grad`` evaluate the model and its adjoint, and
``ra_pose_grad_axis_angle`` chains dL/dR to dL/dw.

``RadiateFn`` returns the signals themselves (they are kept for autograd).
``ChunkedSweepLoss`` evaluates the Stage 1 objective sum (s - y)^2 over a long
sweep frame chunk by frame chunk.  When the sweep's signals fit a device-memory
budget (``KEEP_SIGNAL_BYTES``, 16 GiB: the 256 frames of a 128-element array at
K = 2048 take 268 MB), its forward keeps them and the backward takes each chunk's
residual and adjoint from them (``RA_SIGNALS_GIVEN``), so a step runs the forward
once.  Above the budget (or with ``keep_signals=False``) the forward stores no
signals and the backward recomputes each chunk (forward, residual, adjoint);
memory is then one chunk of signals plus the volume, not F frames of signals.
Either way dL/dp0 accumulates in place.
"""
from __future__ import annotations

import os

import torch

from . import _lib as L


def _check_pose6(pose6):
    if pose6.dtype != torch.float64 or pose6.dim() != 2 or pose6.shape[1] != 6:
        raise ValueError("pose6 must be a float64 [F, 6] tensor (axis-angle, translation)")


class RadiateFn(torch.autograd.Function):
    """s = forward(p0, poses(pose6)); gradients to p0 (float32) and pose6 (float64)."""

    @staticmethod
    def forward(ctx, p0, pose6, elem, grid: L.Grid, samp: L.Sampling):
        _check_pose6(pose6)
        p0c, pose6c = p0.contiguous(), pose6.contiguous()
        poses = L.pose_from_axis_angle(pose6c)
        s = L.radiate_forward(grid, p0c, elem, poses, samp)
        ctx.save_for_backward(p0c, pose6c, poses, elem)
        ctx.grid, ctx.samp = grid, samp
        return s

    @staticmethod
    def backward(ctx, gs):
        p0, pose6, poses, elem = ctx.saved_tensors
        want_p0, want_pose = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gp0 = torch.empty_like(p0) if want_p0 else None
        gpose = torch.empty((pose6.shape[0], 12), dtype=torch.float64, device=p0.device) if want_pose else None
        if want_p0 or want_pose:
            L.radiate_adjoint(ctx.grid, p0, elem, poses, ctx.samp, gs.contiguous(), grad_p0=gp0, grad_pose=gpose)
        g6 = L.pose_grad_axis_angle(pose6, gpose) if want_pose else None
        return gp0, g6, None, None, None


def radiate(p0, pose6, elem, grid: L.Grid, samp: L.Sampling):
    return RadiateFn.apply(p0, pose6, elem, grid, samp)


KEEP_SIGNAL_BYTES = 16 << 30


class ChunkedSweepLoss(torch.autograd.Function):
    """L = sum_f sum (s_f - y_f)^2 over frame chunks; the backward takes the kept signals or
    recomputes them chunk by chunk."""

    @staticmethod
    def forward(ctx, p0, pose6, y, elem, grid: L.Grid, samp: L.Sampling, chunk: int, keep_signals=None):
        _check_pose6(pose6)
        p0c, pose6c, yc = p0.contiguous(), pose6.contiguous(), y.contiguous()
        F = pose6c.shape[0]
        keep = (4 * yc.numel() <= KEEP_SIGNAL_BYTES) if keep_signals is None else bool(keep_signals)
        sig = torch.empty_like(yc) if keep else None
        # each chunk's loss is written on the device (no host synchronisation per chunk)
        parts = torch.empty((F + chunk - 1) // chunk, dtype=torch.float64, device=p0.device)
        for i, f0 in enumerate(range(0, F, chunk)):
            f1 = min(F, f0 + chunk)
            poses = L.pose_from_axis_angle(pose6c[f0:f1])
            L.loss_and_grad(grid, p0c, elem, poses, samp, yc[f0:f1], loss_out=parts[i:i + 1],
                            s_out=sig[f0:f1] if keep else None)
        ctx.save_for_backward(p0c, pose6c, yc, elem, sig)
        ctx.grid, ctx.samp, ctx.chunk = grid, samp, chunk
        return parts.sum()

    @staticmethod
    def backward(ctx, gL):
        p0, pose6, y, elem, sig = ctx.saved_tensors
        want_p0, want_pose = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        F = pose6.shape[0]
        gp0 = torch.zeros_like(p0) if want_p0 else None
        g6 = torch.empty((F, 6), dtype=torch.float64, device=p0.device) if want_pose else None
        for f0 in range(0, F, ctx.chunk):
            f1 = min(F, f0 + ctx.chunk)
            poses = L.pose_from_axis_angle(pose6[f0:f1])
            gpose = torch.zeros((f1 - f0, 12), dtype=torch.float64, device=p0.device) if want_pose else None
            L.loss_and_grad(ctx.grid, p0, elem, poses, ctx.samp, y[f0:f1], want_loss=False, grad_p0=gp0,
                            grad_pose=gpose, accumulate=True, s_out=sig[f0:f1] if sig is not None else None,
                            signals_given=sig is not None)
            if want_pose:
                L.pose_grad_axis_angle(pose6[f0:f1], gpose, grad6=g6[f0:f1])
        if gL is not None and not bool(gL == 1):
            gp0 = gp0 * gL.to(gp0.dtype) if gp0 is not None else None
            g6 = g6 * gL if g6 is not None else None
        return gp0, g6, None, None, None, None, None, None


def sweep_loss(p0, pose6, y, elem, grid: L.Grid, samp: L.Sampling, chunk: int = 16, keep_signals=None):
    """Stage 1 objective over a sweep.  keep_signals: None keeps the signals for the backward
    when they fit KEEP_SIGNAL_BYTES; True / False force keeping / recomputing."""
    return ChunkedSweepLoss.apply(p0, pose6, y, elem, grid, samp, chunk, keep_signals)


def joint_optimise(p0, pose6, y, elem, grid: L.Grid, samp: L.Sampling, steps: int = 50, chunk: int = 16,
                   lr_p0: float = 1e-2, lr_t: float = 2e-5, lr_w: float = 2e-3, callback=None,
                   checkpoint: str = None, checkpoint_every: int = 0, resume: str = None, keep_signals=None):
    """Joint Adam optimisation of the volume and the per-frame poses against measured
    signals y (Stage 1 objective without regulariser, with free poses).  Returns the
    optimised (p0, pose6) and the loss history.

    With `checkpoint` (a file path) and checkpoint_every = N > 0, the state (volume, rotation and
    translation parameters, Adam's moments and step, the loss history) is written with torch.save
    after every N-th step and after the last, through a temporary file so that an interrupted
    write leaves the previous checkpoint whole.  `resume` (a file written so) restarts from that
    state; `steps` counts all steps, those before the checkpoint included.  A resumed run takes
    the steps the uninterrupted one would have, up to the rounding of the forward's atomic row
    adds.  `keep_signals` is passed to sweep_loss."""
    p = p0.detach().clone().requires_grad_(True)
    w = pose6[:, :3].detach().clone().requires_grad_(True)
    t = pose6[:, 3:].detach().clone().requires_grad_(True)
    opt = torch.optim.Adam([{"params": [p], "lr": lr_p0}, {"params": [w], "lr": lr_w},
                            {"params": [t], "lr": lr_t}])
    history = []
    start = 0
    if resume is not None:
        st = torch.load(resume, map_location=p.device, weights_only=True)
        if tuple(st["p0"].shape) != tuple(p.shape) or tuple(st["w"].shape) != tuple(w.shape):
            raise ValueError("checkpoint %s holds another problem's shapes" % resume)
        with torch.no_grad():
            p.copy_(st["p0"])
            w.copy_(st["w"])
            t.copy_(st["t"])
        opt.load_state_dict(st["adam"])
        history = [float(v) for v in st["history"]]
        start = int(st["step"])
    for it in range(start, steps):
        opt.zero_grad(set_to_none=True)
        loss = sweep_loss(p, torch.cat([w, t], dim=1), y, elem, grid, samp, chunk, keep_signals)
        loss.backward()
        opt.step()
        history.append(float(loss.detach()))
        if callback is not None:
            callback(it, history[-1])
        if checkpoint is not None and checkpoint_every > 0 and ((it + 1) % checkpoint_every == 0 or it + 1 == steps):
            state = {"p0": p.detach(), "w": w.detach(), "t": t.detach(), "adam": opt.state_dict(),
                     "step": it + 1, "history": list(history)}
            tmp = checkpoint + ".tmp"
            torch.save(state, tmp)
            os.replace(tmp, checkpoint)
    return p.detach(), torch.cat([w, t], dim=1).detach(), history


def reconstruct(p0, pose6, y, elem, grid: L.Grid, samp: L.Sampling, steps: int = 50, lr: float = 1e-2,
                lam: float = 0.0, alpha0: float = 2.0, alpha1: float = 1.0, eps: float = 1e-3, chunk: int = 16,
                callback=None):
    """Stages 1 and 5: argmin over p0 of sum (F(p0, X) - S)^2 + lam TGV(p0) with the poses known
    (axis-angle pose6 [F, 6]).  Adam on p0 and, when lam > 0, on TGV's auxiliary field w
    [3, nx, ny, nz]; the data term is taken frame chunk by frame chunk (loss_and_grad, dL/dp0
    accumulated in place) and the regulariser's gradient is added by tgv_loss_and_grad.
    Returns (p0, w or None)."""
    p = p0.detach().clone().contiguous().requires_grad_(True)
    params = [p]
    wv = None
    if lam > 0.0:
        wv = torch.zeros((3,) + tuple(p.shape), dtype=torch.float32, device=p.device, requires_grad=True)
        params.append(wv)
    opt = torch.optim.Adam(params, lr=lr)
    F = pose6.shape[0]
    poses = [(f0, min(F, f0 + chunk), L.pose_from_axis_angle(pose6[f0:min(F, f0 + chunk)].contiguous()))
             for f0 in range(0, F, chunk)]
    yc = y.contiguous()
    for it in range(steps):
        gp = torch.zeros_like(p)
        total = 0.0
        for f0, f1, pc in poses:
            total += L.loss_and_grad(grid, p.detach(), elem, pc, samp, yc[f0:f1], grad_p0=gp, accumulate=True)
        if wv is not None:
            gw = torch.zeros_like(wv)
            total += L.tgv_loss_and_grad(p.detach(), wv.detach(), alpha0, alpha1, eps, scale=lam, grad_u=gp,
                                         grad_w=gw, accumulate=True)
            wv.grad = gw
        p.grad = gp
        opt.step()
        if callback is not None:
            callback(it, total)
    return p.detach(), (wv.detach() if wv is not None else None)
