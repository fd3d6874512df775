"""The three model calls captured into one HIP graph and replayed.

With scratch reserved beforehand, radiate_forward, radiate_adjoint and loss_and_grad with
RA_LOSS_ON_DEVICE launch kernels only and never synchronise, so they can be captured.  The
graph is replayed twice, with eager work, synchronisation and new input values between the
replays (the graph reads its inputs at fixed addresses); every replay is checked against the
FP64 oracle on the inputs it saw, and the first also against the eager calls.
"""
import numpy as np
import pytest

from gpu_helpers import TOL_GRAD, TOL_SIGNAL, announce, gpu_desc, oracle_desc, rel_l2, to_gpu
from oracle import oracle as O
from paper_2604_09643_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_09643_amd import _lib
    _lib.load()
    return torch


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def oracle_all(w, p0, r, y):
    og, os_ = oracle_desc(w)
    s = O.grid_forward(og, p0, w.poses, w.elem, os_)
    g_r = O.grid_adjoint_p0(og, w.poses, w.elem, os_, r)
    gp_r = O.pose_grad(w.elem, O.grid_adjoint_elem(og, p0, w.poses, w.elem, os_, r))
    Lv, res = O.loss_residual(s, y)
    g_y = O.grid_adjoint_p0(og, w.poses, w.elem, os_, res)
    gp_y = O.pose_grad(w.elem, O.grid_adjoint_elem(og, p0, w.poses, w.elem, os_, res))
    return {"s": s, "gp0": g_r, "gpose": gp_r, "L": Lv, "gp0_L": g_y, "gpose_L": gp_y}


def check(name, got, ref):
    e = {"s": rel_l2(got["s"], ref["s"]), "gp0": rel_l2(got["gp0"], ref["gp0"]),
         "gR": rel_l2(got["gpose"][:, :9], ref["gpose"][:, :9]), "gt": rel_l2(got["gpose"][:, 9:], ref["gpose"][:, 9:]),
         "L": abs(got["L"] - ref["L"]) / ref["L"], "gp0_L": rel_l2(got["gp0_L"], ref["gp0_L"]),
         "gR_L": rel_l2(got["gpose_L"][:, :9], ref["gpose_L"][:, :9]),
         "gt_L": rel_l2(got["gpose_L"][:, 9:], ref["gpose_L"][:, 9:])}
    print("[graph] %s %s" % (name, " ".join("%s=%.2e" % kv for kv in e.items())), flush=True)
    assert e["s"] <= TOL_SIGNAL and e["L"] <= 2e-5
    for k in ("gp0", "gR", "gt", "gp0_L", "gR_L", "gt_L"):
        assert e[k] <= TOL_GRAD, (name, k, e[k])


def test_capture_forward_adjoint_loss(torch_cuda):
    torch = torch_cuda
    from paper_2604_09643_amd import _lib as L
    w = W.c1()
    g, s = gpu_desc(w)
    p0, elem, poses = to_gpu(w)
    dev = p0.device
    ctx = L.context(0)
    ctx.reserve(ctx.scratch_bytes(g, w.M, w.F, s))
    rng = np.random.default_rng(3)
    r_np = [w.extra["r"].astype(np.float32), rng.normal(size=w.extra["r"].shape).astype(np.float32)]
    p_np = [w.p0.astype(np.float32), (0.7 * w.p0 + 0.1 * rng.random(w.p0.shape)).astype(np.float32)]
    og, os_ = oracle_desc(w)
    s_true = O.grid_forward(og, f32(w.p0), w.poses, w.elem, os_)
    y_np = [(-0.5 * s_true).astype(np.float32), (0.3 * s_true + 0.01 * rng.normal(size=s_true.shape)).astype(np.float32)]
    r = torch.tensor(r_np[0], device=dev)
    y = torch.tensor(y_np[0], device=dev)
    sig = torch.empty((w.F, w.M, w.K), dtype=torch.float32, device=dev)
    gp0 = torch.empty_like(p0)
    gpose = torch.empty((w.F, 12), dtype=torch.float64, device=dev)
    gp0_L = torch.empty_like(p0)
    gpose_L = torch.empty((w.F, 12), dtype=torch.float64, device=dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev)

    def calls():
        L.radiate_forward(g, p0, elem, poses, s, sig, ctx=ctx)
        L.radiate_adjoint(g, p0, elem, poses, s, r, grad_p0=gp0, grad_pose=gpose, ctx=ctx)
        L.loss_and_grad(g, p0, elem, poses, s, y, grad_p0=gp0_L, grad_pose=gpose_L, ctx=ctx, loss_out=loss)

    def read():
        torch.cuda.synchronize()
        return {"s": sig.cpu().numpy(), "gp0": gp0.cpu().numpy(), "gpose": gpose.cpu().numpy(),
                "L": float(loss.cpu()[0]), "gp0_L": gp0_L.cpu().numpy(), "gpose_L": gpose_L.cpu().numpy()}

    announce("graph: eager calls")
    calls()
    eager = read()
    graph = torch.cuda.CUDAGraph()
    announce("graph: capture")
    with torch.cuda.graph(graph):
        calls()
    for name in ("s", "gp0", "gpose", "gp0_L", "gpose_L"):
        {"s": sig, "gp0": gp0, "gpose": gpose, "gp0_L": gp0_L, "gpose_L": gpose_L}[name].fill_(-7.0)
    loss.fill_(-7.0)
    for rep in range(2):
        if rep == 1:                                     # new values at the same addresses, eager work between
            p0.copy_(torch.tensor(p_np[1], device=dev))
            r.copy_(torch.tensor(r_np[1], device=dev))
            y.copy_(torch.tensor(y_np[1], device=dev))
            _ = L.radiate_forward(g, p0, elem, poses, s, ctx=ctx)
            torch.cuda.synchronize()
        announce("graph: replay %d" % rep)
        graph.replay()
        got = read()
        ref = oracle_all(w, f32(p_np[rep]), f32(r_np[rep]), f32(y_np[rep]))
        check("replay %d" % rep, got, ref)
        if rep == 0:
            for k in ("s", "gp0", "gpose", "gp0_L", "gpose_L"):
                np.testing.assert_allclose(got[k], eager[k], rtol=1e-5, atol=1e-6 * np.abs(eager[k]).max())
            assert abs(got["L"] - eager["L"]) <= 1e-6 * abs(eager["L"])
