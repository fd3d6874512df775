"""The TGV regulariser on the GPU (through the C ABI) against the FP64 oracle, and the Stage 1
reconstruction objective with it."""
import numpy as np
import pytest

from gpu_helpers import TOL_GRAD, announce, rel_l2
from oracle import oracle as O

pytestmark = pytest.mark.gpu
A0, A1 = 0.6, 1.1


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_09643_amd import _lib
    _lib.load()
    return torch


@pytest.mark.parametrize("shape,eps", [((13, 7, 11), 1e-2), ((64, 48, 40), 1e-3), ((1, 5, 9), 1e-2),
                                       ((10, 9, 130), 1e-2)])
def test_tgv_parity(torch_cuda, shape, eps):
    torch = torch_cuda
    from paper_2604_09643_amd import _lib as L
    rng = np.random.default_rng(sum(shape))
    u = rng.normal(size=shape).astype(np.float32)
    u[shape[0] // 2:] += 3.0                        # an edge
    w = (0.3 * rng.normal(size=(3,) + shape)).astype(np.float32)
    ut, wt = torch.tensor(u, device="cuda:0"), torch.tensor(w, device="cuda:0")
    gu = torch.empty_like(ut)
    gw = torch.empty_like(wt)
    announce("tgv %s" % (shape,))
    val = L.tgv_loss_and_grad(ut, wt, A0, A1, eps, scale=0.5, grad_u=gu, grad_w=gw)
    ref = 0.5 * O.tgv_value(u, w, A0, A1, eps)
    gu_ref, gw_ref = O.tgv_grad(u, w, A0, A1, eps)
    e_u, e_w = rel_l2(gu.cpu().numpy(), 0.5 * gu_ref), rel_l2(gw.cpu().numpy(), 0.5 * gw_ref)
    print("[tgv] %s value %.9e vs %.9e, grad_u %.2e grad_w %.2e" % (shape, val, ref, e_u, e_w), flush=True)
    assert abs(val - ref) <= 1e-5 * abs(ref)
    assert e_u <= TOL_GRAD and e_w <= TOL_GRAD
    # accumulate adds scale * gradient
    L.tgv_loss_and_grad(ut, wt, A0, A1, eps, scale=2.0, want_loss=False, grad_u=gu, grad_w=gw, accumulate=True)
    assert rel_l2(gu.cpu().numpy(), 2.5 * gu_ref) <= TOL_GRAD


def test_stage1_objective_with_tgv_decreases(torch_cuda):
    """Adam on (p0, w) for the Stage 1 objective sum (s - y)^2 + lambda TGV over a 6-frame sweep."""
    torch = torch_cuda
    from paper_2604_09643_amd import autograd as A
    from paper_2604_09643_amd import _lib as L
    from paper_2604_09643_amd import workloads as W
    w = W.small(shape=(24, 20, 16), F=6, M=48, K=700, sigma=0.1e-3, h=0.1e-3)
    g = L.Grid(*w.shape, tuple(w.origin), w.spacing)
    s = L.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)
    elem = torch.tensor(w.elem, device="cuda:0")
    pose6 = torch.tensor(w.pose6, device="cuda:0")
    p_true = torch.tensor(np.clip(w.p0, 0, None).astype(np.float32), device="cuda:0")
    y = L.radiate_forward(g, p_true, elem, L.pose_from_axis_angle(pose6), s)
    announce("stage 1 with TGV")
    hist = []
    p, _ = A.reconstruct(torch.zeros_like(p_true), pose6, y, elem, g, s, steps=12, lr=0.05, lam=1e-4,
                         alpha0=2.0, alpha1=1.0, eps=1e-3, callback=lambda i, v: hist.append(v))
    print("[tgv] stage 1 objective %s" % " ".join("%.4e" % v for v in hist), flush=True)
    assert hist[-1] < 0.5 * hist[0]
