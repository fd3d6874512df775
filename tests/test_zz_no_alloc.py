"""radiate_forward_static: the forward model with its scratch in the library's static per-device
array (no allocation), against radiate_forward on the same inputs.

Two calls in a row, the second on a smaller input (so stale contents of the shared array from
the first call would show), the first with FP64 sums in the static array, the second with FP32
sums; both also against the FP64 oracle.  A request larger than the array is refused with
RA_ENOMEM, and a fresh context with no scratch of its own can capture the call into a HIP graph
(the call allocates nothing), replayed twice with new values in between.
"""
import numpy as np
import pytest

from gpu_helpers import TOL_SIGNAL, announce, gpu_desc, oracle_desc, rel_l2, to_gpu
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


def run_pair(torch, L, ctx, w, mode):
    """radiate_forward_static and radiate_forward with forward sums `mode`; both outputs."""
    g, s = gpu_desc(w)
    p0, elem, poses = to_gpu(w)
    out_static = torch.full((w.F, w.M, w.K), -3.0, dtype=torch.float32, device=p0.device)
    ctx.set_forward_sums(mode)
    try:
        announce("no-alloc forward %s %s F=%d M=%d K=%d mode %d" % (w.name, w.shape, w.F, w.M, w.K, mode))
        L.radiate_forward_static(g, p0, elem, poses, s, out_static, ctx=ctx)
        ref = L.radiate_forward(g, p0, elem, poses, s, ctx=ctx)
        torch.cuda.synchronize()
    finally:
        ctx.set_forward_sums(L.RA_SUMS_AUTO)
    return out_static.cpu().numpy(), ref.cpu().numpy()


def test_static_forward_two_calls(torch_cuda):
    torch = torch_cuda
    from paper_2604_09643_amd import _lib as L
    ctx = L.Context(0)
    big = W.small(seed=4, shape=(40, 36, 24), h=0.1 * W.MM, M=64, F=6, K=900, sigma=0.08 * W.MM)
    little = W.small(seed=5, shape=(13, 11, 9), h=0.1 * W.MM, M=24, F=2, K=700, sigma=0.08 * W.MM)
    for w, mode in ((big, L.RA_SUMS_F64), (little, L.RA_SUMS_F32)):
        got, ref = run_pair(torch, L, ctx, w, mode)
        og, os_ = oracle_desc(w)
        s_or = O.grid_forward(og, f32(w.p0), w.poses, w.elem, os_)
        e_ref, e_or = rel_l2(got, ref), rel_l2(got, s_or)
        print("[no-alloc] %s: vs radiate_forward %.2e, vs oracle %.2e (radiate_forward vs oracle %.2e)"
              % (w.shape, e_ref, e_or, rel_l2(ref, s_or)), flush=True)
        assert e_ref <= TOL_SIGNAL and e_or <= TOL_SIGNAL


def test_static_forward_refuses_oversize(torch_cuda):
    torch = torch_cuda
    from paper_2604_09643_amd import _lib as L
    ctx = L.Context(0)
    w = W.c2()                                   # FP64 sums of 64 x 128 x 1024 samples: 64 MiB
    g, s = gpu_desc(w)
    p0, elem, poses = to_gpu(w)
    out = torch.empty((w.F, w.M, w.K), dtype=torch.float32, device=p0.device)
    ctx.set_forward_sums(L.RA_SUMS_F64)
    try:
        with pytest.raises(L.RadiateError) as ei:
            L.radiate_forward_static(g, p0, elem, poses, s, out, ctx=ctx)
    finally:
        ctx.set_forward_sums(L.RA_SUMS_AUTO)
    assert ei.value.code == L.RA_ENOMEM and "static array" in str(ei.value)
    announce("no-alloc forward at C2 size with FP32 sums")
    L.radiate_forward_static(g, p0, elem, poses, s, out, ctx=ctx)        # fits: 24 B per element
    ref = L.radiate_forward(g, p0, elem, poses, s, ctx=ctx)
    torch.cuda.synchronize()
    e = rel_l2(out.cpu().numpy(), ref.cpu().numpy())
    print("[no-alloc] C2 FP32 sums vs radiate_forward %.2e" % e, flush=True)
    assert e <= TOL_SIGNAL


def test_static_forward_under_capture(torch_cuda):
    torch = torch_cuda
    from paper_2604_09643_amd import _lib as L
    w = W.small(seed=6, shape=(17, 15, 12), h=0.1 * W.MM, M=32, F=3, K=800, sigma=0.08 * W.MM)
    g, s = gpu_desc(w)
    p0, elem, poses = to_gpu(w)
    out = torch.empty((w.F, w.M, w.K), dtype=torch.float32, device=p0.device)
    warm = L.Context(0)
    L.radiate_forward_static(g, p0, elem, poses, s, out, ctx=warm)       # sets the kernels' LDS limit
    torch.cuda.synchronize()
    ctx = L.Context(0)                            # no scratch of its own: capture must not allocate
    graph = torch.cuda.CUDAGraph()
    announce("no-alloc forward: capture")
    with torch.cuda.graph(graph):
        L.radiate_forward_static(g, p0, elem, poses, s, out, ctx=ctx)
    og, os_ = oracle_desc(w)
    rng = np.random.default_rng(8)
    for rep in range(2):
        vol = w.p0 if rep == 0 else 0.6 * w.p0 + 0.2 * rng.random(w.p0.shape)
        p0.copy_(torch.tensor(vol.astype(np.float32), device=p0.device))
        out.fill_(-5.0)
        _ = L.radiate_forward(g, p0, elem, poses, s)                        # eager work between replays
        torch.cuda.synchronize()
        announce("no-alloc forward: replay %d" % rep)
        graph.replay()
        torch.cuda.synchronize()
        e = rel_l2(out.cpu().numpy(), O.grid_forward(og, f32(vol), w.poses, w.elem, os_))
        print("[no-alloc] replay %d vs oracle %.2e" % (rep, e), flush=True)
        assert e <= TOL_SIGNAL
