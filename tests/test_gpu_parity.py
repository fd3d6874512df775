"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Inputs are the seeded workloads; the oracle sees the same FP64 geometry and the
FP32-rounded volume and residuals that the GPU receives.  Bars: relative L2
<= 1e-5 on signals, <= 1e-4 on each gradient (rotation and translation blocks
of the pose gradient separately).
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


def run_all(torch, w, r=None, name=""):
    """GPU forward, adjoint (p0, pose, elem) for workload w with residual r; returns numpy."""
    from paper_2604_09643_amd import _lib as L
    g, s = gpu_desc(w)
    p0, elem, poses = to_gpu(w)
    announce("%s forward shape=%s F=%d M=%d K=%d" % (name, w.shape, w.F, w.M, w.K))
    sig = L.radiate_forward(g, p0, elem, poses, s)
    torch.cuda.synchronize()
    out = {"s": sig.cpu().numpy().astype(np.float64)}
    if r is not None:
        rt = torch.tensor(r.astype(np.float32), device="cuda:0").contiguous()
        gp0 = torch.empty_like(p0)
        gpose = torch.empty((w.F, 12), dtype=torch.float64, device="cuda:0")
        gelem = torch.empty((w.F, w.M, 3), dtype=torch.float64, device="cuda:0")
        announce("%s adjoint" % name)
        L.radiate_adjoint(g, p0, elem, poses, s, rt, grad_p0=gp0, grad_pose=gpose, grad_elem=gelem)
        torch.cuda.synchronize()
        out.update(gp0=gp0.cpu().numpy().astype(np.float64), gpose=gpose.cpu().numpy(),
                   gelem=gelem.cpu().numpy())
        announce("%s adjoint p0 only" % name)
        gp0b = torch.empty_like(p0)
        L.radiate_adjoint(g, p0, elem, poses, s, rt, grad_p0=gp0b)
        torch.cuda.synchronize()
        out["gp0_only"] = gp0b.cpu().numpy().astype(np.float64)
    return out


def check_full(w, out, r):
    og, os_ = oracle_desc(w)
    p0 = f32(w.p0)
    s_ref = O.grid_forward(og, p0, w.poses, w.elem, os_)
    errs = {"s": rel_l2(out["s"], s_ref)}
    if r is not None:
        r32 = f32(r)
        g_ref = O.grid_adjoint_p0(og, w.poses, w.elem, os_, r32)
        ge_ref = O.grid_adjoint_elem(og, p0, w.poses, w.elem, os_, r32)
        gp_ref = O.pose_grad(w.elem, ge_ref)
        errs.update(gp0=rel_l2(out["gp0"], g_ref), gp0_only=rel_l2(out["gp0_only"], g_ref),
                    gelem=rel_l2(out["gelem"], ge_ref), gR=rel_l2(out["gpose"][:, :9], gp_ref[:, :9]),
                    gt=rel_l2(out["gpose"][:, 9:], gp_ref[:, 9:]))
    print("[parity] %s %s" % (w.name, " ".join("%s=%.2e" % kv for kv in errs.items())), flush=True)
    assert errs["s"] <= TOL_SIGNAL
    for k in ("gp0", "gp0_only", "gelem", "gR", "gt"):
        if k in errs:
            assert errs[k] <= TOL_GRAD, (k, errs[k])


def test_c1_full(torch_cuda):
    """Plain forward + adjoint at the 32^3 / 64-element / K=512 configuration, every output."""
    w = W.c1()
    r = w.extra["r"]
    out = run_all(torch_cuda, w, r, "C1")
    check_full(w, out, r)


@pytest.mark.parametrize("shape,F,M,K,sigma", [((9, 7, 5), 2, 5, 400, 1e-4),
                                               ((13, 11, 17), 3, 7, 700, 0.08e-3),
                                               ((20, 3, 9), 1, 66, 500, 0.15e-3),
                                               ((11, 9, 10), 2, 9, 600, 0.2e-3),
                                               ((8, 6, 7), 1, 65, 700, 0.25e-3),
                                               ((10, 8, 6), 2, 9, 500, 0.07e-3),
                                               ((10, 8, 6), 2, 9, 500, 0.06e-3)])
def test_small_ragged(torch_cuda, shape, F, M, K, sigma):
    """Grids that do not divide into regions, several jittered frames, element counts that
    leave a partial 64-lane chunk, and window half-widths 16, 12, 23 (kernels compiled for
    that width), 31 and 39 samples (the generic 32- and 40-step kernels).  sigma = 0.07 mm
    (delta/sigma = 0.55) is the narrowest kernel the adjoints' moment form admits; at 0.06 mm
    (0.64) its truncation bound fails and the Gaussian adjoints take the row forms."""
    w = W.small(shape=shape, F=F, M=M, K=K, sigma=sigma)
    r = w.extra["r"]
    out = run_all(torch_cuda, w, r, "small%s" % (shape,))
    check_full(w, out, r)


@pytest.mark.parametrize("shape,F,M,K,sigma,h", [((13, 11, 18), 3, 70, 700, 0.08e-3, 0.1e-3),
                                                 ((20, 9, 12), 2, 33, 600, 0.1e-3, 0.08e-3),
                                                 ((9, 7, 5), 2, 5, 500, 0.1e-3, 0.1e-3)])
def test_small_fine_spacing(torch_cuda, shape, F, M, K, sigma, h):
    """Spacing below three sample lengths: the forward takes z-neighbours in pairs.  The grids
    cut regions at every edge (bounds-tested path) and leave whole interior regions (untested
    path); the 9x7x5 grid has an odd region depth, where pairing is switched off."""
    w = W.small(shape=shape, F=F, M=M, K=K, sigma=sigma, h=h)
    r = w.extra["r"]
    out = run_all(torch_cuda, w, r, "fine%s" % (shape,))
    check_full(w, out, r)


@pytest.mark.parametrize("shape,F,M,K", [((1, 1, 1), 1, 1, 400), ((1, 1, 9), 1, 64, 400), ((5, 1, 1), 2, 65, 400),
                                         ((3, 4, 2), 1, 3, 37), ((2, 2, 2), 1, 2, 1)])
def test_degenerate_sizes(torch_cuda, shape, F, M, K):
    """A single voxel, single lines of voxels, one element, exactly one 64-lane chunk and one
    more than one; records too short to reach the volume (K = 37 and K = 1: every sample of
    every window is clipped, so every output is exactly zero on both sides)."""
    from paper_2604_09643_amd import _lib as L
    w = W.small(shape=shape, F=F, M=M, K=K)
    r = w.extra["r"]
    out = run_all(torch_cuda, w, r, "degenerate%s K=%d" % (shape, K))
    og, os_ = oracle_desc(w)
    g, s = gpu_desc(w)
    _, elem, poses = to_gpu(w)
    n = L.count_updates(g, elem, poses, s)
    assert n == O.grid_count_updates(og, w.poses, w.elem, os_)
    if n == 0:
        for k in ("s", "gp0", "gp0_only", "gelem", "gpose"):
            assert np.all(out[k] == 0.0), k
        assert np.all(O.grid_forward(og, f32(w.p0), w.poses, w.elem, os_) == 0.0)
    else:
        check_full(w, out, r)


def check_sampled(torch, w, name, n_rows, n_vox, n_elem, seed=123):
    """Full-size GPU forward and adjoint, checked on outputs the oracle computes one by one:
    whole signal rows of n_rows elements, dL/dp0 of n_vox voxels, dL/dx_e of n_elem elements."""
    rng = np.random.default_rng(seed)
    r = rng.normal(size=(w.F, w.M, w.K))
    out = run_all(torch, w, r, name)
    og, os_ = oracle_desc(w)
    p0 = f32(w.p0)
    rows = rng.choice(w.F * w.M, size=n_rows, replace=False)
    s_ref = O.grid_forward(og, p0, w.poses, w.elem, os_, elements=rows)
    e_s = rel_l2(out["s"].reshape(-1, w.K)[rows], s_ref)
    vox = rng.choice(w.n_voxels, size=n_vox, replace=False)
    g_ref = O.grid_adjoint_p0(og, w.poses, w.elem, os_, f32(r), voxels=vox)
    e_g = rel_l2(out["gp0"].reshape(-1)[vox], g_ref)
    e_g1 = rel_l2(out["gp0_only"].reshape(-1)[vox], g_ref)
    els = rng.choice(w.F * w.M, size=n_elem, replace=False)
    ge_ref = O.grid_adjoint_elem(og, p0, w.poses, w.elem, os_, f32(r), elements=els)
    e_e = rel_l2(out["gelem"].reshape(-1, 3)[els], ge_ref)
    print("[parity] %s sampled s=%.2e gp0=%.2e gp0_only=%.2e gelem=%.2e" % (name, e_s, e_g, e_g1, e_e),
          flush=True)
    assert e_s <= TOL_SIGNAL and e_g <= TOL_GRAD and e_g1 <= TOL_GRAD and e_e <= TOL_GRAD


def test_c2_sampled(torch_cuda):
    """The benchmarked 128x128x64 / 64-frame / 128-element / K=1024 sweep at full size."""
    check_sampled(torch_cuda, W.c2(), "C2", n_rows=6, n_vox=256, n_elem=3)


def test_c3_chunk_sampled(torch_cuda):
    """A 16-frame chunk of the 256x256x128 (0.08 mm) / 128-element / K=2048 reconstruction,
    the unit the chunked loss processes, on the full volume."""
    check_sampled(torch_cuda, W.c3(frames=16), "C3x16", n_rows=3, n_vox=256, n_elem=2)


def test_c4_sampled(torch_cuda):
    """256^3 volume, 32x32 matrix array (1024 elements), 8 frames, K=2048: the full adjoint
    with the FP64 pose reduction at M=1024."""
    check_sampled(torch_cuda, W.c4(), "C4", n_rows=2, n_vox=256, n_elem=2)


def test_cap33_sampled(torch_cuda):
    """The 33-element spherical-cap array in three views (rotated and shifted) around a 256^3
    volume: elements facing the grid from every side, distances up to 63 mm."""
    check_sampled(torch_cuda, W.cap33(), "cap33", n_rows=3, n_vox=256, n_elem=2)


def test_hemisphere_view_sampled(torch_cuda):
    """One 512-element view of the 1024-element hemispherical array (radius 60 mm), K=2560."""
    check_sampled(torch_cuda, W.hemisphere1024(view=1), "hemi512", n_rows=2, n_vox=256, n_elem=2)


def test_reciprocity_gpu(torch_cuda):
    """<A p0, r> = <p0, A^T r> for the GPU operators (FP32 level)."""
    w = W.small(shape=(16, 16, 16), F=2, M=40, K=600)
    r = w.extra["r"]
    out = run_all(torch_cuda, w, r, "reciprocity")
    lhs = np.sum(out["s"] * f32(r))
    rhs = np.sum(f32(w.p0) * out["gp0"])
    scale = np.sum(np.abs(out["s"] * f32(r)))
    assert abs(lhs - rhs) <= 1e-6 * scale


def _model_gpu(torch, shape, origin, h, p0, poses, w, r):
    """Signals, dL/dp0 and element gradients on an explicit grid (numpy in, numpy out)."""
    from paper_2604_09643_amd import _lib as L
    g = L.Grid(*shape, tuple(origin), h)
    s = L.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)
    dev = torch.device("cuda:0")
    p0t = torch.tensor(np.ascontiguousarray(p0, dtype=np.float32), device=dev)
    elem = torch.tensor(w.elem, dtype=torch.float64, device=dev)
    post = torch.tensor(poses, dtype=torch.float64, device=dev)
    sig = L.radiate_forward(g, p0t, elem, post, s)
    rt = torch.tensor(r, device=dev)
    gp0 = torch.empty_like(p0t)
    gelem = torch.empty((w.F, w.M, 3), dtype=torch.float64, device=dev)
    L.radiate_adjoint(g, p0t, elem, post, s, rt, grad_p0=gp0, grad_elem=gelem)
    torch.cuda.synchronize()
    return sig.cpu().numpy().astype(np.float64), gp0.cpu().numpy().astype(np.float64), gelem.cpu().numpy()


def test_grid_invariance_c2(torch_cuda):
    """Rigid re-indexings of the sweep's full volume leave the model unchanged (the kernel depends on
    |x - x_e| only): (1) the voxel array rotated by 90 degrees about z with the posed arrays moved by
    the matching rigid motion gives the same signals, the rotated dL/dp0 and rotated element
    gradients; (2) the volume padded with zero voxels (an integer-voxel shift of every index, so the
    regions fall differently on the data, and ragged at the ends) with the origin moved back gives
    the same signals, dL/dp0 and element gradients."""
    torch = torch_cuda
    w = W.c2()
    r = np.random.default_rng(21).normal(size=(w.F, w.M, w.K)).astype(np.float32)
    nx, ny, nz = w.shape
    h = w.spacing
    o0 = np.asarray(w.origin, dtype=np.float64)
    announce("invariance: sweep as given")
    s0, g0, e0 = _model_gpu(torch, w.shape, o0, h, w.p0, w.poses, w, r)

    Q = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    o1 = o0 + np.array([0.7e-3, -1.3e-3, 0.4e-3])
    b = np.array([o1[0] + o0[1] + (ny - 1) * h, o1[1] - o0[0], o1[2] - o0[2]])
    poses1 = w.poses.copy()
    for f in range(w.F):
        poses1[f, :9] = (Q @ w.poses[f, :9].reshape(3, 3)).reshape(9)
        poses1[f, 9:] = Q @ w.poses[f, 9:] + b
    announce("invariance: rotated 90 degrees about z")
    s1, g1, e1 = _model_gpu(torch, (ny, nx, nz), o1, h, np.rot90(w.p0, 1, axes=(0, 1)), poses1, w, r)
    errs = {"rot s": rel_l2(s1, s0), "rot gp0": rel_l2(g1, np.rot90(g0, 1, axes=(0, 1))),
            "rot gelem": rel_l2(e1, e0 @ Q.T)}

    lo, hi = (3, 5, 2), (1, 6, 3)
    p2 = np.pad(w.p0, tuple(zip(lo, hi)))
    o2 = o0 - np.array(lo) * h
    announce("invariance: zero-padded by %s / %s voxels" % (lo, hi))
    s2, g2, e2 = _model_gpu(torch, p2.shape, o2, h, p2, w.poses, w, r)
    errs.update({"pad s": rel_l2(s2, s0),
                 "pad gp0": rel_l2(g2[lo[0]:lo[0] + nx, lo[1]:lo[1] + ny, lo[2]:lo[2] + nz], g0),
                 "pad gelem": rel_l2(e2, e0)})
    print("[parity] C2 invariance " + " ".join("%s=%.2e" % kv for kv in errs.items()), flush=True)
    for k, v in errs.items():
        assert v <= (TOL_SIGNAL if k.endswith(" s") else TOL_GRAD), (k, v)


def test_repeat_runs_c2(torch_cuda):
    """Race check by repetition at the sweep's full size: the adjoints add in a fixed order (dL/dp0
    gathered per voxel and summed over wavefronts in LDS in wavefront order; element gradients in
    FP64 per wavefront, then over regions in region order), so three runs give bitwise equal dL/dp0,
    element gradients and pose blocks; the forward's row adds are atomic, so its repeats agree to
    rounding only."""
    torch = torch_cuda
    w = W.c2()
    r = np.random.default_rng(22).normal(size=(w.F, w.M, w.K)).astype(np.float32)
    outs = []
    for i in range(3):
        announce("repeat %d" % i)
        sig, gp0, gelem = _model_gpu(torch, w.shape, w.origin, w.spacing, w.p0, w.poses, w, r)
        outs.append((sig, gp0, gelem))
    for sig, gp0, gelem in outs[1:]:
        assert np.array_equal(gp0, outs[0][1])
        assert np.array_equal(gelem, outs[0][2])
        assert rel_l2(sig, outs[0][0]) <= 1e-6
    from paper_2604_09643_amd import _lib as L
    g = L.Grid(*w.shape, tuple(w.origin), w.spacing)
    s = L.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)
    p0, elem, poses = to_gpu(w)
    rt = torch.tensor(r, device="cuda:0")
    blocks = []
    for i in range(3):
        gpose = torch.empty((w.F, 12), dtype=torch.float64, device="cuda:0")
        L.radiate_adjoint(g, p0, elem, poses, s, rt, grad_pose=gpose)
        torch.cuda.synchronize()
        blocks.append(gpose.cpu().numpy())
    assert all(np.array_equal(b, blocks[0]) for b in blocks[1:])
    print("[parity] C2 repeats: dL/dp0, element gradients and pose blocks bitwise equal; signals within "
          "%.1e" % max(rel_l2(o[0], outs[0][0]) for o in outs[1:]), flush=True)


def test_count_updates_exact(torch_cuda):
    from paper_2604_09643_amd import _lib as L
    for w in (W.c1(), W.small(shape=(13, 11, 17), F=3, M=7, K=700, sigma=0.08e-3)):
        g, s = gpu_desc(w)
        _, elem, poses = to_gpu(w)
        announce("count %s" % w.name)
        n = L.count_updates(g, elem, poses, s)
        og, os_ = oracle_desc(w)
        assert n == O.grid_count_updates(og, w.poses, w.elem, os_)


def test_axis_angle_maps(torch_cuda):
    import torch
    from paper_2604_09643_amd import _lib as L
    rng = np.random.default_rng(5)
    pose6 = np.concatenate([rng.normal(scale=0.3, size=(6, 3)), rng.normal(scale=1e-3, size=(6, 3))], axis=1)
    pose6[0, :3] = 0.0
    pose6[1, :3] = [1e-9, -2e-9, 5e-10]
    pose6[2, :3] = [0.049, 0.0, 0.001]
    pose6[3, :3] = [0.051, 0.0, -0.001]
    gpose = rng.normal(size=(6, 12))
    t6 = torch.tensor(pose6, device="cuda:0")
    announce("axis-angle maps")
    P = L.pose_from_axis_angle(t6).cpu().numpy()
    G = L.pose_grad_axis_angle(t6, torch.tensor(gpose, device="cuda:0")).cpu().numpy()
    np.testing.assert_allclose(P, O.poses_from_pose6(pose6), rtol=0, atol=1e-14)
    np.testing.assert_allclose(G, O.pose6_grad(pose6, gpose), rtol=0, atol=1e-12)


def test_loss_and_grad_c1(torch_cuda):
    import torch
    from paper_2604_09643_amd import _lib as L
    w = W.c1()
    g, s = gpu_desc(w)
    p0, elem, poses = to_gpu(w)
    og, os_ = oracle_desc(w)
    s_true = O.grid_forward(og, f32(w.p0), w.poses, w.elem, os_)
    # measured signals of a different volume plus noise: the residual is as large as the signal,
    # so the FP32 error of the forward stays small next to it
    noise = np.random.default_rng(9).normal(scale=0.05 * np.abs(s_true).max(), size=s_true.shape)
    y = (-0.5 * s_true + noise).astype(np.float32)
    yt = torch.tensor(y, device="cuda:0")
    gp0 = torch.empty_like(p0)
    gpose = torch.empty((w.F, 12), dtype=torch.float64, device="cuda:0")
    s_out = torch.empty_like(yt)
    announce("loss_and_grad C1")
    Lval = L.loss_and_grad(g, p0, elem, poses, s, yt, s_out=s_out, grad_p0=gp0, grad_pose=gpose)
    L_ref, r_ref = O.loss_residual(s_true, f32(y))
    print("[parity] loss gpu=%.10e oracle=%.10e" % (Lval, L_ref), flush=True)
    assert abs(Lval - L_ref) <= 2e-5 * L_ref
    assert rel_l2(s_out.cpu().numpy(), s_true) <= TOL_SIGNAL
    g_ref = O.grid_adjoint_p0(og, w.poses, w.elem, os_, r_ref)
    assert rel_l2(gp0.cpu().numpy(), g_ref) <= TOL_GRAD
    gp_ref = O.pose_grad(w.elem, O.grid_adjoint_elem(og, f32(w.p0), w.poses, w.elem, os_, r_ref))
    e_t = rel_l2(gpose.cpu().numpy()[:, 9:], gp_ref[:, 9:])
    e_R = rel_l2(gpose.cpu().numpy()[:, :9], gp_ref[:, :9])
    print("[parity] loss_and_grad pose gR=%.2e gt=%.2e" % (e_R, e_t), flush=True)
    assert e_t <= TOL_GRAD and e_R <= TOL_GRAD


def test_signals_given_c1(torch_cuda):
    """loss_and_grad with RA_SIGNALS_GIVEN takes the signals an earlier call wrote to s_out, leaves
    them unchanged, and gives the loss and gradients of the call that computed them (the same FP32
    signals, so the same residual), each within the bar of the oracle; without s_out the flag is
    refused."""
    torch = torch_cuda
    from paper_2604_09643_amd import _lib as L
    w = W.c1()
    g, s = gpu_desc(w)
    p0, elem, poses = to_gpu(w)
    y = torch.tensor((0.3 * w.extra["r"]).astype(np.float32), device="cuda:0")
    sig = torch.empty_like(y)
    gp0a, gp0b = torch.empty_like(p0), torch.empty_like(p0)
    gpa = torch.empty((w.F, 12), dtype=torch.float64, device="cuda:0")
    gpb = torch.empty_like(gpa)
    announce("loss_and_grad computing the signals")
    la = L.loss_and_grad(g, p0, elem, poses, s, y, s_out=sig, grad_p0=gp0a, grad_pose=gpa)
    kept = sig.clone()
    announce("loss_and_grad with the signals given")
    lb = L.loss_and_grad(g, p0, elem, poses, s, y, s_out=sig, signals_given=True, grad_p0=gp0b, grad_pose=gpb)
    torch.cuda.synchronize()
    assert torch.equal(sig, kept)
    assert abs(lb / la - 1.0) <= 1e-12
    assert torch.equal(gp0a, gp0b) and torch.equal(gpa, gpb)        # same residual, fixed-order adjoint
    og, os_ = oracle_desc(w)
    s_ref = O.grid_forward(og, f32(w.p0), w.poses, w.elem, os_)
    r_ref = 2.0 * (s_ref - f32(0.3 * w.extra["r"]))
    g_ref = O.grid_adjoint_p0(og, w.poses, w.elem, os_, r_ref)
    e = rel_l2(gp0b.cpu().numpy(), g_ref)
    print("[parity] C1 signals given: loss ratio - 1 = %.1e, dL/dp0 %.2e" % (lb / la - 1.0, e), flush=True)
    assert e <= TOL_GRAD
    import ctypes
    ctx = L.context(0)
    rc = ctx.lib.loss_and_grad(ctx.ptr, ctypes.byref(g.c()), ctypes.c_void_p(p0.data_ptr()), w.M,
                               ctypes.c_void_p(elem.data_ptr()), ctypes.c_void_p(poses.data_ptr()), w.F,
                               ctypes.byref(s.cs()), ctypes.c_void_p(y.data_ptr()), None, None, None, None, None,
                               L.RA_SIGNALS_GIVEN, None)
    assert rc == L.RA_EINVAL and b"s_out" in ctx.lib.ra_last_error(ctx.ptr)


def test_accumulate_flag(torch_cuda):
    import torch
    from paper_2604_09643_amd import _lib as L
    w = W.small(shape=(9, 7, 5), F=2, M=5, K=400)
    g, s = gpu_desc(w)
    p0, elem, poses = to_gpu(w)
    r = torch.tensor(w.extra["r"].astype(np.float32), device="cuda:0")
    a = torch.empty_like(p0)
    pa = torch.empty((w.F, 12), dtype=torch.float64, device="cuda:0")
    announce("accumulate")
    L.radiate_adjoint(g, p0, elem, poses, s, r, grad_p0=a, grad_pose=pa)
    b = a.clone() + 1.0
    pb = pa.clone() + 1.0
    L.radiate_adjoint(g, p0, elem, poses, s, r, grad_p0=b, grad_pose=pb, accumulate=True)
    torch.cuda.synchronize()
    np.testing.assert_allclose(b.cpu().numpy(), 2 * a.cpu().numpy() + 1.0, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(pb.cpu().numpy(), 2 * pa.cpu().numpy() + 1.0, rtol=1e-12, atol=1e-12)


def test_geometry_status(torch_cuda):
    """An element inside the grid box is reported as RA_EGEOM by ra_status; a clean call is OK."""
    import torch
    from paper_2604_09643_amd import _lib as L
    w = W.small(shape=(9, 7, 5), F=1, M=5, K=400)
    g, s = gpu_desc(w)
    p0, elem, poses = to_gpu(w)
    ctx = L.context(0)
    announce("geometry status")
    L.radiate_forward(g, p0, elem, poses, s)
    assert ctx.status() == L.RA_OK
    bad = poses.clone()
    bad[0, 9:] = torch.tensor(w.origin, dtype=torch.float64) + 2 * w.spacing
    L.radiate_forward(g, p0, elem, bad, s)
    assert ctx.status() == L.RA_EGEOM
    assert ctx.status() == L.RA_OK


def test_invalid_arguments(torch_cuda):
    import torch
    from paper_2604_09643_amd import _lib as L
    w = W.small(shape=(9, 7, 5), F=1, M=5, K=400)
    g, s = gpu_desc(w)
    p0, elem, poses = to_gpu(w)
    with pytest.raises(L.RadiateError) as ei:
        L.radiate_forward(g, p0, elem, poses, L.Sampling(w.c, w.fs, w.K, -1.0))
    assert ei.value.code == L.RA_EINVAL
    with pytest.raises(L.RadiateError) as ei:
        L.radiate_forward(L.Grid(0, 7, 5, tuple(w.origin), w.spacing), p0[:0], elem, poses, s)
    assert ei.value.code == L.RA_EINVAL
    with pytest.raises(L.RadiateError) as ei:   # window wider than the compiled maximum
        L.radiate_forward(g, p0, elem, poses, L.Sampling(w.c, w.fs, w.K, 100 * w.sigma))
    assert ei.value.code == L.RA_EINVAL


def _fixture_module():
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_c4_pose_fixture.py")
    spec = importlib.util.spec_from_file_location("make_c4_pose_fixture", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _pose_block_errors(name, gpose, gelem, gp_ref, ge_ref):
    e = {"gR": rel_l2(gpose[:, :9], gp_ref[:, :9]), "gt": rel_l2(gpose[:, 9:], gp_ref[:, 9:]),
         "gelem": rel_l2(gelem, ge_ref)}
    print("[parity] %s whole frames %s" % (name, " ".join("%s=%.2e" % kv for kv in e.items())), flush=True)
    for k, v in e.items():
        assert v <= TOL_GRAD, (name, k, v)


def test_c2_pose_blocks_whole_frames(torch_cuda):
    """The benchmarked sweep at full size (a million voxels, 64 frames): every element gradient of
    two whole frames and their dL/dR, dL/dt blocks, the FP64 reduction over all regions of the
    volume, against the oracle."""
    import torch
    from paper_2604_09643_amd import _lib as L
    w = W.c2()
    g, s = gpu_desc(w)
    p0, elem, poses = to_gpu(w)
    r = np.random.default_rng(31).normal(size=(w.F, w.M, w.K)).astype(np.float32)
    gpose = torch.empty((w.F, 12), dtype=torch.float64, device="cuda:0")
    gelem = torch.empty((w.F, w.M, 3), dtype=torch.float64, device="cuda:0")
    announce("C2 pose blocks: adjoint with element gradients")
    L.radiate_adjoint(g, p0, elem, poses, s, torch.tensor(r, device="cuda:0"), grad_pose=gpose, grad_elem=gelem)
    torch.cuda.synchronize()
    frames = np.array([5, 40])
    og, os_ = oracle_desc(w)
    els = (frames[:, None] * w.M + np.arange(w.M)[None, :]).reshape(-1)
    ge_ref = O.grid_adjoint_elem(og, f32(w.p0), w.poses, w.elem, os_, r.astype(np.float64), elements=els)
    ge_ref = ge_ref.reshape(len(frames), w.M, 3)
    gp_ref = O.pose_grad(w.elem, ge_ref)
    _pose_block_errors("C2 frames %s" % list(frames), gpose.cpu().numpy()[frames], gelem.cpu().numpy()[frames],
                       gp_ref, ge_ref)


def test_c4_subarray_pose_blocks(torch_cuda):
    """The 256^3 matrix-array configuration at full volume size, one frame of a 16 x 8 block of the
    32 x 32 array: element gradients and the frame's dL/dR, dL/dt against the oracle's values
    stored by tests/golden/make_c4_pose_fixture.py (16.7 million voxels per element)."""
    import torch
    from paper_2604_09643_amd import _lib as L
    fx = _fixture_module()
    w, elem_np, poses_np, r = fx.inputs()
    ge_ref, gp_ref = fx.load()
    g, s = gpu_desc(w)
    dev = torch.device("cuda:0")
    p0 = torch.tensor(w.p0.astype(np.float32), device=dev)
    elem = torch.tensor(elem_np, device=dev)
    poses = torch.tensor(poses_np, device=dev)
    gpose = torch.empty((1, 12), dtype=torch.float64, device=dev)
    gelem = torch.empty((1, elem_np.shape[0], 3), dtype=torch.float64, device=dev)
    announce("C4 sub-array pose blocks")
    L.radiate_adjoint(g, p0, elem, poses, s, torch.tensor(r, device=dev), grad_pose=gpose, grad_elem=gelem)
    torch.cuda.synchronize()
    _pose_block_errors("C4 16x8 block", gpose.cpu().numpy(), gelem.cpu().numpy()[0], gp_ref[None], ge_ref)


@pytest.mark.parametrize("workload", ["C2", "hemi512"])
def test_forward_sum_modes(torch_cuda, workload):
    """The forward's partial rows added in FP32 and in FP64, at the benchmarked sweep (1024 forward
    regions) and at the 512-element hemispherical view of a 256^3 volume (16384 regions, up to
    ~1000 regions meeting in one sample): sampled signal rows against the oracle.  Both modes
    meet the bar at the sweep; the automatic choice takes FP32 there and FP64 for the large grid,
    which must meet the bar."""
    import torch
    from paper_2604_09643_amd import _lib as L
    w = W.c2() if workload == "C2" else W.hemisphere1024(view=1)
    g, s = gpu_desc(w)
    p0, elem, poses = to_gpu(w)
    rng = np.random.default_rng(77)
    rows = rng.choice(w.F * w.M, size=4, replace=False)
    og, os_ = oracle_desc(w)
    s_ref = O.grid_forward(og, f32(w.p0), w.poses, w.elem, os_, elements=rows)
    ctx = L.context(0)
    errs = {}
    try:
        for name, mode in (("f32", L.RA_SUMS_F32), ("f64", L.RA_SUMS_F64), ("auto", L.RA_SUMS_AUTO)):
            ctx.set_forward_sums(mode)
            announce("%s forward sums %s" % (workload, name))
            sig = L.radiate_forward(g, p0, elem, poses, s, ctx=ctx)
            torch.cuda.synchronize()
            errs[name] = rel_l2(sig.cpu().numpy().reshape(-1, w.K)[rows], s_ref)
    finally:
        ctx.set_forward_sums(L.RA_SUMS_AUTO)
    print("[parity] %s forward sums %s" % (workload, " ".join("%s=%.2e" % kv for kv in errs.items())), flush=True)
    assert errs["f64"] <= TOL_SIGNAL and errs["auto"] <= TOL_SIGNAL
    if workload == "C2":
        assert errs["f32"] <= TOL_SIGNAL
