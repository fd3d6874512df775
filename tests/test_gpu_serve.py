"""Serving path on the GPU: the batched step against the single-call library path, and
each request's result alone versus inside a continuous batch replayed through a HIP graph."""
import numpy as np
import pytest

from gpu_helpers import announce, rel_l2
from paper_2604_09643_amd import workloads as W

pytestmark = pytest.mark.gpu

SIGMA = 0.1e-3


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_09643_amd import _lib as L
    L.load()
    shape, origin, h, p0 = W.serving_volume(seed=0, n=96, branches=20)
    vol = torch.tensor(p0.astype(np.float32), device="cuda:0").contiguous()
    grid = L.Grid(*shape, origin, h)
    samp = L.Sampling(W.C_SOUND, W.FS, 1024, SIGMA)
    return torch, L, vol, grid, samp


def make_requests(env, n, seed, rate=1e9, Ms=(16, 32, 48), Ks=(512, 1024), side=(24, 40)):
    """Requests with measured signals from the single-call forward at the true pose plus noise."""
    torch, L, vol, grid, samp = env
    from paper_2604_09643_amd.serve import Request
    specs = W.serving_stream(n, rate, grid.shape, grid.origin, grid.spacing, seed=seed, Ms=Ms, Ks=Ks,
                             side=side, pose_steps=4)
    rng = np.random.default_rng(seed + 100)
    reqs = []
    for sp in specs:
        i0, j0, k0, nx, ny, nz = sp.box
        box = vol[i0:i0 + nx, j0:j0 + ny, k0:k0 + nz].contiguous()
        bg = L.Grid(nx, ny, nz, (grid.origin[0] + i0 * grid.spacing, grid.origin[1] + j0 * grid.spacing,
                                  grid.origin[2] + k0 * grid.spacing), grid.spacing)
        s = L.Sampling(samp.c, samp.fs, sp.K, samp.sigma)
        poses = L.pose_from_axis_angle(torch.tensor(sp.true6[None], device="cuda:0"))
        y = L.radiate_forward(bg, box, torch.tensor(sp.elem, device="cuda:0"), poses, s)[0].cpu().numpy()
        y = y + rng.normal(scale=0.01 * np.abs(y).max() + 1e-12, size=y.shape)
        if sp.kind == 1:
            y = 0.5 * y                       # volume updates see a mismatch to correct
        reqs.append(Request(sp.rid, sp.kind, sp.box, sp.elem, sp.init6, y.astype(np.float32), sp.steps,
                            sp.arrival))
    return reqs


def box_call(env, req):
    """Single-call path for one step of a request: loss, dL/dp0 of the box, (dL/dw, dL/dt)."""
    torch, L, vol, grid, samp = env
    i0, j0, k0, nx, ny, nz = req.box
    box = vol[i0:i0 + nx, j0:j0 + ny, k0:k0 + nz].contiguous()
    bg = L.Grid(nx, ny, nz, (grid.origin[0] + i0 * grid.spacing, grid.origin[1] + j0 * grid.spacing,
                              grid.origin[2] + k0 * grid.spacing), grid.spacing)
    s = L.Sampling(samp.c, samp.fs, req.K, samp.sigma)
    p6 = torch.tensor(req.pose6[None], device="cuda:0")
    poses = L.pose_from_axis_angle(p6)
    gp0 = torch.empty_like(box)
    gpose = torch.empty((1, 12), dtype=torch.float64, device="cuda:0")
    loss = L.loss_and_grad(bg, box, torch.tensor(req.elem, device="cuda:0"), poses, s,
                           torch.tensor(req.y[None], device="cuda:0"), grad_p0=gp0, grad_pose=gpose)
    g6 = L.pose_grad_axis_angle(p6, gpose)[0].cpu().numpy()
    return loss, gp0.cpu().numpy(), g6


def executor(env, **kw):
    torch, L, vol, grid, samp = env
    from paper_2604_09643_amd.serve import GpuExecutor
    return GpuExecutor(vol, grid, samp, arena_bytes=1 << 30, **kw)


def test_batch_step_matches_single_call(env):
    from paper_2604_09643_amd.serve import POSE, Scheduler
    reqs = make_requests(env, 6, seed=1)
    for r in reqs:
        r.steps = 2                        # still active after one tick, so each slot's state can be read
    ex = executor(env, slots=8, graph=False, apply_updates=False)
    sch = Scheduler(ex, 8, 1 << 40)
    for r in reqs:
        sch.submit(r)
    announce("batch step, %d requests" % len(reqs))
    sch.tick()
    assert ex.info0.pair_d == 3            # 0.1 mm spacing: the batched forward pairs z-neighbours
    assert len(ex.state) == len(reqs)
    # the first step ran; compare the state of each slot
    for s, st in ex.state.items():
        r = st["req"]
        loss, gp0, g6 = box_call(env, r)
        assert abs(st["losses"][0] - loss) <= 2e-5 * loss
        if r.kind == POSE:
            gb = st["adam"].cpu().numpy()[:6] / (1.0 - 0.9)   # first Adam step: m = (1 - beta1) g
            e = rel_l2(gb, g6)
            # bias-corrected first step of Adam with torch's eps: lr g / (|g| + 1e-8)
            expect = r.pose6 - np.where(np.arange(6) < 3, r.lr_w, r.lr_t) * gb / (np.abs(gb) + 1e-8)
            assert np.allclose(st["pose6"].cpu().numpy(), expect, rtol=0, atol=1e-12)
        else:
            e = rel_l2(st["grad"].cpu().numpy(), gp0)
        print("[serve] request %d kind %d rel-L2 %.2e" % (r.rid, r.kind, e), flush=True)
        assert e <= 1e-5


def test_volume_update_applies_step(env):
    torch, L, vol, grid, samp = env
    from paper_2604_09643_amd.serve import VOLUME, Scheduler
    reqs = [r for r in make_requests(env, 12, seed=2) if r.kind == VOLUME][:1]
    assert reqs
    r = reqs[0]
    i0, j0, k0, nx, ny, nz = r.box
    before = vol[i0:i0 + nx, j0:j0 + ny, k0:k0 + nz].clone()
    _, gp0, _ = box_call(env, r)
    ex = executor(env, slots=2, graph=False, apply_updates=True, lr_volume=0.5)
    sch = Scheduler(ex, 2, 1 << 40)
    announce("volume update apply")
    sch.run([r], realtime=False)
    after = vol[i0:i0 + nx, j0:j0 + ny, k0:k0 + nz].clone()
    vol[i0:i0 + nx, j0:j0 + ny, k0:k0 + nz] = before            # restore the shared volume
    delta = (after - before).cpu().numpy()
    assert rel_l2(delta, -0.5 * gp0) <= 1e-5


def test_alone_equals_in_mix_with_graph(env):
    """Each request run alone (eager launches) and inside a continuous batch with staggered
    arrivals, replayed through one captured HIP graph, gives the same result."""
    from paper_2604_09643_amd.serve import POSE, Scheduler
    reqs = make_requests(env, 10, seed=3)
    for i, r in enumerate(reqs):
        r.arrival = 0.0
    alone = {}
    ex1 = executor(env, slots=1, graph=False, apply_updates=False)
    for r in reqs:
        sch = Scheduler(ex1, 1, 1 << 40)
        announce("alone request %d" % r.rid)
        alone[r.rid] = sch.run([r], realtime=False)[0]
    clock = {"t": 0.0}

    def tick_clock():
        clock["t"] += 1.0
        return clock["t"]
    mixed_reqs = make_requests(env, 10, seed=3)
    for i, r in enumerate(mixed_reqs):
        r.arrival = float(i // 3) * 2.0           # batches of arrivals while others are mid-way
    ex2 = executor(env, slots=6, graph=True, apply_updates=False)
    sch = Scheduler(ex2, 6, 1 << 40, clock=tick_clock)
    announce("mixed stream with graph")
    res = {r.rid: r for r in sch.run(mixed_reqs, realtime=False, t0=0.0)}
    assert max(sch.batch_sizes) >= 3 and len(set(sch.batch_sizes)) > 1
    for rid, a in alone.items():
        b = res[rid]
        assert len(a.losses) == len(b.losses)
        np.testing.assert_allclose(b.losses, a.losses, rtol=1e-5)
        if a.kind == POSE:
            init = [r for r in reqs if r.rid == rid][0].pose6
            e = rel_l2(b.pose6 - init, a.pose6 - init)
            assert e <= 1e-4, (rid, e)
        else:
            assert rel_l2(b.grad_p0, a.grad_p0) <= 1e-5


def test_batch_step_matches_oracle(env):
    """One batched step (ra_batch_step) on a mixed batch of two pose-refinement and two volume
    requests with different element counts, sample counts and boxes, against the FP64 oracle:
    each request's residual buffer 2 (s - y) (the batched forward, FP32 atomics into the
    request's signals), its loss, the volume requests' dL/dp0 of their boxes, and the pose
    requests' first-step gradient (dL/dw, dL/dt), read back from Adam's first moment
    m = (1 - beta1) g, rotation and translation blocks separately.  The measured signals are
    the oracle's forward at the true pose plus noise."""
    torch, L, vol, grid, samp = env
    from oracle import oracle as O
    from paper_2604_09643_amd.serve import POSE, VOLUME, Request, Scheduler
    shape, origin, h, p0_np = W.serving_volume(seed=0, n=96, branches=20)
    p0_np = p0_np.astype(np.float32).astype(np.float64)
    specs = W.serving_stream(24, 1e9, shape, origin, h, seed=11, Ms=(16, 32, 48), Ks=(512, 1024), side=(24, 40),
                             pose_steps=1)
    def has_source(sp):                       # boxes that miss every vessel give y = 0, L = 0
        i0, j0, k0, nx, ny, nz = sp.box
        return np.abs(p0_np[i0:i0 + nx, j0:j0 + ny, k0:k0 + nz]).max() > 0.1

    picked, seen = [], set()
    for kind in (POSE, POSE, VOLUME, VOLUME):
        for sp in specs:
            key = (sp.M, sp.K, sp.box[3])
            if sp.kind == kind and sp.rid not in {p.rid for p in picked} and key not in seen and has_source(sp):
                picked.append(sp)
                seen.add(key)
                break
    assert [sp.kind for sp in picked] == [POSE, POSE, VOLUME, VOLUME]
    rng = np.random.default_rng(12)
    reqs, ref = [], {}
    for sp in picked:
        i0, j0, k0, nx, ny, nz = sp.box
        og = O.Grid(nx, ny, nz, (origin[0] + i0 * h, origin[1] + j0 * h, origin[2] + k0 * h), h)
        os_ = O.Sampling(samp.c, samp.fs, sp.K, samp.sigma, samp.trunc)
        box = np.ascontiguousarray(p0_np[i0:i0 + nx, j0:j0 + ny, k0:k0 + nz])
        y = O.grid_forward(og, box, O.poses_from_pose6(sp.true6[None]), sp.elem, os_)[0]
        y = y + rng.normal(scale=0.01 * np.abs(y).max(), size=y.shape)
        if sp.kind == VOLUME:
            y = 0.5 * y
        y = y.astype(np.float32)
        reqs.append(Request(sp.rid, sp.kind, sp.box, sp.elem, sp.init6, y, 2, 0.0))   # active after one tick
        poses = O.poses_from_pose6(sp.init6[None])
        s_ref = O.grid_forward(og, box, poses, sp.elem, os_)
        L_ref, r_ref = O.loss_residual(s_ref, y.astype(np.float64)[None])
        out = {"L": L_ref, "r": r_ref[0]}
        if sp.kind == VOLUME:
            out["gp0"] = O.grid_adjoint_p0(og, poses, sp.elem, os_, r_ref)
        else:
            ge = O.grid_adjoint_elem(og, box, poses, sp.elem, os_, r_ref)
            out["g6"] = O.pose6_grad(sp.init6[None], O.pose_grad(sp.elem, ge))[0]
        ref[sp.rid] = out
    ex = executor(env, slots=8, graph=False, apply_updates=False)
    sch = Scheduler(ex, 8, 1 << 40)
    for r in reqs:
        sch.submit(r)
    announce("batch step vs oracle, %d requests" % len(reqs))
    sch.tick()
    assert len(ex.state) == len(reqs)
    for slot, st in ex.state.items():
        r = st["req"]
        o = ref[r.rid]
        off, n = st["offs"]["s"], st["sizes"]["s"]
        resid = ex.buf[off:off + n].view(torch.float32).view(r.M, r.K).cpu().numpy()
        e_r = rel_l2(resid, o["r"])
        e_L = abs(st["losses"][0] - o["L"]) / o["L"]
        msg = "[serve-oracle] request %d kind %d M=%d K=%d box=%d: residual %.2e loss %.2e" % (
            r.rid, r.kind, r.M, r.K, r.box[3], e_r, e_L)
        assert e_r <= 1e-5 and e_L <= 1e-5, msg
        if r.kind == VOLUME:
            e_g = rel_l2(st["grad"].cpu().numpy(), o["gp0"])
            print(msg + " dL/dp0 %.2e" % e_g, flush=True)
            assert e_g <= 1e-4
        else:
            g6 = st["adam"].cpu().numpy()[:6] / 0.1
            e_w, e_t = rel_l2(g6[:3], o["g6"][:3]), rel_l2(g6[3:], o["g6"][3:])
            print(msg + " dL/dw %.2e dL/dt %.2e" % (e_w, e_t), flush=True)
            assert e_w <= 1e-4 and e_t <= 1e-4


def _disjoint(a, b):
    return any(a[i] + a[3 + i] <= b[i] or b[i] + b[3 + i] <= a[i] for i in range(3))


def test_alone_equals_in_mix_with_updates(env):
    """Volume updates applied to the resident volume while the stream runs (graph replay): each
    tick reads the volume as the previous tick left it, and a volume request's update lands at the
    end of its step.  So a request whose box meets no volume request's box gives the same result
    alone and in the mix, and with the volume requests' boxes pairwise disjoint the volume ends at
    the start volume minus lr times the sum of their gradients taken alone.  Requests whose box
    meets a volume request's box take part but depend on when that update lands, and are not
    compared."""
    torch, L, vol, grid, samp = env
    from paper_2604_09643_amd.serve import POSE, VOLUME, Scheduler
    cand = make_requests(env, 24, seed=4)
    vols = []
    for r in cand:
        if r.kind == VOLUME and all(_disjoint(r.box, v.box) for v in vols):
            vols.append(r)
    poses = [r for r in cand if r.kind == POSE][:8]
    reqs = sorted(vols + poses, key=lambda r: r.rid)
    clean = {r.rid for r in reqs if all(_disjoint(r.box, v.box) for v in vols if v.rid != r.rid)}
    assert len(vols) >= 2 and len([r for r in poses if r.rid in clean]) >= 2 and len(clean) < len(reqs)
    before = vol.clone()
    lr = 0.5
    try:
        alone = {}
        ex1 = executor(env, slots=1, graph=False, apply_updates=False)
        for r in reqs:
            sch = Scheduler(ex1, 1, 1 << 40)
            announce("alone request %d (kind %d)" % (r.rid, r.kind))
            alone[r.rid] = sch.run([r], realtime=False)[0]
        clock = {"t": 0.0}

        def tick_clock():
            clock["t"] += 1.0
            return clock["t"]
        mixed = [type(r)(**{**r.__dict__}) for r in reqs]
        for i, r in enumerate(mixed):
            r.arrival = float(i // 3) * 2.0
        ex2 = executor(env, slots=6, graph=True, apply_updates=True, lr_volume=lr)
        sch = Scheduler(ex2, 6, 1 << 40, clock=tick_clock)
        announce("mixed stream with updates applied")
        res = {r.rid: r for r in sch.run(mixed, realtime=False, t0=0.0)}
        torch.cuda.synchronize()
        after = vol.clone()
    finally:
        vol.copy_(before)
    assert len(res) == len(reqs) and max(sch.batch_sizes) >= 3
    for rid in sorted(clean):
        a, b = alone[rid], res[rid]
        np.testing.assert_allclose(b.losses, a.losses, rtol=1e-5)
        if a.kind == POSE:
            init = [r for r in reqs if r.rid == rid][0].pose6
            e = rel_l2(b.pose6 - init, a.pose6 - init)
        else:
            e = rel_l2(b.grad_p0, a.grad_p0)
        print("[serve] updates applied: request %d kind %d alone vs mix %.2e" % (rid, a.kind, e), flush=True)
        assert e <= 1e-4, (rid, e)
    expect = before.clone()
    for v in vols:
        i0, j0, k0, nx, ny, nz = v.box
        expect[i0:i0 + nx, j0:j0 + ny, k0:k0 + nz] -= lr * torch.tensor(alone[v.rid].grad_p0, device=vol.device)
    e_v = rel_l2((after - before).cpu().numpy(), (expect - before).cpu().numpy())
    print("[serve] resident volume after the stream vs start - lr sum of the alone gradients: %.2e" % e_v, flush=True)
    assert e_v <= 1e-5


def test_batch_step_refuses_bad_moment_fields(env):
    """ra_batch_step checks the moment-form fields of the batch on the host and refuses, before any
    launch, a batch without the coefficient scratch, with a bin count outside what a workgroup's LDS
    window holds, or with the moment form on a window it does not cover."""
    import ctypes
    torch, L, vol, grid, samp = env
    reqs = make_requests(env, 4, seed=5)
    ex = executor(env, slots=2, graph=False)
    announce("batch step: moment-field checks")
    assert ex.admit(reqs[0], 0)
    assert ex.info0.moment == 1                  # sigma 0.1 mm at 40 MHz: the moment form applies
    lib, ctx = ex.lib, ex.ctx

    def rc_of(**fields):
        b = ex._cbatch()
        for k, v in fields.items():
            setattr(b, k, v)
        rc = lib.ra_batch_step(ctx.ptr, ctypes.byref(b), 0, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        return rc, lib.ra_last_error(ctx.ptr).decode()

    rc, msg = rc_of(coef=None)
    assert rc == L.RA_EINVAL and "coef" in msg
    for nbin in (0, 41):
        rc, msg = rc_of(nbin=nbin)
        assert rc == L.RA_EINVAL and "nbin" in msg
    rc, msg = rc_of(exact=0, pair_d=0)
    assert rc == L.RA_EINVAL and "moment form" in msg
    ex.release(0)
    torch.cuda.synchronize()


def test_injected_launch_failure_on_the_device_loop(env):
    """A launch failure injected into the GPU executor (the second step raises on the host before
    anything is queued) fails exactly the requests of that batch; their slots and arena blocks are
    freed, the captured graph keeps serving, and every other request gives its alone result."""
    from paper_2604_09643_amd.serve import POSE, Scheduler
    reqs = make_requests(env, 6, seed=7)
    for r in reqs:
        r.arrival = 0.0
    alone = {}
    ex1 = executor(env, slots=1, graph=False, apply_updates=False)
    for r in reqs:
        announce("alone request %d" % r.rid)
        alone[r.rid] = Scheduler(ex1, 1, 1 << 40).run([r], realtime=False)[0]
    clock = {"t": 0.0}

    def tick_clock():
        clock["t"] += 1.0
        return clock["t"]
    mixed = make_requests(env, 6, seed=7)
    for r in mixed:
        r.arrival = 0.0
    ex2 = executor(env, slots=3, graph=True, apply_updates=False, fail_launch_at=2)
    sch = Scheduler(ex2, 3, 1 << 40, clock=tick_clock)
    announce("stream with a launch failure at step 2")
    res = {r.rid: r for r in sch.run(mixed, realtime=False, t0=0.0)}
    failed = {rid for rid, _ in sch.failed}
    assert len(failed) == sch.batch_sizes[1] >= 1               # exactly the batch of the failed step
    assert all("injected launch failure" in why for _, why in sch.failed)
    assert not (failed & set(res)) and failed | set(res) == {r.rid for r in mixed}
    assert sch.mem_used == 0 and ex2.arena.used == 0 and not ex2.state
    for rid, b in res.items():
        a = alone[rid]
        np.testing.assert_allclose(b.losses, a.losses, rtol=1e-5)
        if a.kind == POSE:
            init = [r for r in reqs if r.rid == rid][0].pose6
            assert rel_l2(b.pose6 - init, a.pose6 - init) <= 1e-4
        else:
            assert rel_l2(b.grad_p0, a.grad_p0) <= 1e-5
