"""Throughput of the radiation model on one MI355X.

One step = loss_and_grad on the single-freehand-sweep workload (128x128x64 voxels at
0.1 mm, 64 frames of a 128-element linear array, K=1024 samples at 40 MHz,
sigma=0.08 mm): element positions, forward model, residual and loss, and the p0
adjoint, all inputs resident in HBM.  The metric counts in-window (voxel, element,
sample) updates of the forward and the adjoint, with the update count decided in
FP64 (ra_count_updates) and checked against the oracle by the test suite.

Prints one JSON line (see the repository's bench contract) with a `roofline` object
for the dominant kernel (timed with HIP events on the stream it runs on) and a
`cpu_baseline` object (the FP64 oracle on a bounded sample of the same workload, on
the host cores).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+adj voxel·element·sample updates/s (FP32)"
PEAK_FP32_TFLOPS = 157.3          # MI355X published FP32 vector peak
# algorithmic work of one in-window update (direct form of Eq. (A13)): u = d - c t_k (1), u^2 (1),
# scale by -1/(2 sigma^2) (1), u e (1), times p0/(2d) (1), accumulate (FMA, 2) = 7 FLOP, plus one
# exponential, reported separately against the measured v_exp_f32 rate
FLOP_PER_UPDATE = 7
EXP_PER_UPDATE = 1
# transcendentals the forward kernel executes per (voxel, element) pair: two exponentials of the
# factorised window (the start of the pair's row chain and its ratio H) and one reciprocal square
# root of the distance
TRANS_PER_PAIR_FWD = 3
# algorithmic work of the moment-form dL/dp0 adjoint: per (voxel, element) pair the distance (18
# FLOP and one reciprocal square root), the centre sample and offset (3), Horner's rule over the 8
# moments (14), the 1/(2d) factor and the lane sum (2) = 37 FLOP; per element and row of the moment
# table (K + 2 JT rows, JT = floor(6 sigma / delta + 1/2)), 8 moments of 2 JT + 1 taps
FLOP_PER_PAIR_ADJ_MOMENT = 37


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy, the reference for HBM byte counters")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 256^3 matrix-array and 256-frame autograd measurements")
    ap.add_argument("--serving-requests", type=int, default=120)
    ap.add_argument("--serving-rate", type=float, default=200.0)
    ap.add_argument("--c3-adam", type=int, default=0, metavar="STEPS",
                    help="only run the 256-frame joint p0 + pose optimisation for STEPS Adam steps and print "
                         "its loss curve, pose errors and peak device memory as one JSON line")
    ap.add_argument("--c3-checkpoint", metavar="PATH",
                    help="with --c3-adam: write the optimisation state to PATH every --c3-checkpoint-every steps")
    ap.add_argument("--c3-checkpoint-every", type=int, default=10, metavar="N")
    ap.add_argument("--c3-resume", metavar="PATH", help="with --c3-adam: continue from a checkpoint written so")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "'bench.py --copy-calibration' into profiles/traffic.json and exit")
    return ap.parse_args()


def source_hash() -> str:
    p = os.path.join(ROOT, "paper_2604_09643_amd", "csrc", "radiate.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def traffic_from_profile(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was taken on the
    current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        if d.get("source_sha256_16") != source_hash():
            return None
        return d["kernels"][kernel]["hbm_bytes_per_launch"]
    except Exception:
        return None


def host_info():
    """Logical CPUs and the CPU model of the host the oracle runs on."""
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model}


def device_info(dev, fma_rate: float, busy):
    """Device name, CU count and memory; the clock the FP32 FMA probe implies (128 FLOP per clock per
    CU unpacked); and, given `busy` (work that keeps the GPU loaded meanwhile), a rocm-smi reading of
    clocks and power (best effort: null where the tool is missing or its output is not JSON)."""
    import subprocess
    import torch
    pr = torch.cuda.get_device_properties(dev)
    out = {"name": pr.name, "arch": getattr(pr, "gcnArchName", None), "compute_units": pr.multi_processor_count,
           "memory_gib": pr.total_memory / 2 ** 30,
           "sclk_ghz_from_fma_probe": 2.0 * fma_rate / (pr.multi_processor_count * 128) / 1e9, "smi_under_load": None}
    if busy is None:
        return out
    busy()
    try:
        res = subprocess.run(["rocm-smi", "--showclocks", "--showpower", "--json"], capture_output=True, text=True,
                             timeout=30)
        data = json.loads(res.stdout)
        keep = {}
        for card, fields in data.items():
            if isinstance(fields, dict):
                keep[card] = {k: v for k, v in fields.items()
                              if "sclk" in k.lower() or "power" in k.lower() or "mclk" in k.lower()}
        out["smi_under_load"] = keep
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    torch.cuda.synchronize()
    return out


def spread(ms):
    """Median, 10th and 90th percentiles of per-call durations."""
    import numpy as np
    return {"median": float(np.median(ms)), "p10": float(np.percentile(ms, 10)), "p90": float(np.percentile(ms, 90)),
            "n": len(ms)}


def cpu_baseline(w, budget_s: float):
    """FP64 oracle on bounded samples of the same workload, with all of its OpenMP threads and
    with one thread: whole forward rows of randomly chosen elements and p0-adjoint values of
    randomly chosen voxels."""
    from oracle import oracle as O
    n_all = O.num_threads()
    full = _cpu_sample(w, budget_s)
    O.set_threads(1)
    try:
        one = _cpu_sample(w, budget_s / 2)
    finally:
        O.set_threads(n_all)
    out = {"value": full["rate"], "unit": "updates/s", "cores": n_all, "kind": "oracle",
           "sample": full["sample"], "single_thread": {"value": one["rate"], "cores": 1, "sample": one["sample"]}}
    out.update(host_info())
    return out


def _cpu_sample(w, budget_s: float):
    import numpy as np
    from oracle import oracle as O
    og = O.Grid(*w.shape, w.origin, w.spacing)
    os_ = O.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)
    rng = np.random.default_rng(7)
    p0 = w.p0.astype(np.float32).astype(np.float64)
    r = rng.normal(size=(w.F, w.M, w.K))

    def run(n_rows, n_vox):
        rows = rng.choice(w.F * w.M, size=n_rows, replace=False)
        vox = rng.choice(w.n_voxels, size=n_vox, replace=False)
        xe = O.element_positions(w.poses, w.elem).reshape(-1, 3)
        u = O.count_updates(O.voxel_centres(og), xe[rows], os_)
        u += O.count_updates(O.voxel_centres(og, vox), xe, os_)
        t0 = time.perf_counter()
        O.grid_forward(og, p0, w.poses, w.elem, os_, elements=rows)
        O.grid_adjoint_p0(og, w.poses, w.elem, os_, r, voxels=vox)
        return u, time.perf_counter() - t0, n_rows, n_vox

    nr, nv = 2, 64
    u, dt, _, _ = run(nr, nv)                  # calibration, grown until it takes about budget_s
    for _ in range(3):
        if dt >= 0.6 * budget_s:
            break
        scale = min(budget_s / max(dt, 1e-3), 64.0)
        nr, nv = min(int(nr * scale) + 1, w.F * w.M), min(int(nv * scale) + 1, w.n_voxels)
        u, dt, nr, nv = run(nr, nv)
    return {"rate": u / dt,
            "sample": "FP64 oracle (%d threads): forward rows of %d random (frame, element) pairs over all %d "
                      "voxels + p0-adjoint of %d random voxels over all %d elements; %d updates in %.1f s"
                      % (O.num_threads(), nr, w.n_voxels, nv, w.F * w.M, u, dt)}


def write_traffic(fetch_csv: str, write_csv: str):
    """HBM bytes per launch of each kernel from rocprofv3 counter dumps, scaled by what the
    same counters read for the 1 GiB calibration copy (the dispatch writing ~1 GiB)."""
    import csv
    import numpy as np

    def load(path):
        per = {}
        calib = None
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]
            v = float(r["Counter_Value"]) * 1024.0
            per.setdefault(name, []).append(v)
            if "copyBuffer" in name or "elementwise" in name:
                calib = v if calib is None or abs(v - 2**30) < abs(calib - 2**30) else calib
        return per, calib
    fetch, cf = load(fetch_csv)
    write, cw = load(write_csv)
    f_fac, w_fac = 2**30 / cf, 2**30 / cw
    out = {"source_sha256_16": source_hash(), "unit": "bytes per launch",
           "calibration": {"copy_bytes": 2**30, "fetch_counter_bytes": cf, "write_counter_bytes": cw,
                           "fetch_scale": f_fac, "write_scale": w_fac},
           "kernels": {}}
    for name in sorted(set(fetch) & set(write)):
        fb, wb = float(np.mean(fetch[name])) * f_fac, float(np.mean(write[name])) * w_fac
        short = name.split("<")[0]
        out["kernels"][short] = {"template": name, "fetch_bytes": fb, "write_bytes": wb,
                                 "hbm_bytes_per_launch": fb + wb}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    json.dump(out, open(path, "w"), indent=1)
    print(json.dumps(out["calibration"]))
    for k, v in out["kernels"].items():
        print("%-14s fetch %.3e B  write %.3e B" % (k, v["fetch_bytes"], v["write_bytes"]))


SERVING_WORK_BUDGET = 2e8     # (voxel, element) pairs per tick: about one median request's step


def serving_bench(n_requests: int, rate: float, seed: int = 0, rates=(10.0, 20.0, 40.0)):
    """Continuous batching (graph-replayed batched steps, 16 slots) against unbatched FIFO (one
    request at a time, eager launches) on the same Poisson streams of mixed requests, at the
    headline offered rate, at about the batched loop's capacity (measured at the headline rate)
    and at lower rates.  Two batched loops: "batched" admits into a running batch only while the
    tick's work stays within SERVING_WORK_BUDGET (a request that fills the GPU runs alone, as in
    FIFO; smaller ones share ticks), "batched_unlimited" admits whenever a slot and memory are free.
    Volume updates are applied to the resident volume, which is restored before every run; each
    loop's executor is built, warmed up and captured once, untimed.  GPU utilisation = time
    inside the batched steps (HIP events) / wall time."""
    import numpy as np
    import torch
    from paper_2604_09643_amd import _lib as L
    from paper_2604_09643_amd import serve as S
    from paper_2604_09643_amd import workloads as W
    dev = torch.device("cuda:0")
    shape, origin, h, p0 = W.serving_volume(seed=seed, n=256, branches=60)
    vol0 = torch.tensor(p0.astype(np.float32), device=dev).contiguous()
    vol = vol0.clone()
    grid = L.Grid(*shape, origin, h)
    samp = L.Sampling(W.C_SOUND, W.FS, 1024, 0.1e-3)

    def requests(n, r, sd):
        specs = W.serving_stream(n, r, shape, origin, h, seed=sd)
        rng = np.random.default_rng(sd + 1)
        out = []
        for sp in specs:
            i0, j0, k0, nx, ny, nz = sp.box
            box = vol0[i0:i0 + nx, j0:j0 + ny, k0:k0 + nz].contiguous()
            bg = L.Grid(nx, ny, nz, (origin[0] + i0 * h, origin[1] + j0 * h, origin[2] + k0 * h), h)
            ss = L.Sampling(samp.c, samp.fs, sp.K, samp.sigma)
            poses = L.pose_from_axis_angle(torch.tensor(sp.true6[None], device=dev))
            y = L.radiate_forward(bg, box, torch.tensor(sp.elem, device=dev), poses, ss)[0]
            y = (y + torch.randn_like(y) * 0.01 * float(y.abs().max())).cpu().numpy()
            out.append(S.Request(sp.rid, sp.kind, sp.box, sp.elem, sp.init6, y, sp.steps, sp.arrival))
        return out, specs

    def updates(specs):
        tot = 0
        for sp in specs:
            i0, j0, k0, nx, ny, nz = sp.box
            bg = L.Grid(nx, ny, nz, (origin[0] + i0 * h, origin[1] + j0 * h, origin[2] + k0 * h), h)
            ss = L.Sampling(samp.c, samp.fs, sp.K, samp.sigma)
            poses = L.pose_from_axis_angle(torch.tensor(sp.init6[None], device=dev))
            tot += 2 * sp.steps * L.count_updates(bg, torch.tensor(sp.elem, device=dev), poses, ss)
        return tot

    ex_b = S.GpuExecutor(vol, grid, samp, slots=16, arena_bytes=6 << 30, graph=True, apply_updates=True)
    ex_u = S.GpuExecutor(vol, grid, samp, slots=1, arena_bytes=6 << 30, graph=False, apply_updates=True)

    def run(mode, reqs):
        vol.copy_(vol0)
        ex = ex_u if mode == "unbatched" else ex_b
        ex.gpu_ms, ex.n_steps = 0.0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode == "unbatched":
            sch, res = S.serve_unbatched(ex, reqs)
        else:
            sch, res = S.serve(ex, reqs, slots=16, mem_cap=200 << 30,
                               work_budget=SERVING_WORK_BUDGET if mode == "batched" else None)
        wall = time.perf_counter() - t0
        st = S.latency_stats(res)
        pose = S.latency_stats(res, S.POSE)
        st.update(pose_p50_ms=pose.get("p50_ms", float("nan")), pose_p99_ms=pose.get("p99_ms", float("nan")),
                  wall_s=wall, completed=len(res),
                  failed=len(sch.failed), ticks=sch.ticks, throughput_req_s=len(res) / wall,
                  gpu_utilisation=ex.gpu_ms * 1e-3 / wall,
                  mean_batch=float(np.mean(sch.batch_sizes)) if sch.batch_sizes else 0.0)
        return st

    t_start = time.perf_counter()
    warm, _ = requests(6, 1e6, seed + 99)
    run("batched", warm)                                   # build and capture once, untimed
    run("unbatched", warm[:2])
    print("[bench] serving: executors built and warmed (%.1f s)" % (time.perf_counter() - t_start),
          file=sys.stderr, flush=True)
    points = []

    def point(r, sd):
        out = {"offered_rate_req_s": r, "n_requests": n_requests}
        for mode in ("batched", "batched_unlimited", "unbatched"):
            reqs, specs = requests(n_requests, r, sd)
            if "updates" not in out:
                out["updates"] = updates(specs)
            out[mode] = run(mode, reqs)
            out[mode]["updates_per_s"] = out["updates"] / out[mode]["wall_s"]
            print("[bench] serving %.1f req/s, %s loop: %.1f s" % (r, mode, out[mode]["wall_s"]),
                  file=sys.stderr, flush=True)
        points.append(out)
        print("[bench] serving %.1f req/s: pose p50 / p99 ms, req/s, GPU: batched %.1f / %.1f, %.1f, %.0f%%; "
              "unlimited %.1f / %.1f, %.1f, %.0f%%; unbatched %.1f / %.1f, %.1f, %.0f%%"
              % tuple([r] + [out[m][k] * (100 if k == "gpu_utilisation" else 1)
                             for m in ("batched", "batched_unlimited", "unbatched")
                             for k in ("pose_p50_ms", "pose_p99_ms", "throughput_req_s", "gpu_utilisation")]),
              file=sys.stderr, flush=True)
        return out

    head = point(rate, seed)
    capacity = head["batched_unlimited"]["throughput_req_s"]
    for i, r in enumerate(sorted(set(list(rates) + [round(capacity, 1)]))):
        point(r, seed + 10 + i)
    return {"offered_rate_req_s": rate, "n_requests": n_requests, "updates": head["updates"],
            "batched": head["batched"], "batched_unlimited": head["batched_unlimited"],
            "unbatched": head["unbatched"], "capacity_req_s": capacity, "work_budget_pairs": SERVING_WORK_BUDGET,
            "sweep": sorted(points, key=lambda q: q["offered_rate_req_s"]), "apply_updates": True}


def large_configs(ctx):
    """The two larger configurations at full size, each timed after one warm-up:
    the 256^3 / 1024-element matrix array forward and full adjoint (dL/dp0, dL/dx_e and the
    FP64 per-frame pose reduction), and one autograd step of the 256-frame 256x256x128
    reconstruction (chunked loss: forward for the loss, then forward again and the adjoint
    per 16-frame chunk in backward)."""
    import numpy as np
    import torch
    from paper_2604_09643_amd import _lib as L
    from paper_2604_09643_amd import autograd as A
    from paper_2604_09643_amd import workloads as W
    dev = torch.device("cuda:0")
    st = torch.cuda.current_stream()
    out = {}

    def ev_ms(fn, n):
        fn()
        e = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for e0, e1 in e:
            e0.record(st)
            fn()
            e1.record(st)
        torch.cuda.synchronize()
        return float(np.mean([e0.elapsed_time(e1) for e0, e1 in e]))

    w = W.c4()
    g = L.Grid(*w.shape, tuple(w.origin), w.spacing)
    s = L.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)
    p0 = torch.tensor(w.p0.astype(np.float32), device=dev)
    elem = torch.tensor(w.elem, device=dev)
    poses = torch.tensor(w.poses, device=dev)
    n4 = L.count_updates(g, elem, poses, s, ctx=ctx)
    sig = torch.empty((w.F, w.M, w.K), dtype=torch.float32, device=dev)
    r = torch.randn_like(sig)
    gp0 = torch.empty_like(p0)
    gpose = torch.empty((w.F, 12), dtype=torch.float64, device=dev)
    gelem = torch.empty((w.F, w.M, 3), dtype=torch.float64, device=dev)
    ms_f = ev_ms(lambda: L.radiate_forward(g, p0, elem, poses, s, sig, ctx=ctx), 2)
    ms_a = ev_ms(lambda: L.radiate_adjoint(g, p0, elem, poses, s, r, grad_p0=gp0, grad_pose=gpose,
                                           grad_elem=gelem, ctx=ctx), 2)
    out["matrix_array_256cube"] = {
        "workload": "256^3 voxels at 0.1 mm, 8 frames x 32x32 matrix array (pitch 0.5 mm), K=2048, sigma=0.1 mm",
        "updates_per_pass": n4, "ms_forward": ms_f, "ms_adjoint_p0_pose_elem": ms_a,
        "updates_per_s_forward": n4 / (ms_f * 1e-3), "updates_per_s_adjoint": n4 / (ms_a * 1e-3)}
    print("[bench] 256^3 matrix array: forward %.1f ms, full adjoint %.1f ms (%d updates per pass)"
          % (ms_f, ms_a, n4), file=sys.stderr, flush=True)
    del p0, sig, r, gp0, gpose, gelem

    w = W.hemisphere1024(view=0)
    g = L.Grid(*w.shape, tuple(w.origin), w.spacing)
    s = L.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)
    p0 = torch.tensor(w.p0.astype(np.float32), device=dev)
    elem = torch.tensor(w.elem, device=dev)
    poses = torch.tensor(w.poses, device=dev)
    nh = L.count_updates(g, elem, poses, s, ctx=ctx)
    sig = torch.empty((w.F, w.M, w.K), dtype=torch.float32, device=dev)
    r = torch.randn_like(sig)
    gp0 = torch.empty_like(p0)
    gpose = torch.empty((w.F, 12), dtype=torch.float64, device=dev)
    ms_f = ev_ms(lambda: L.radiate_forward(g, p0, elem, poses, s, sig, ctx=ctx), 3)
    ms_a = ev_ms(lambda: L.radiate_adjoint(g, p0, elem, poses, s, r, grad_p0=gp0, grad_pose=gpose, ctx=ctx), 3)
    out["hemisphere_512_view"] = {
        "workload": "one 512-element view of a 1024-element hemispherical array (radius 60 mm) around "
                    "256^3 voxels at 0.1 mm, K=2560, sigma=0.1 mm",
        "updates_per_pass": nh, "ms_forward": ms_f, "ms_adjoint_p0_pose": ms_a,
        "updates_per_s_forward": nh / (ms_f * 1e-3), "updates_per_s_adjoint": nh / (ms_a * 1e-3)}
    print("[bench] hemispherical view: forward %.1f ms, adjoint %.1f ms (%d updates per pass)"
          % (ms_f, ms_a, nh), file=sys.stderr, flush=True)
    del p0, sig, r, gp0, gpose

    # TGV regulariser on the 256^3 volume: value and both gradients
    n = 256 ** 3
    u = torch.randn((256, 256, 256), dtype=torch.float32, device=dev)
    wf = torch.randn((3, 256, 256, 256), dtype=torch.float32, device=dev)
    gu, gwf = torch.empty_like(u), torch.empty_like(wf)
    ms_t = ev_ms(lambda: L.tgv_loss_and_grad(u, wf, 2.0, 1.0, 1e-3, want_loss=False, grad_u=gu, grad_w=gwf,
                                             ctx=ctx), 5)
    algo = 32.0 * n                                  # read u, w; write grad_u, grad_w (float32)
    out["tgv_256cube"] = {"workload": "second-order TGV of a 256^3 volume and its 3-component auxiliary "
                                      "field: value pass and gradient pass",
                          "ms": ms_t, "algorithmic_bytes": algo, "achieved_GBps": algo / (ms_t * 1e-3) / 1e9,
                          "hbm_peak_GBps": 8000.0, "frac": algo / (ms_t * 1e-3) / 8e12}
    print("[bench] TGV 256^3: %.3f ms (%.0f GB/s algorithmic)" % (ms_t, algo / (ms_t * 1e-3) / 1e9),
          file=sys.stderr, flush=True)
    del u, wf, gu, gwf

    # the other source profiles on the 128x128x64 / 64-frame sweep: forward and adjoint
    # (dL/dp0 and pose gradient), with windows where each profile has decayed
    w = W.c2()
    g = L.Grid(*w.shape, tuple(w.origin), w.spacing)
    p0 = torch.tensor(w.p0.astype(np.float32), device=dev)
    elem = torch.tensor(w.elem, device=dev)
    poses = torch.tensor(w.poses, device=dev)
    sig = torch.empty((w.F, w.M, w.K), dtype=torch.float32, device=dev)
    r = torch.randn_like(sig)
    gp0 = torch.empty_like(p0)
    gpose = torch.empty((w.F, 12), dtype=torch.float64, device=dev)
    prof = {}
    for name, kernel, trunc, nu in (("gaussian", 0, w.trunc, 1.0), ("exponential", 1, 12.0, 1.0),
                                    ("power_law_nu2", 2, 10.0, 2.0), ("uniform_sphere", 3, 1.0, 1.0)):
        s = L.Sampling(w.c, w.fs, w.K, w.sigma, trunc, kernel, nu)
        nk = L.count_updates(g, elem, poses, s, ctx=ctx)
        ms_f = ev_ms(lambda: L.radiate_forward(g, p0, elem, poses, s, sig, ctx=ctx), 3)
        ms_a = ev_ms(lambda: L.radiate_adjoint(g, p0, elem, poses, s, r, grad_p0=gp0, grad_pose=gpose, ctx=ctx),
                     3)
        prof[name] = {"trunc": trunc, "nu": nu, "updates_per_pass": nk, "ms_forward": ms_f,
                      "ms_adjoint_p0_pose": ms_a, "updates_per_s_forward": nk / (ms_f * 1e-3),
                      "updates_per_s_adjoint": nk / (ms_a * 1e-3)}
        print("[bench] C2 %s profile (trunc %g): forward %.1f ms, adjoint %.1f ms (%d updates per pass)"
              % (name, trunc, ms_f, ms_a, nk), file=sys.stderr, flush=True)
    out["source_profiles_c2"] = {"workload": "128x128x64 voxels at 0.1 mm, 64 frames x 128-element linear "
                                             "array, K=1024, width 0.08 mm; Appendix A profiles", **prof}
    del p0, sig, r, gp0, gpose

    w = W.c3()
    g = L.Grid(*w.shape, tuple(w.origin), w.spacing)
    s = L.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)
    elem = torch.tensor(w.elem, device=dev)
    true_poses = torch.tensor(w.poses, device=dev)
    n3 = L.count_updates(g, elem, true_poses, s, ctx=ctx)
    y = L.radiate_forward(g, torch.tensor(w.p0.astype(np.float32), device=dev), elem, true_poses, s, ctx=ctx)
    y += torch.randn_like(y) * (0.01 * float(y.abs().max()))
    p = torch.zeros(w.shape, dtype=torch.float32, device=dev, requires_grad=True)
    pose6 = torch.tensor(w.extra["init_pose6"], device=dev, requires_grad=True)

    def step(keep):
        p.grad = None
        pose6.grad = None
        loss = A.sweep_loss(p, pose6, y, elem, g, s, chunk=16, keep_signals=keep)
        loss.backward()
        return float(loss.detach())

    def timed_steps(keep, reps=2):
        step(keep)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            step(keep)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    ms = timed_steps(True)            # signals kept from the loss pass (268 MB): forward once per step
    ms_re = timed_steps(False)        # signals recomputed chunk by chunk in backward
    out["sweep_256_frames_autograd"] = {
        "workload": "256x256x128 voxels at 0.08 mm, 256 frames x 128-element linear array, K=2048, "
                    "sigma=0.08 mm; one step of the chunked loss (16-frame chunks) with gradients to "
                    "p0 and the 6-DoF poses; the loss pass keeps the signals for the backward",
        "updates_per_pass": n3, "ms_per_step": ms, "passes_per_step": 2,
        "updates_per_s": 2 * n3 / (ms * 1e-3), "ms_per_step_recomputing": ms_re}
    print("[bench] 256-frame sweep autograd step: %.1f ms with the signals kept (2 passes of %d updates), "
          "%.1f ms recomputing them" % (ms, n3, ms_re), file=sys.stderr, flush=True)
    return out


def c3_joint(steps: int, chunk: int = 16, checkpoint: str = None, checkpoint_every: int = 10, resume: str = None):
    """The 256x256x128 / 256-frame sweep as configured: measured signals = forward of the true
    volume at the true poses + 1% noise; starting from p0 = 0 and poses perturbed from the truth
    (0.5 mm, 2 degrees), `steps` Adam steps on p0 and the 6-DoF poses with frame-chunk
    recomputation.  Reports the loss curve, pose and volume errors against the truth, wall time
    per step and the peak device memory."""
    import numpy as np
    import torch
    from paper_2604_09643_amd import _lib as L
    from paper_2604_09643_amd import autograd as A
    from paper_2604_09643_amd import workloads as W
    dev = torch.device("cuda:0")
    w = W.c3()
    g = L.Grid(*w.shape, tuple(w.origin), w.spacing)
    s = L.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)
    elem = torch.tensor(w.elem, device=dev)
    p_true = torch.tensor(w.p0.astype(np.float32), device=dev)
    true6 = torch.tensor(w.pose6, device=dev)
    init6 = torch.tensor(w.extra["init_pose6"], device=dev)
    y = L.radiate_forward(g, p_true, elem, L.pose_from_axis_angle(true6), s)
    # seeded noise: a resumed run sees the signals the interrupted one saw
    noise = torch.randn(y.shape, generator=torch.Generator(device=dev).manual_seed(3), device=dev)
    y += noise * (0.01 * float(y.abs().max()))
    del noise
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats(dev)
    base_mem = torch.cuda.memory_allocated(dev)

    def pose_err(p6):
        d = (p6 - true6).cpu().numpy()
        return {"rot_deg_rms": float(np.degrees(np.sqrt((d[:, :3] ** 2).sum(1).mean()))),
                "trans_mm_rms": float(1e3 * np.sqrt((d[:, 3:] ** 2).sum(1).mean()))}

    t_step = []
    t_last = [time.perf_counter()]

    def cb(it, loss):
        torch.cuda.synchronize()
        now = time.perf_counter()
        t_step.append(now - t_last[0])
        t_last[0] = now
        print("[c3] step %d loss %.6e (%.2f s)" % (it, loss, t_step[-1]), file=sys.stderr, flush=True)

    p0 = torch.zeros_like(p_true)
    t0 = time.perf_counter()
    p_fin, pose_fin, hist = A.joint_optimise(p0, init6, y, elem, g, s, steps=steps, chunk=chunk, callback=cb,
                                             checkpoint=checkpoint, checkpoint_every=checkpoint_every,
                                             resume=resume)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nt = float(torch.linalg.vector_norm(p_true))
    return {"workload": "256x256x128 voxels at 0.08 mm, 256 frames x 128-element linear array, K=2048, "
                        "sigma=0.08 mm; y = forward(true p0, true poses) + 1%% noise; start p0 = 0, poses "
                        "perturbed by N(0, 0.5 mm) / N(0, 2 deg); Adam (p0 lr 1e-2, w lr 2e-3, t lr 2e-5), "
                        "frame chunks of %d; the loss pass keeps the signals for the backward" % chunk,
            "steps": steps, "loss": hist, "wall_s": wall, "s_per_step_median": float(np.median(t_step)),
            "pose_error_initial": pose_err(init6), "pose_error_final": pose_err(pose_fin),
            "p0_rel_error_initial": 1.0, "p0_rel_error_final": float(torch.linalg.vector_norm(p_fin - p_true)) / nt,
            "peak_device_bytes": int(torch.cuda.max_memory_allocated(dev)),
            "resident_before_bytes": int(base_mem),
            "signals_one_chunk_bytes": 4 * chunk * w.M * w.K, "signals_all_frames_bytes": 4 * w.F * w.M * w.K}


def pose_pipeline_bench(ctx):
    """Stages 2-4 of the pose recovery on the benchmark sweep's volume: an 8x8 matrix array
    (0.5 mm pitch) at an unknown rotated and shifted pose, 1% noise and 8 corrupted rows.
    Stage 2: coarse search (9^3 lattice, 46,656 candidate rows) and 60 annealed refinement
    steps; Stage 3: RANSAC (host); Stage 4: 80 inlier-masked fine-tuning steps.  Wall time
    of each stage (GPU work synchronised) and the final element error."""
    from dataclasses import replace
    import numpy as np
    import torch
    from paper_2604_09643_amd import _lib as L
    from paper_2604_09643_amd import localise as Z
    from paper_2604_09643_amd import rigid
    from paper_2604_09643_amd import workloads as W
    dev = torch.device("cuda:0")
    w = W.c2()
    g = L.Grid(*w.shape, tuple(w.origin), w.spacing)
    s = L.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)
    p0 = torch.tensor(w.p0.astype(np.float32), device=dev)
    rng = np.random.default_rng(2)
    tmpl = W.matrix_array(8, 0.5e-3)
    true6 = torch.tensor([[0.03, -0.02, 0.1, 0.2e-3, -0.3e-3, 0.1e-3]], dtype=torch.float64, device=dev)
    true_poses = L.pose_from_euler(true6, ctx=ctx)
    tm = torch.tensor(tmpl, device=dev)
    y = L.radiate_forward(g, p0, tm, true_poses, s, ctx=ctx)[0]
    y = y + torch.randn_like(y) * 0.01 * float(y.abs().max())
    bad = rng.choice(64, size=8, replace=False)
    y[torch.as_tensor(bad, device=dev)] = torch.randn((8, s.K), device=dev) * float(y.std())
    y = y.contiguous()
    R0 = true_poses[0, :9].reshape(3, 3).cpu().numpy()
    true_x = tmpl @ R0.T + true_poses[0, 9:].cpu().numpy()
    sigmas = [1.5 * w.sigma, 1.25 * w.sigma, w.sigma]

    def run():
        t = [time.perf_counter()]
        top, _ = Z.coarse_search(g, p0, replace(s, sigma=sigmas[0]), y, tmpl, 0.4e-3, 9, ctx=ctx)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        x2 = Z.refine(g, p0, s, y, top[:, 0, :], sigmas, 20, 2e-5, ctx=ctx).cpu().numpy()
        t.append(time.perf_counter())
        R, tr, inl, _ = rigid.ransac_rigid(tmpl, x2, threshold=50e-6, iterations=400, seed=3)
        t.append(time.perf_counter())
        p6 = rigid.finetune(g, p0, s, y, tmpl, np.concatenate([rigid.euler_from_matrix(R), tr]), inl, steps=80,
                            lr_angle=3e-4, lr_t=3e-6, ctx=ctx).cpu().numpy()
        t.append(time.perf_counter())
        Rf = _euler_matrix(p6[:3])
        err = np.linalg.norm(tmpl @ Rf.T + p6[3:] - true_x, axis=1)
        return np.diff(t) * 1e3, err, int(inl.sum())

    run()
    ms, err, n_inl = run()
    out = {"workload": "8x8 matrix array (0.5 mm pitch) at an unknown pose over the 128x128x64 vessel-tree "
                       "volume, K=1024, sigma=0.08 mm; 8 of 64 signal rows corrupted",
           "stage2_coarse_ms": ms[0], "stage2_coarse_candidates": 64 * 729, "stage2_refine_ms": ms[1],
           "stage2_refine_steps": 60, "stage3_ransac_ms": ms[2], "stage3_inliers": n_inl,
           "stage4_finetune_ms": ms[3], "stage4_steps": 80, "final_element_error_max_um": 1e6 * float(err.max())}
    print("[bench] pose recovery: coarse %.0f ms, refine %.0f ms, RANSAC %.0f ms, fine-tune %.0f ms; "
          "max element error %.2f um" % (ms[0], ms[1], ms[2], ms[3], 1e6 * err.max()), file=sys.stderr, flush=True)
    return out


def _euler_matrix(a):
    """R = Rz(a2) Ry(a1) Rx(a0) (host, for scoring the recovered pose)."""
    import numpy as np
    cx, sx, cy, sy, cz, sz = np.cos(a[0]), np.sin(a[0]), np.cos(a[1]), np.sin(a[1]), np.cos(a[2]), np.sin(a[2])
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def main():
    a = parse()
    if a.write_traffic:
        write_traffic(*a.write_traffic)
        return
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus %d requested)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2604_09643_amd import _lib as L
    from paper_2604_09643_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if a.c3_adam:
        print(json.dumps({"c3_joint_optimisation": c3_joint(a.c3_adam, checkpoint=a.c3_checkpoint,
                                                            checkpoint_every=a.c3_checkpoint_every,
                                                            resume=a.c3_resume)}), flush=True)
        return
    if a.copy_calibration:
        # 1 GiB device-to-device copy of a buffer that was evicted from the caches by
        # writing another 1 GiB first: the reference for FETCH_SIZE / WRITE_SIZE
        src = torch.ones(256 << 20, dtype=torch.float32, device=dev)
        evict = torch.zeros(256 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst, evict
    w = W.c2()
    g = L.Grid(*w.shape, tuple(w.origin), w.spacing)
    s = L.Sampling(w.c, w.fs, w.K, w.sigma, w.trunc)
    p0 = torch.tensor(w.p0.astype(np.float32), device=dev)
    elem = torch.tensor(w.elem, device=dev)
    poses = torch.tensor(w.poses, device=dev)
    y = torch.tensor(np.random.default_rng(11).normal(scale=1e-3, size=(w.F, w.M, w.K)).astype(np.float32),
                     device=dev)
    gp0 = torch.empty_like(p0)
    ctx = L.context(0)
    ctx.reserve(ctx.scratch_bytes(g, w.M, w.F, s))
    n_upd = L.count_updates(g, elem, poses, s, ctx=ctx)
    print("[bench] workload C2: %d voxels x %d elements, K=%d; %d in-window updates per pass"
          % (w.n_voxels, w.F * w.M, w.K, n_upd), file=sys.stderr, flush=True)

    def step():
        return L.loss_and_grad(g, p0, elem, poses, s, y, want_loss=True, grad_p0=gp0, ctx=ctx)

    for _ in range(a.warmup):
        step()
    st = torch.cuda.current_stream()
    step_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step_ev[i][0].record(st)
        loss = step()
        step_ev[i][1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [e0.elapsed_time(e1) for e0, e1 in step_ev]
    ms_per_step = 1e3 * wall / a.steps
    print("[bench] %d steps: %.3f ms/step, loss %.6e" % (a.steps, ms_per_step, loss), file=sys.stderr, flush=True)

    # per-kernel durations with HIP events on the stream the kernels run on
    sig = torch.empty_like(y)
    r = torch.empty_like(y).normal_()

    def timed(fn, n):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for e0, e1 in ev:
            e0.record(st)
            fn()
            e1.record(st)
        torch.cuda.synchronize()
        return [e0.elapsed_time(e1) for e0, e1 in ev]

    n_t = max(3, min(a.steps, 20))
    t_fwd = timed(lambda: L.radiate_forward(g, p0, elem, poses, s, sig, ctx=ctx), n_t)
    t_adj = timed(lambda: L.radiate_adjoint(g, p0, elem, poses, s, r, grad_p0=gp0, ctx=ctx), n_t)
    ms_fwd, ms_adj = float(np.mean(t_fwd)), float(np.mean(t_adj))
    print("[bench] radiate_forward %.3f ms, radiate_adjoint(p0) %.3f ms" % (ms_fwd, ms_adj),
          file=sys.stderr, flush=True)
    dom_name, dom_ms = ("k_forward", ms_fwd) if ms_fwd >= ms_adj else ("k_adjoint", ms_adj)
    achieved = FLOP_PER_UPDATE * n_upd / (dom_ms * 1e-3) / 1e12
    fma_rate, exp_rate = ctx.probe_rates()
    pairs = w.n_voxels * w.F * w.M
    print("[bench] probes: %.1f TFLOP/s FP32 FMA (unpacked), %.3e v_exp_f32/s" % (2 * fma_rate / 1e12, exp_rate),
          file=sys.stderr, flush=True)

    def busy():            # about 1.6 s of queued forward calls: the device reading below is under load
        for _ in range(60):
            L.radiate_forward(g, p0, elem, poses, s, sig, ctx=ctx)
    # the loaded reading only in full runs, so that the short profiled runs launch what they did
    device = device_info(dev, fma_rate, None if a.no_large else busy)

    value = 2.0 * n_upd / (ms_per_step * 1e-3)
    jt = int(np.floor(w.trunc * w.sigma * w.fs / w.c + 0.5))
    table_rows = w.F * w.M * (w.K + 2 * jt)
    adj_flop = FLOP_PER_PAIR_ADJ_MOMENT * pairs + 2.0 * 8 * (2 * jt + 1) * table_rows
    adj_achieved = adj_flop / (ms_adj * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": value, "unit": "updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "single freehand sweep (forward + p0-adjoint): 128x128x64 voxels at 0.1 mm, "
                               "64 frames x 128-element linear array (pitch 0.3 mm), K=1024 at 40 MHz, "
                               "sigma=0.08 mm, 40-branch vessel tree + N(0,0.01^2) background; step = "
                               "loss_and_grad (forward, residual/loss, dL/dp0)",
                   "updates_per_pass": n_upd, "ms_forward": ms_fwd, "ms_adjoint_p0": ms_adj},
        "timing": {"step_ms": spread(step_ms), "forward_ms": spread(t_fwd), "adjoint_p0_ms": spread(t_adj),
                   "events": "HIP events on the kernels' stream; ms_per_step is the wall clock over the timed steps"},
        "device": device,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic_from_profile(dom_name),
                     "kernel": dom_name, "timed": "radiate_forward call (HIP events on its stream)",
                     "flop_per_update": FLOP_PER_UPDATE, "updates_per_launch": n_upd,
                     "measured_fp32_fma_peak_tflops": 2 * fma_rate / 1e12,
                     "transcendental": {
                         "algorithmic_exp_per_s": EXP_PER_UPDATE * n_upd / (ms_fwd * 1e-3),
                         "executed_per_s": TRANS_PER_PAIR_FWD * pairs / (ms_fwd * 1e-3),
                         "measured_exp_peak_per_s": exp_rate,
                         "frac_executed": TRANS_PER_PAIR_FWD * pairs / (ms_fwd * 1e-3) / exp_rate}},
        "adjoint_roofline": {"kernel": "k_adjoint_mom with k_moment_table (dL/dp0, moment form)", "bound": "alu",
                             "achieved": adj_achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                             "frac": adj_achieved / PEAK_FP32_TFLOPS, "flop_per_pair": FLOP_PER_PAIR_ADJ_MOMENT,
                             "pairs_per_launch": pairs, "table_rows": table_rows,
                             "flop_per_table_row": 2 * 8 * (2 * jt + 1),
                             "timed": "radiate_adjoint call, dL/dp0 only (HIP events on its stream)",
                             "updates_per_s": n_upd / (ms_adj * 1e-3)},
    }
    if not a.no_serving:
        sv = serving_bench(a.serving_requests, a.serving_rate)
        out["serving"] = sv
        out["p50_frame_pose_latency_ms"] = sv["batched"]["pose_p50_ms"]
        out["p99_frame_pose_latency_ms"] = sv["batched"]["pose_p99_ms"]
        print("[bench] serving at %.0f req/s: batched p50 %.1f ms p99 %.1f ms (%.1f req/s); unbatched p50 %.1f p99 "
              "%.1f (%.1f req/s)" % (sv["offered_rate_req_s"], sv["batched"]["p50_ms"], sv["batched"]["p99_ms"],
                                     sv["batched"]["throughput_req_s"], sv["unbatched"]["p50_ms"],
                                     sv["unbatched"]["p99_ms"], sv["unbatched"]["throughput_req_s"]),
              file=sys.stderr, flush=True)
    if not a.no_large:
        out["larger_configs"] = large_configs(ctx)
        out["pose_recovery"] = pose_pipeline_bench(ctx)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
