"""Continuous-batching request loop for per-frame pose refinement and volume updates.

As the probe moves, requests arrive for the newest frame.  A pose-refinement request
runs a fixed number of gradient steps (Adam on the 6-DoF pose, loss sum (s - y)^2 over one
frame) against a box of the resident volume.  A volume-update request runs one gradient
step on its box.  Requests differ in element count M, samples K and box size.

The loop is iteration-level continuous batching:

* a request is admitted when a slot is free, its device footprint fits the memory cap and,
  with a work budget, the step work of the active requests plus its own stays within the
  budget (a request is always admitted into an empty batch; a queue of queue_lifts_budget
  arrived requests lifts the budget).  A request whose work fills the GPU then runs alone, as
  in FIFO, while smaller ones share ticks, and under a queue every request shares; admission
  is strict FIFO: the oldest waiting request goes first, and no request overtakes it;
* each tick runs one gradient step for every active request in a single batched step
  of the library (``ra_batch_step``).  New arrivals join at the next tick and finished
  requests leave, so their work overlaps on the device with requests that are mid-way;
* the step is captured once into a HIP graph over device-side work lists sized for the
  slot capacity and replayed every tick (``graph=True``).

``Scheduler`` holds the host logic and talks to an executor.  ``GpuExecutor`` is the
device implementation.  Tests drive the scheduler with a fake executor on the CPU.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

POSE, VOLUME = 0, 1


# ----------------------------------------------------------------------------------------------
# requests and results
# ----------------------------------------------------------------------------------------------

@dataclass
class Request:
    """One request.  ``box`` = (i0, j0, k0, nx, ny, nz) in voxels of the resident volume;
    ``elem`` [M,3] array template; ``pose6`` (w, t) initial (pose) or known (volume) pose;
    ``y`` [M,K] measured signals; ``steps`` gradient steps to run."""
    rid: int
    kind: int
    box: tuple
    elem: np.ndarray
    pose6: np.ndarray
    y: np.ndarray
    steps: int
    arrival: float = 0.0
    lr_w: float = 2e-3
    lr_t: float = 2e-5

    @property
    def M(self):
        return self.elem.shape[0]

    @property
    def K(self):
        return self.y.shape[1]


@dataclass
class Result:
    rid: int
    kind: int
    pose6: Optional[np.ndarray]
    losses: List[float]
    grad_p0: Optional[np.ndarray]
    arrival: float
    admitted: float
    finished: float

    @property
    def latency(self):
        return self.finished - self.arrival


# ----------------------------------------------------------------------------------------------
# device arena (first fit)
# ----------------------------------------------------------------------------------------------

class Arena:
    """First-fit allocator over [0, size) with 256-byte alignment; offsets only."""

    ALIGN = 256

    def __init__(self, size: int):
        self.size = int(size)
        self.free = [(0, self.size)]
        self.used = 0

    def alloc(self, n: int) -> Optional[int]:
        n = (int(n) + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, ln - n)
                self.used += n
                return off
        return None

    def release(self, off: int, n: int):
        n = (int(n) + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        self.used -= n
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged


# ----------------------------------------------------------------------------------------------
# scheduler (host logic only)
# ----------------------------------------------------------------------------------------------

class Scheduler:
    """Iteration-level continuous batching over an executor with ``slots`` slots.

    The executor provides: footprint(req) -> bytes, admit(req, slot) -> bool (False when its
    memory is exhausted), step(slots) (one gradient step for each listed slot; may raise),
    collect(slot, req) -> Result fields (pose6, losses, grad_p0), release(slot), and, for a
    work budget, work(req) -> the work of one of its steps (any unit the budget shares)."""

    def __init__(self, executor, slots: int, mem_cap: int, clock=time.perf_counter, work_budget=None,
                 queue_lifts_budget: Optional[int] = None, queue_timeout: Optional[float] = None):
        self.ex = executor
        self.slots = slots
        self.mem_cap = int(mem_cap)
        self.clock = clock
        self.waiting: List[Request] = []
        self.active: Dict[int, dict] = {}
        self.free_slots = list(range(slots))
        self.mem_used = 0
        self.results: List[Result] = []
        self.failed: List[tuple] = []
        self.ticks = 0
        self.batch_sizes: List[int] = []
        self.work_budget = work_budget
        self.queue_lifts_budget = queue_lifts_budget
        self.queue_timeout = queue_timeout     # seconds an arrived request may wait for admission
        self.active_work = 0.0

    def submit(self, req: Request):
        fp = self.ex.footprint(req)
        if fp > self.mem_cap:
            self.failed.append((req.rid, "footprint %d exceeds the memory cap %d" % (fp, self.mem_cap)))
            return False
        self.waiting.append(req)
        return True

    def _expire(self, now: float):
        """Fail the arrived requests that have waited longer than queue_timeout for admission."""
        if self.queue_timeout is None:
            return
        keep = []
        for r in self.waiting:
            if r.arrival <= now and now - r.arrival > self.queue_timeout:
                self.failed.append((r.rid, "queue timeout: waited %.3f s" % (now - r.arrival)))
            else:
                keep.append(r)
        self.waiting = keep

    def _admit(self, now: float):
        # below the queue threshold a request whose work fills the GPU keeps it to itself (sharing
        # would only stretch it over more ticks); once queue_lifts_budget requests have arrived and
        # wait, throughput matters more and the budget is lifted
        budget = self.work_budget
        if budget is not None and self.queue_lifts_budget is not None:
            if sum(1 for r in self.waiting if r.arrival <= now) >= self.queue_lifts_budget:
                budget = None
        # strict FIFO over requests that have arrived
        while self.waiting and self.waiting[0].arrival <= now and self.free_slots:
            req = self.waiting[0]
            fp = self.ex.footprint(req)
            if self.mem_used + fp > self.mem_cap:
                break
            wk = self.ex.work(req) if self.work_budget is not None else 0.0
            if budget is not None and self.active and self.active_work + wk > budget:
                break
            slot = self.free_slots[0]
            if not self.ex.admit(req, slot):
                break
            self.free_slots.pop(0)
            self.waiting.pop(0)
            self.mem_used += fp
            self.active_work += wk
            self.active[slot] = {"req": req, "left": req.steps, "admitted": now, "fp": fp, "work": wk}

    def tick(self) -> bool:
        """Admit, run one batched step, retire.  Returns False when idle (nothing active)."""
        now = self.clock()
        self._expire(now)
        self._admit(now)
        if not self.active:
            return False
        slots = sorted(self.active)
        self.batch_sizes.append(len(slots))
        self.ticks += 1
        try:
            self.ex.step(slots)
        except Exception as exc:              # a failed launch fails this batch's requests only
            for s in slots:
                st = self.active.pop(s)
                self.failed.append((st["req"].rid, repr(exc)))
                self.ex.release(s)
                self.free_slots.append(s)
                self.mem_used -= st["fp"]
                self.active_work -= st["work"]
            self.free_slots.sort()
            return True
        done = []
        for s in slots:
            self.active[s]["left"] -= 1
            if self.active[s]["left"] <= 0:
                done.append(s)
        if done:
            fin = self.clock()
            for s in done:
                st = self.active.pop(s)
                pose6, losses, grad = self.ex.collect(s, st["req"])
                req = st["req"]
                self.results.append(Result(req.rid, req.kind, pose6, losses, grad, req.arrival, st["admitted"], fin))
                self.ex.release(s)
                self.free_slots.append(s)
                self.mem_used -= st["fp"]
                self.active_work -= st["work"]
            self.free_slots.sort()
        return True

    def run(self, requests: List[Request], realtime: bool = True, t0: Optional[float] = None):
        """Serve `requests` (arrival = offset in seconds from t0) until all are finished."""
        t0 = self.clock() if t0 is None else t0
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            r.arrival = t0 + r.arrival
            self.submit(r)
        while self.waiting or self.active:
            busy = self.tick()
            if not busy and self.waiting:
                wait = self.waiting[0].arrival - self.clock()
                if realtime and wait > 0:
                    time.sleep(min(wait, 0.01))
                elif not realtime:
                    self.waiting[0].arrival = min(self.waiting[0].arrival, self.clock())
        return self.results


# ----------------------------------------------------------------------------------------------
# ctypes mirrors of the batch structures in include/radiate.h
# ----------------------------------------------------------------------------------------------

class CBatchRequest(ctypes.Structure):
    _fields_ = [("p0", ctypes.c_void_p), ("s", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("grad_p0", ctypes.c_void_p), ("pose_part", ctypes.c_void_p), ("pose6", ctypes.c_void_p),
                ("adam", ctypes.c_void_p), ("elem", ctypes.c_void_p), ("xe", ctypes.c_void_p),
                ("loss", ctypes.c_void_p), ("q", ctypes.c_void_p), ("kind", ctypes.c_int32), ("nreg", ctypes.c_int32),
                ("lr_w", ctypes.c_double), ("lr_t", ctypes.c_double)]


class CBatchInfo(ctypes.Structure):
    _fields_ = [("nreg", ctypes.c_int32), ("jt", ctypes.c_int32), ("exact", ctypes.c_int32),
                ("pair_d", ctypes.c_int32), ("lmax", ctypes.c_int32), ("nvpad", ctypes.c_int32),
                ("rx", ctypes.c_int32), ("ry", ctypes.c_int32), ("rz", ctypes.c_int32),
                ("moment", ctypes.c_int32), ("nbin", ctypes.c_int32), ("q_bytes", ctypes.c_int64)]


class CBatch(ctypes.Structure):
    _fields_ = [("geos", ctypes.c_void_p), ("reqs", ctypes.c_void_p), ("vtab", ctypes.c_void_p),
                ("itab", ctypes.c_void_p), ("items_fwd", ctypes.c_void_p), ("items_pose", ctypes.c_void_p),
                ("items_vol", ctypes.c_void_p), ("items_elem", ctypes.c_void_p), ("counts", ctypes.c_void_p),
                ("jt", ctypes.c_int32), ("exact", ctypes.c_int32), ("pair_d", ctypes.c_int32),
                ("lmax", ctypes.c_int32), ("nvpad", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("moment", ctypes.c_int32), ("nbin", ctypes.c_int32), ("coef", ctypes.c_void_p)]


def _bind(lib):
    if getattr(lib, "_batch_bound", False):
        return
    P = ctypes.c_void_p
    lib.ra_batch_geo_bytes.restype = ctypes.c_size_t
    lib.ra_batch_geo_bytes.argtypes = []
    lib.ra_batch_describe.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, P, P,
                                      ctypes.POINTER(CBatchInfo)]
    lib.ra_batch_describe.restype = ctypes.c_int
    lib.ra_batch_tables.argtypes = [P, P, P, P, P]
    lib.ra_batch_tables.restype = ctypes.c_int
    lib.ra_batch_step.argtypes = [P, ctypes.POINTER(CBatch), ctypes.c_uint32, P]
    lib.ra_batch_step.restype = ctypes.c_int
    lib._batch_bound = True


# ----------------------------------------------------------------------------------------------
# GPU executor
# ----------------------------------------------------------------------------------------------

class GpuExecutor:
    """Device state and the batched step.

    The resident volume (float32 [nx][ny][nz]) stays on the device.  Per-request buffers
    come from one device arena.  Descriptor tables have fixed addresses and capacity for
    `slots` requests, so one captured graph serves every batch."""

    def __init__(self, volume, grid, samp, slots: int = 16, arena_bytes: int = 1 << 31,
                 max_items: int = 1 << 18, graph: bool = True, apply_updates: bool = True,
                 lr_volume: float = 1e-3, grid_blocks: int = 1024, fail_launch_at: Optional[int] = None):
        import torch
        from . import _lib as L
        self.torch, self.L = torch, L
        self.ctx = L.context(volume.device.index)
        self.lib = self.ctx.lib
        _bind(self.lib)
        self.dev = volume.device
        self.volume = volume
        assert volume.dtype == torch.float32 and volume.is_contiguous()
        self.grid, self.samp = grid, samp
        self.slots = slots
        self.graph_on = graph
        self.apply_updates = apply_updates
        self.lr_volume = lr_volume
        self.grid_blocks = grid_blocks
        self.geo_bytes = int(self.lib.ra_batch_geo_bytes())
        self.arena = Arena(arena_bytes)
        self.buf = torch.empty(arena_bytes, dtype=torch.uint8, device=self.dev)
        self.max_items = max_items
        dev = self.dev
        self.d_geos = torch.zeros(slots * self.geo_bytes, dtype=torch.uint8, device=dev)
        self.d_reqs = torch.zeros(slots * ctypes.sizeof(CBatchRequest), dtype=torch.uint8, device=dev)
        self.d_items = torch.zeros((4, max_items, 2), dtype=torch.int32, device=dev)
        self.d_counts = torch.zeros(8, dtype=torch.int32, device=dev)
        self.h_geos = torch.zeros_like(self.d_geos, device="cpu").pin_memory()
        self.h_reqs = torch.zeros_like(self.d_reqs, device="cpu").pin_memory()
        self.h_items = torch.zeros((4, max_items, 2), dtype=torch.int32).pin_memory()
        self.h_counts = torch.zeros(8, dtype=torch.int32).pin_memory()
        # moment-form coefficients of the batched adjoints (8 per window step, at most 81 steps)
        self.d_coef = torch.zeros(8 * 81, dtype=torch.float32, device=dev)
        # one loss per slot, read back with one copy per tick
        self.d_loss = torch.zeros(slots, dtype=torch.float32, device=dev)
        self.h_loss = torch.zeros(slots, dtype=torch.float32).pin_memory()
        # GPU time of the batched steps (HIP events around each launch or replay)
        self.gpu_ms = 0.0
        self.n_steps = 0
        self.launches = 0
        self.fail_launch_at = fail_launch_at       # test hook: the step with this number raises
        self.ev0 = torch.cuda.Event(enable_timing=True)
        self.ev1 = torch.cuda.Event(enable_timing=True)
        self.state: Dict[int, dict] = {}
        self.tables = None
        self.info0 = None
        self.cgraph = None
        self.graph_key = None
        self.stream = torch.cuda.current_stream(dev)

    # -- geometry ----------------------------------------------------------------------------
    def _box_grid(self, box):
        i0, j0, k0, nx, ny, nz = box
        g = self.grid
        o = (g.origin[0] + i0 * g.spacing, g.origin[1] + j0 * g.spacing, g.origin[2] + k0 * g.spacing)
        return self.L.Grid(nx, ny, nz, o, g.spacing)

    def _describe(self, req: Request):
        L = self.L
        g = self.grid
        bg = self._box_grid(req.box)
        samp = L.Sampling(self.samp.c, self.samp.fs, req.K, self.samp.sigma, self.samp.trunc,
                          getattr(self.samp, "kernel", 0), getattr(self.samp, "nu", 1.0))
        geo = (ctypes.c_uint8 * self.geo_bytes)()
        info = CBatchInfo()
        self.ctx.check(self.lib.ra_batch_describe(self.ctx.ptr, ctypes.byref(bg.c()), g.ny * g.nz, g.nz, req.M,
                                                  ctypes.byref(samp.cs()), geo, ctypes.byref(info)))
        return bytes(geo), info

    def work(self, req: Request) -> float:
        """(voxel, element) pairs of one step: the forward and the adjoint each visit them once."""
        return float(req.box[3] * req.box[4] * req.box[5] * req.M)

    def footprint(self, req: Request) -> int:
        M, K = req.M, req.K
        _, info = self._describe(req)
        nbox = req.box[3] * req.box[4] * req.box[5]
        n = 2 * M * K * 4 + M * 3 * 8 + M * 6 * 4 + 6 * 8 + 13 * 8
        if req.kind == POSE:
            n += info.nreg * M * 3 * 8
        else:
            n += nbox * 4
        n += info.q_bytes
        return n + 13 * Arena.ALIGN

    # -- slots --------------------------------------------------------------------------------
    def admit(self, req: Request, slot: int) -> bool:
        torch = self.torch
        i0, j0, k0, nx, ny, nz = req.box
        g = self.grid
        if not (0 <= i0 and i0 + nx <= g.nx and 0 <= j0 and j0 + ny <= g.ny and 0 <= k0 and k0 + nz <= g.nz):
            raise ValueError("request %d: box outside the resident volume" % req.rid)
        geo, info = self._describe(req)
        if self.info0 is None:
            self.info0 = info
            self.tables = torch.empty((2, info.nvpad, 4), dtype=torch.int32, device=self.dev)
            gbuf = ctypes.create_string_buffer(geo, len(geo))
            self.ctx.check(self.lib.ra_batch_tables(self.ctx.ptr, gbuf, ctypes.c_void_p(self.tables[0].data_ptr()),
                                                    ctypes.c_void_p(self.tables[1].data_ptr()),
                                                    ctypes.c_void_p(self.stream.cuda_stream)))
        i0_ = self.info0
        if (info.rx, info.ry, info.rz, info.nvpad, info.jt, info.exact, info.pair_d, info.moment, info.nbin) != \
                (i0_.rx, i0_.ry, i0_.rz, i0_.nvpad, i0_.jt, i0_.exact, i0_.pair_d, i0_.moment, i0_.nbin):
            raise ValueError("request %d: geometry incompatible with the batch" % req.rid)
        M, K = req.M, req.K
        sizes = {"s": M * K * 4, "y": M * K * 4, "elem": M * 3 * 8, "xe": M * 6 * 4, "pose6": 6 * 8,
                 "adam": 13 * 8}
        if req.kind == POSE:
            sizes["pose_part"] = info.nreg * M * 3 * 8
        else:
            sizes["grad"] = nx * ny * nz * 4
        if info.q_bytes > 0:
            sizes["q"] = info.q_bytes
        offs = {}
        for k, n in sizes.items():
            o = self.arena.alloc(n)
            if o is None:
                for kk, oo in offs.items():
                    self.arena.release(oo, sizes[kk])
                return False
            offs[k] = o
        base = self.buf.data_ptr()

        def view(key, dtype, shape):
            return self.buf[offs[key]:offs[key] + sizes[key]].view(dtype).view(shape)
        st = {"req": req, "geo": geo, "info": info, "offs": offs, "sizes": sizes, "losses": [],
              "y": view("y", torch.float32, (M, K)), "elem": view("elem", torch.float64, (M, 3)),
              "pose6": view("pose6", torch.float64, (6,)), "adam": view("adam", torch.float64, (13,))}
        st["y"].copy_(torch.from_numpy(np.ascontiguousarray(req.y, dtype=np.float32)), non_blocking=False)
        st["elem"].copy_(torch.from_numpy(np.ascontiguousarray(req.elem, dtype=np.float64)))
        st["pose6"].copy_(torch.from_numpy(np.ascontiguousarray(req.pose6, dtype=np.float64)))
        st["adam"].zero_()
        if req.kind == VOLUME:
            st["grad"] = view("grad", torch.float32, (nx, ny, nz))
        cr = CBatchRequest()
        cr.p0 = self.volume.data_ptr() + 4 * ((i0 * g.ny + j0) * g.nz + k0)
        cr.s = base + offs["s"]
        cr.y = base + offs["y"]
        cr.grad_p0 = base + offs["grad"] if req.kind == VOLUME else None
        cr.pose_part = base + offs["pose_part"] if req.kind == POSE else None
        cr.pose6 = base + offs["pose6"]
        cr.adam = base + offs["adam"]
        cr.elem = base + offs["elem"]
        cr.xe = base + offs["xe"]
        cr.loss = self.d_loss.data_ptr() + 4 * slot
        cr.q = base + offs["q"] if "q" in offs else None
        cr.kind = req.kind
        cr.nreg = info.nreg
        cr.lr_w = req.lr_w if req.kind == POSE else self.lr_volume
        cr.lr_t = req.lr_t
        st["creq"] = bytes(cr)
        self.state[slot] = st
        return True

    def release(self, slot: int):
        st = self.state.pop(slot, None)
        if st is None:
            return
        for k, o in st["offs"].items():
            self.arena.release(o, st["sizes"][k])

    # -- the batched step ----------------------------------------------------------------------
    def _tables(self, slots: List[int]):
        """Fill the host tables for this batch: descriptors by slot index, work lists."""
        gb, rb = self.geo_bytes, ctypes.sizeof(CBatchRequest)
        hg, hr = self.h_geos.numpy(), self.h_reqs.numpy()
        n_slots = max(slots) + 1
        fwd, pose, vol, elem = [], [], [], []
        for s in slots:
            st = self.state[s]
            hg[s * gb:(s + 1) * gb] = np.frombuffer(st["geo"], dtype=np.uint8)
            hr[s * rb:(s + 1) * rb] = np.frombuffer(st["creq"], dtype=np.uint8)
            nreg = st["info"].nreg
            pairs = np.stack([np.full(nreg, s, np.int32), np.arange(nreg, dtype=np.int32)], axis=1)
            fwd.append(pairs)
            (pose if st["req"].kind == POSE else vol).append(pairs)
            M = st["req"].M
            elem.append(np.stack([np.full(M, s, np.int32), np.arange(M, dtype=np.int32)], axis=1))
        # slots below n_slots that are not in this batch take part with zero work
        for s in range(n_slots):
            if s not in self.state or s not in slots:
                hr[s * rb:(s + 1) * rb] = 0
                cr = CBatchRequest()
                cr.kind = -1
                hr[s * rb:(s + 1) * rb] = np.frombuffer(bytes(cr), dtype=np.uint8)
                hg[s * gb:(s + 1) * gb] = 0
        hi = self.h_items.numpy()
        counts = []
        for i, lst in enumerate((fwd, pose, vol, elem)):
            arr = np.concatenate(lst) if lst else np.zeros((0, 2), np.int32)
            if arr.shape[0] > self.max_items:
                raise RuntimeError("batch has %d work items, capacity %d" % (arr.shape[0], self.max_items))
            hi[i, :arr.shape[0]] = arr
            counts.append(arr.shape[0])
        hc = self.h_counts.numpy()
        hc[:5] = counts + [n_slots]
        return counts

    def _cbatch(self):
        i = self.info0
        b = CBatch()
        b.geos = self.d_geos.data_ptr()
        b.reqs = self.d_reqs.data_ptr()
        b.vtab = self.tables[0].data_ptr()
        b.itab = self.tables[1].data_ptr()
        b.items_fwd = self.d_items[0].data_ptr()
        b.items_pose = self.d_items[1].data_ptr()
        b.items_vol = self.d_items[2].data_ptr()
        b.items_elem = self.d_items[3].data_ptr()
        b.counts = self.d_counts.data_ptr()
        b.jt, b.exact, b.pair_d, b.lmax, b.nvpad = i.jt, i.exact, i.pair_d, i.lmax, i.nvpad
        b.grid_blocks = self.grid_blocks
        b.moment, b.nbin = i.moment, i.nbin
        b.coef = self.d_coef.data_ptr()
        return b

    def _launch(self):
        flags = 1 if self.apply_updates else 0
        b = self._cbatch()
        self.ctx.check(self.lib.ra_batch_step(self.ctx.ptr, ctypes.byref(b), flags,
                                              ctypes.c_void_p(self.torch.cuda.current_stream(self.dev).cuda_stream)))

    def step(self, slots: List[int]):
        torch = self.torch
        self.launches += 1
        if self.fail_launch_at is not None and self.launches == self.fail_launch_at:
            # test hook: this step fails on the host before anything is queued on the device
            raise RuntimeError("injected launch failure at step %d" % self.launches)
        counts = self._tables(slots)
        self.d_geos.copy_(self.h_geos, non_blocking=True)
        self.d_reqs.copy_(self.h_reqs, non_blocking=True)
        for i in range(4):
            if counts[i]:
                self.d_items[i, :counts[i]].copy_(self.h_items[i, :counts[i]], non_blocking=True)
        self.d_counts.copy_(self.h_counts, non_blocking=True)
        stream = torch.cuda.current_stream(self.dev)
        self.ev0.record(stream)
        if self.graph_on and self.cgraph is not None:
            self.cgraph.replay()
        else:
            self._launch()
            if self.graph_on:
                # capture once, after an eager step has set the kernels' attributes; the
                # captured graph reads the tables at their fixed addresses on every replay
                torch.cuda.synchronize(self.dev)
                self.cgraph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(self.cgraph):
                    self._launch()
        self.ev1.record(stream)
        self.h_loss.copy_(self.d_loss, non_blocking=True)
        stream.synchronize()
        self.gpu_ms += self.ev0.elapsed_time(self.ev1)
        self.n_steps += 1
        hl = self.h_loss.numpy()
        for s in slots:
            self.state[s]["losses"].append(float(hl[s]))

    def collect(self, slot: int, req: Request):
        st = self.state[slot]
        pose6 = st["pose6"].cpu().numpy().copy() if req.kind == POSE else None
        grad = st["grad"].cpu().numpy().copy() if req.kind == VOLUME else None
        return pose6, list(st["losses"]), grad


def serve(executor, requests: List[Request], slots: int, mem_cap: int, realtime: bool = True, work_budget=None,
          queue_lifts_budget: Optional[int] = None):
    sched = Scheduler(executor, slots, mem_cap, work_budget=work_budget, queue_lifts_budget=queue_lifts_budget)
    res = sched.run(requests, realtime=realtime)
    return sched, res


def serve_unbatched(executor, requests: List[Request], realtime: bool = True):
    """FIFO, one request at a time, each request's steps launched on their own (no graph)."""
    executor.graph_on = False
    sched = Scheduler(executor, 1, 1 << 62)
    return sched, sched.run(requests, realtime=realtime)


def latency_stats(results: List[Result], kind: Optional[int] = None):
    """Arrival-to-result latency percentiles, over every request or over one kind."""
    lat = np.array([r.latency for r in results if kind is None or r.kind == kind])
    if lat.size == 0:
        return {"n": 0}
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3)}
