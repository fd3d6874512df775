"""ctypes binding of ``libradiate.so`` (see include/radiate.h).

Argument marshalling only: every step of the model runs in the library's HIP
kernels.  Tensors are passed by device pointer together with the current HIP
stream; torch provides memory and streams.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

from . import build as _build

RA_OK, RA_EINVAL, RA_EGEOM, RA_ENOMEM, RA_EHIP, RA_ENOTSUP = range(6)
RA_ACCUMULATE = 1
RA_LOSS_ON_DEVICE = 2
RA_SIGNALS_GIVEN = 4
RA_SUMS_AUTO, RA_SUMS_F32, RA_SUMS_F64 = range(3)
_NAMES = {0: "RA_OK", 1: "RA_EINVAL", 2: "RA_EGEOM", 3: "RA_ENOMEM", 4: "RA_EHIP", 5: "RA_ENOTSUP"}

EXPORTS = ("ra_create", "ra_destroy", "ra_last_error", "ra_status", "ra_reserve", "ra_scratch_bytes",
           "radiate_forward", "radiate_adjoint", "loss_and_grad", "nc_loss_and_grad", "ra_pose_from_axis_angle",
           "ra_pose_grad_axis_angle", "ra_pose_from_euler", "ra_pose_grad_euler", "ra_count_updates", "ra_batch_geo_bytes", "ra_batch_describe",
           "ra_batch_tables", "ra_batch_step", "ra_tgv_scratch_bytes", "tgv_loss_and_grad", "ra_set_forward_sums",
           "ra_probe_rates", "radiate_forward_static")


class RadiateError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_NAMES.get(code, str(code)), msg))
        self.code = code


class CGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("origin", ctypes.c_double * 3), ("spacing", ctypes.c_double)]


class CSampling(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("fs", ctypes.c_double), ("K", ctypes.c_int32),
                ("sigma", ctypes.c_double), ("trunc", ctypes.c_double), ("kernel", ctypes.c_int32),
                ("nu", ctypes.c_double)]


@dataclass(frozen=True)
class Grid:
    """Voxel (i,j,k) centre = origin + (i,j,k) * spacing [m]; volumes are [nx][ny][nz]."""
    nx: int
    ny: int
    nz: int
    origin: tuple
    spacing: float

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    def c(self) -> CGrid:
        return CGrid(self.nx, self.ny, self.nz, (ctypes.c_double * 3)(*[float(v) for v in self.origin]),
                     float(self.spacing))


@dataclass(frozen=True)
class Sampling:
    """t_k = k / fs, k < K; kernel width sigma; window |d - c t| <= trunc * sigma; kernel
    RA_KERNEL_* (0 Gaussian, 1 exponential, 2 power law with exponent nu, 3 uniform sphere)."""
    c: float
    fs: float
    K: int
    sigma: float
    trunc: float = 6.0
    kernel: int = 0
    nu: float = 1.0

    def cs(self) -> CSampling:
        return CSampling(float(self.c), float(self.fs), int(self.K), float(self.sigma), float(self.trunc),
                         int(self.kernel), float(self.nu))


_lib = None


def lib_path() -> str:
    return _build.LIB


def load(path: str = None):
    """Load the library; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (binds this library to the HIP runtime PyTorch loaded: one runtime per process)
    path = path or lib_path()
    if not os.path.exists(path):
        raise RuntimeError("libradiate.so is not built (%s); run __graft_entry__.build() or "
                           "python -m paper_2604_09643_amd.build" % path)
    L = ctypes.CDLL(path)
    P, I32, U32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    G, S = ctypes.POINTER(CGrid), ctypes.POINTER(CSampling)
    L.ra_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
    L.ra_create.restype = ctypes.c_int
    L.ra_destroy.argtypes = [P]
    L.ra_destroy.restype = None
    L.ra_last_error.argtypes = [P]
    L.ra_last_error.restype = ctypes.c_char_p
    L.ra_status.argtypes = [P, P]
    L.ra_reserve.argtypes = [P, ctypes.c_size_t]
    L.ra_scratch_bytes.argtypes = [G, I32, I32, S]
    L.ra_scratch_bytes.restype = ctypes.c_size_t
    L.radiate_forward.argtypes = [P, G, P, I32, P, P, I32, S, P, P]
    L.radiate_forward_static.argtypes = [P, G, P, I32, P, P, I32, S, P, P]
    L.radiate_adjoint.argtypes = [P, G, P, I32, P, P, I32, S, P, P, P, P, U32, P]
    L.loss_and_grad.argtypes = [P, G, P, I32, P, P, I32, S, P, P, P, P, P, P, U32, P]
    L.nc_loss_and_grad.argtypes = [P, G, P, I32, P, P, I32, S, P, P, ctypes.POINTER(D), P, P, P, P, P, U32, P]
    L.ra_pose_from_axis_angle.argtypes = [P, P, I32, P, P]
    L.ra_pose_grad_axis_angle.argtypes = [P, P, P, I32, P, P]
    L.ra_pose_from_euler.argtypes = [P, P, I32, P, P]
    L.ra_tgv_scratch_bytes.argtypes = [I32, I32, I32]
    L.ra_tgv_scratch_bytes.restype = ctypes.c_size_t
    L.tgv_loss_and_grad.argtypes = [P, I32, I32, I32, P, P, D, D, D, D, ctypes.POINTER(D), P, P, U32, P]
    L.ra_pose_grad_euler.argtypes = [P, P, P, I32, P, P]
    L.ra_count_updates.argtypes = [P, G, I32, P, P, I32, S, ctypes.POINTER(ctypes.c_longlong), P]
    L.ra_set_forward_sums.argtypes = [P, I32]
    L.ra_probe_rates.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(D), P]
    for name in ("ra_status", "ra_reserve", "radiate_forward", "radiate_forward_static", "radiate_adjoint", "loss_and_grad",
                 "ra_pose_from_axis_angle", "ra_pose_grad_axis_angle", "ra_count_updates", "ra_set_forward_sums",
                 "nc_loss_and_grad", "tgv_loss_and_grad", "ra_pose_from_euler", "ra_pose_grad_euler", "ra_probe_rates", "radiate_forward_static"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class Context:
    """One ra_ctx bound to a device."""

    def __init__(self, device: int = 0):
        self.lib = load()
        self.ptr = ctypes.c_void_p()
        self.device = device
        rc = self.lib.ra_create(ctypes.byref(self.ptr), int(device))
        if rc != RA_OK:
            raise RadiateError(rc, "ra_create failed")

    def close(self):
        if self.ptr:
            self.lib.ra_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int):
        if rc != RA_OK:
            raise RadiateError(rc, self.lib.ra_last_error(self.ptr).decode())
        return rc

    def status(self, stream=None) -> int:
        return self.lib.ra_status(self.ptr, _stream(stream))

    def reserve(self, nbytes: int):
        self.check(self.lib.ra_reserve(self.ptr, int(nbytes)))

    def scratch_bytes(self, grid: Grid, M: int, F: int, samp: Sampling) -> int:
        return int(self.lib.ra_scratch_bytes(ctypes.byref(grid.c()), M, F, ctypes.byref(samp.cs())))

    def probe_rates(self, stream=None):
        """Measured (FP32 FMA, v_exp_f32) lane-operation rates per second of this device."""
        f, e = ctypes.c_double(0.0), ctypes.c_double(0.0)
        self.check(self.lib.ra_probe_rates(self.ptr, ctypes.byref(f), ctypes.byref(e), _stream(stream)))
        return f.value, e.value

    def set_forward_sums(self, mode: int):
        """RA_SUMS_AUTO / RA_SUMS_F32 / RA_SUMS_F64: how the forward adds its partial rows."""
        self.check(self.lib.ra_set_forward_sums(self.ptr, int(mode)))


_default = {}


def context(device: int = None) -> Context:
    import torch
    if device is None:
        device = torch.cuda.current_device()
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def _stream(stream=None):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t, dtype, name, numel=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


def _sizes(grid: Grid, elem, poses, samp: Sampling):
    M = elem.shape[0]
    F = poses.shape[0]
    return M, F, grid.nx * grid.ny * grid.nz, F * M * samp.K


def radiate_forward(grid: Grid, p0, elem, poses, samp: Sampling, s=None, ctx: Context = None, stream=None):
    """s[F,M,K] = forward(p0, poses); see include/radiate.h."""
    import torch
    ctx = ctx or context(p0.device.index)
    M, F, nv, ns = _sizes(grid, elem, poses, samp)
    if s is None:
        s = torch.empty((F, M, samp.K), dtype=torch.float32, device=p0.device)
    ctx.check(ctx.lib.radiate_forward(
        ctx.ptr, ctypes.byref(grid.c()), _ptr(p0, torch.float32, "p0", nv), M,
        _ptr(elem, torch.float64, "elem", 3 * M), _ptr(poses, torch.float64, "poses", 12 * F), F,
        ctypes.byref(samp.cs()), _ptr(s, torch.float32, "s", ns), _stream(stream)))
    return s


def radiate_forward_static(grid: Grid, p0, elem, poses, samp: Sampling, s, ctx: Context = None, stream=None):
    """radiate_forward with its scratch in the library's static per-device array: allocates
    nothing (``s`` must be given); see include/radiate.h for the size limit and sharing rules."""
    import torch
    ctx = ctx or context(p0.device.index)
    M, F, nv, ns = _sizes(grid, elem, poses, samp)
    ctx.check(ctx.lib.radiate_forward_static(
        ctx.ptr, ctypes.byref(grid.c()), _ptr(p0, torch.float32, "p0", nv), M,
        _ptr(elem, torch.float64, "elem", 3 * M), _ptr(poses, torch.float64, "poses", 12 * F), F,
        ctypes.byref(samp.cs()), _ptr(s, torch.float32, "s", ns), _stream(stream)))
    return s


def radiate_adjoint(grid: Grid, p0, elem, poses, samp: Sampling, r, grad_p0=None, grad_pose=None,
                    grad_elem=None, accumulate: bool = False, ctx: Context = None, stream=None):
    """Adjoint into the given (preallocated) outputs; any may be None."""
    import torch
    ctx = ctx or context(r.device.index)
    M, F, nv, ns = _sizes(grid, elem, poses, samp)
    ctx.check(ctx.lib.radiate_adjoint(
        ctx.ptr, ctypes.byref(grid.c()), _ptr(p0, torch.float32, "p0", nv), M,
        _ptr(elem, torch.float64, "elem", 3 * M), _ptr(poses, torch.float64, "poses", 12 * F), F,
        ctypes.byref(samp.cs()), _ptr(r, torch.float32, "r", ns),
        _ptr(grad_p0, torch.float32, "grad_p0", nv), _ptr(grad_pose, torch.float64, "grad_pose", 12 * F),
        _ptr(grad_elem, torch.float64, "grad_elem", 3 * M * F), RA_ACCUMULATE if accumulate else 0,
        _stream(stream)))
    return grad_p0, grad_pose, grad_elem


def loss_and_grad(grid: Grid, p0, elem, poses, samp: Sampling, y, want_loss: bool = True, s_out=None,
                  grad_p0=None, grad_pose=None, grad_elem=None, accumulate: bool = False,
                  ctx: Context = None, stream=None, loss_out=None, signals_given: bool = False):
    """L = sum (s - y)^2 and its gradients; returns L (float) or None.  With ``loss_out`` (a
    float64 CUDA tensor of one element) L is written there on the stream instead, without a
    host synchronisation (RA_LOSS_ON_DEVICE), and the call returns None.  With
    ``signals_given`` (RA_SIGNALS_GIVEN), ``s_out`` holds the signals an earlier call wrote for
    the same p0 and poses, and the forward is not run again."""
    import torch
    ctx = ctx or context(p0.device.index)
    M, F, nv, ns = _sizes(grid, elem, poses, samp)
    L = ctypes.c_double(0.0)
    flags = RA_ACCUMULATE if accumulate else 0
    if signals_given:
        if s_out is None:
            raise ValueError("signals_given needs the signals in s_out")
        flags |= RA_SIGNALS_GIVEN
    if loss_out is not None:
        lptr = _ptr(loss_out, torch.float64, "loss_out", 1)
        flags |= RA_LOSS_ON_DEVICE
    else:
        lptr = ctypes.byref(L) if want_loss else None
    ctx.check(ctx.lib.loss_and_grad(
        ctx.ptr, ctypes.byref(grid.c()), _ptr(p0, torch.float32, "p0", nv), M,
        _ptr(elem, torch.float64, "elem", 3 * M), _ptr(poses, torch.float64, "poses", 12 * F), F,
        ctypes.byref(samp.cs()), _ptr(y, torch.float32, "y", ns), lptr,
        _ptr(s_out, torch.float32, "s_out", ns), _ptr(grad_p0, torch.float32, "grad_p0", nv),
        _ptr(grad_pose, torch.float64, "grad_pose", 12 * F),
        _ptr(grad_elem, torch.float64, "grad_elem", 3 * M * F), flags, _stream(stream)))
    return L.value if (want_loss and loss_out is None) else None


def nc_loss_and_grad(grid: Grid, p0, elem, poses, samp: Sampling, y, weight=None, want_loss: bool = True,
                     loss_elem=None, s_out=None, grad_p0=None, grad_pose=None, grad_elem=None,
                     accumulate: bool = False, ctx: Context = None, stream=None):
    """Stage 2 negative correlation: L = sum_e w_e L_e, L_e = -Cov(s_e, y_e)/(sigma_sim sigma_meas),
    and its gradients; returns L (float) or None.  loss_elem (float64 [F, M]) receives L_e."""
    import torch
    ctx = ctx or context(p0.device.index)
    M, F, nv, ns = _sizes(grid, elem, poses, samp)
    L = ctypes.c_double(0.0)
    ctx.check(ctx.lib.nc_loss_and_grad(
        ctx.ptr, ctypes.byref(grid.c()), _ptr(p0, torch.float32, "p0", nv), M,
        _ptr(elem, torch.float64, "elem", 3 * M), _ptr(poses, torch.float64, "poses", 12 * F), F,
        ctypes.byref(samp.cs()), _ptr(y, torch.float32, "y", ns), _ptr(weight, torch.float32, "weight", M * F),
        ctypes.byref(L) if want_loss else None, _ptr(loss_elem, torch.float64, "loss_elem", M * F),
        _ptr(s_out, torch.float32, "s_out", ns), _ptr(grad_p0, torch.float32, "grad_p0", nv),
        _ptr(grad_pose, torch.float64, "grad_pose", 12 * F),
        _ptr(grad_elem, torch.float64, "grad_elem", 3 * M * F), RA_ACCUMULATE if accumulate else 0,
        _stream(stream)))
    return L.value if want_loss else None


def pose_from_axis_angle(pose6, poses=None, ctx: Context = None, stream=None):
    import torch
    ctx = ctx or context(pose6.device.index)
    F = pose6.shape[0]
    if poses is None:
        poses = torch.empty((F, 12), dtype=torch.float64, device=pose6.device)
    ctx.check(ctx.lib.ra_pose_from_axis_angle(ctx.ptr, _ptr(pose6, torch.float64, "pose6", 6 * F), F,
                                              _ptr(poses, torch.float64, "poses", 12 * F), _stream(stream)))
    return poses


def pose_grad_axis_angle(pose6, grad_pose, grad6=None, ctx: Context = None, stream=None):
    import torch
    ctx = ctx or context(pose6.device.index)
    F = pose6.shape[0]
    if grad6 is None:
        grad6 = torch.empty((F, 6), dtype=torch.float64, device=pose6.device)
    ctx.check(ctx.lib.ra_pose_grad_axis_angle(ctx.ptr, _ptr(pose6, torch.float64, "pose6", 6 * F),
                                              _ptr(grad_pose, torch.float64, "grad_pose", 12 * F), F,
                                              _ptr(grad6, torch.float64, "grad6", 6 * F), _stream(stream)))
    return grad6


def tgv_loss_and_grad(u, w, alpha0: float, alpha1: float, eps: float, scale: float = 1.0, want_loss: bool = True,
                      grad_u=None, grad_w=None, accumulate: bool = False, ctx: Context = None, stream=None):
    """scale * TGV(u, w) (second order, auxiliary field w [3, nx, ny, nz]) and its gradients;
    returns the value (float) or None."""
    import torch
    ctx = ctx or context(u.device.index)
    if u.dim() != 3:
        raise ValueError("u must be [nx, ny, nz]")
    nx, ny, nz = u.shape
    n = nx * ny * nz
    L = ctypes.c_double(0.0)
    ctx.check(ctx.lib.tgv_loss_and_grad(
        ctx.ptr, nx, ny, nz, _ptr(u, torch.float32, "u", n), _ptr(w, torch.float32, "w", 3 * n),
        float(alpha0), float(alpha1), float(eps), float(scale), ctypes.byref(L) if want_loss else None,
        _ptr(grad_u, torch.float32, "grad_u", n), _ptr(grad_w, torch.float32, "grad_w", 3 * n),
        RA_ACCUMULATE if accumulate else 0, _stream(stream)))
    return L.value if want_loss else None


def pose_from_euler(pose6, poses=None, ctx: Context = None, stream=None):
    """[F,6] (Euler angles, t) -> [F,12] (R row-major, t), R = Rz(a2) Ry(a1) Rx(a0)."""
    import torch
    ctx = ctx or context(pose6.device.index)
    F = pose6.shape[0]
    if poses is None:
        poses = torch.empty((F, 12), dtype=torch.float64, device=pose6.device)
    ctx.check(ctx.lib.ra_pose_from_euler(ctx.ptr, _ptr(pose6, torch.float64, "pose6", 6 * F), F,
                                         _ptr(poses, torch.float64, "poses", 12 * F), _stream(stream)))
    return poses


def pose_grad_euler(pose6, grad_pose, grad6=None, ctx: Context = None, stream=None):
    import torch
    ctx = ctx or context(pose6.device.index)
    F = pose6.shape[0]
    if grad6 is None:
        grad6 = torch.empty((F, 6), dtype=torch.float64, device=pose6.device)
    ctx.check(ctx.lib.ra_pose_grad_euler(ctx.ptr, _ptr(pose6, torch.float64, "pose6", 6 * F),
                                         _ptr(grad_pose, torch.float64, "grad_pose", 12 * F), F,
                                         _ptr(grad6, torch.float64, "grad6", 6 * F), _stream(stream)))
    return grad6


def count_updates(grid: Grid, elem, poses, samp: Sampling, ctx: Context = None, stream=None) -> int:
    import torch
    ctx = ctx or context(elem.device.index)
    M, F, _, _ = _sizes(grid, elem, poses, samp)
    n = ctypes.c_longlong(0)
    ctx.check(ctx.lib.ra_count_updates(ctx.ptr, ctypes.byref(grid.c()), M,
                                       _ptr(elem, torch.float64, "elem", 3 * M),
                                       _ptr(poses, torch.float64, "poses", 12 * F), F, ctypes.byref(samp.cs()),
                                       ctypes.byref(n), _stream(stream)))
    return int(n.value)
