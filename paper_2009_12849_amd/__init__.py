"""Python binding of libmonc.so, the MI355X anelastic pressure projection.

Argument marshalling only: every step of the projection runs in the HIP
kernels of the library. PyTorch supplies device memory and streams; tensors
must be contiguous CUDA (HIP) tensors of the plan's dtype (float64 for
"f64", float32 for "mixed") and shape (nz, ny, nx).

The library must have been built in-tree (``python -m
paper_2009_12849_amd.build``); nothing here falls back to another
implementation when it is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

__all__ = ["Plan", "project_batched", "stream_probe", "autotune_batched", "batch_schedule", "set_batch_schedule", "lib", "last_error", "MoncError",
           "FP64", "MIXED", "STAGE_FORWARD", "STAGE_SOLVE", "STAGE_INVERSE",
           "STAGE_GRADIENT", "STAGE_RESIDUAL", "KERNELS"]

FP64, MIXED = 0, 1
OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP = 0, -1, -2, -3, -4
STAGE_FORWARD, STAGE_SOLVE, STAGE_INVERSE, STAGE_GRADIENT, STAGE_RESIDUAL = 1, 2, 3, 4, 5
NPARAMS = 7  # tile parameters: x/y FFT elements per thread, y-FFT columns,
             # tridiagonal lanes per column, tridiagonal columns per workgroup,
             # x transforms per workgroup, y-FFT elements per thread
KERNELS = ["div_fftx", "ffty_fwd", "tridiag", "ffty_inv", "ifftx", "grad",
           "resid_fftx", "grad_final"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmonc.so")
_lib = None


class MoncError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"monc error {code}: {msg}")
        self.code = code


def lib() -> ctypes.CDLL:
    """Load libmonc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2009_12849_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    L.monc_plan_create.restype = vp
    L.monc_plan_create.argtypes = [ip, ip, ip, ctypes.c_double, ctypes.c_double, dp, dp, ip]
    L.monc_plan_destroy.restype = None
    L.monc_plan_destroy.argtypes = [vp]
    L.monc_project.restype = ip
    L.monc_project.argtypes = [vp, vp, vp, vp, vp, vp]
    L.monc_project_noalloc.restype = ip
    L.monc_project_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
    L.monc_project_reduce.restype = ip
    L.monc_project_reduce.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.monc_project_var.restype = ip
    L.monc_project_var.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_double, ip, ctypes.POINTER(ip),
                                   ctypes.POINTER(ctypes.c_double), vp]
    L.monc_project_batched.restype = ip
    L.monc_project_batched.argtypes = [ctypes.POINTER(vp), ip] + [ctypes.POINTER(vp)] * 4 + [vp]
    L.monc_last_error.restype = ctypes.c_char_p
    L.monc_last_error.argtypes = []
    L.monc_spectral_layout.restype = ctypes.c_size_t
    L.monc_spectral_layout.argtypes = [vp, ctypes.POINTER(ip), ctypes.POINTER(ip), ctypes.POINTER(ctypes.c_longlong),
                                       ctypes.POINTER(ip)]
    L.monc_debug_stage.restype = ip
    L.monc_debug_stage.argtypes = [vp, ip, ctypes.POINTER(vp), ip, vp]
    L.monc_kernel_name.restype = ctypes.c_char_p
    L.monc_kernel_name.argtypes = [ip]
    L.monc_profile_enable.restype = ip
    L.monc_profile_enable.argtypes = [vp, ctypes.c_uint]
    L.monc_profile_read.restype = ip
    L.monc_profile_read.argtypes = [vp, dp, ctypes.POINTER(ip)]
    L.monc_autotune.restype = ip
    L.monc_autotune.argtypes = [ctypes.POINTER(vp), ip, vp]
    L.monc_batch_schedule.restype = ip
    L.monc_batch_schedule.argtypes = [ctypes.POINTER(vp), ip, ctypes.POINTER(ip)]
    L.monc_batch_set_schedule.restype = ip
    L.monc_batch_set_schedule.argtypes = [ctypes.POINTER(vp), ip, ip, ip, ip]
    L.monc_plan_params.restype = ip
    L.monc_plan_params.argtypes = [vp, ctypes.POINTER(ip)]
    L.monc_plan_set_params.restype = ip
    L.monc_plan_set_params.argtypes = [vp, ctypes.POINTER(ip)]
    L.monc_stream_probe.restype = ip
    L.monc_stream_probe.argtypes = [ip, vp, vp, vp, vp, ctypes.c_size_t, vp]
    _lib = L
    return L


def last_error() -> str:
    return lib().monc_last_error().decode()


def _check(rc: int):
    if rc != OK:
        raise MoncError(rc, last_error())


def _dtype_code(dtype) -> int:
    if dtype in ("f64", "fp64", FP64):
        return FP64
    if dtype in ("mixed", MIXED):
        return MIXED
    raise ValueError(f"unknown dtype {dtype!r}")


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Plan:
    """Projection plan for one grid (see include/monc.h)."""

    def __init__(self, nx: int, ny: int, nz: int, dx: float, dy: float,
                 dz: Sequence[float], rho0: Sequence[float], dtype="f64"):
        L = lib()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dtype = _dtype_code(dtype)
        dzv = np.ascontiguousarray(dz, dtype=np.float64)
        rv = np.ascontiguousarray(rho0, dtype=np.float64)
        if dzv.shape != (self.nz,) or rv.shape != (self.nz,):
            raise ValueError("dz and rho0 must have nz entries")
        dptr = ctypes.POINTER(ctypes.c_double)
        h = L.monc_plan_create(self.nx, self.ny, self.nz, float(dx), float(dy),
                               dzv.ctypes.data_as(dptr), rv.ctypes.data_as(dptr), self.dtype)
        if not h:
            raise MoncError(EINVAL, last_error())
        self._h = ctypes.c_void_p(h)

    @classmethod
    def from_grid(cls, grid, dtype="f64") -> "Plan":
        return cls(grid.nx, grid.ny, grid.nz, grid.dx, grid.dy, grid.dz, grid.rho0, dtype)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.dtype == FP64 else torch.float32

    def close(self):
        if getattr(self, "_h", None):
            lib().monc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _field(self, t, name):
        if t.dtype != self.torch_dtype or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous CUDA tensor of {self.torch_dtype}")
        if tuple(t.shape) != (self.nz, self.ny, self.nx):
            raise ValueError(f"{name} must have shape (nz, ny, nx) = {(self.nz, self.ny, self.nx)}")
        return ctypes.c_void_p(t.data_ptr())

    def project(self, u, v, w, p, stream=None, stats=None):
        """In-place projection of u, v, w; p receives the pressure. With
        `stats` (a float64 device tensor of 8*nz values), also the per-level
        horizontal mean and max of u, v, w, p: stats.view(4, 2, nz)[f, s, k]
        (see monc_project_reduce)."""
        args = [self._field(t, n) for t, n in ((u, "u"), (v, "v"), (w, "w"), (p, "p"))]
        st = ctypes.c_void_p(_stream_handle(stream))
        if stats is None:
            _check(lib().monc_project(self._h, *args, st))
            return
        import torch
        if stats.dtype != torch.float64 or not stats.is_cuda or stats.numel() != 8 * self.nz \
                or not stats.is_contiguous():
            raise ValueError(f"stats must be a contiguous float64 device tensor of {8 * self.nz} values")
        _check(lib().monc_project_reduce(self._h, *args, ctypes.c_void_p(stats.data_ptr()), st))

    def project_noalloc(self, u, v, w, p, stream=None):
        """project() with its workspace in the library's static device array
        (see monc_project_noalloc): no device allocation."""
        args = [self._field(t, n) for t, n in ((u, "u"), (v, "v"), (w, "w"), (p, "p"))]
        _check(lib().monc_project_noalloc(self._h, *args, ctypes.c_void_p(_stream_handle(stream))))

    def project_var(self, rho, u, v, w, p, tol=1e-12, maxit=200, stream=None):
        """Projection with the density field rho(x, y, z) (see
        monc_project_var): preconditioned conjugate gradients with this
        plan's spectral solve as the preconditioner. rho, u, v, w, p are
        contiguous float64 device tensors of shape (nz, ny, nx) whatever the
        plan's precision; u, v, w are updated in place, p receives the
        pressure. Returns (iterations, final relative residual)."""
        import torch
        args = []
        for t, n in ((rho, "rho"), (u, "u"), (v, "v"), (w, "w"), (p, "p")):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{n} must be a contiguous float64 CUDA tensor")
            if tuple(t.shape) != (self.nz, self.ny, self.nx):
                raise ValueError(f"{n} must have shape (nz, ny, nx) = {(self.nz, self.ny, self.nx)}")
            args.append(ctypes.c_void_p(t.data_ptr()))
        it = ctypes.c_int(0)
        rel = ctypes.c_double(0.0)
        _check(lib().monc_project_var(self._h, *args, float(tol), int(maxit), ctypes.byref(it), ctypes.byref(rel),
                                      ctypes.c_void_p(_stream_handle(stream))))
        return it.value, rel.value

    # -- introspection / stages / profiling / tuning ---------------------
    def spectral_layout(self):
        """(elements, padded row length, column block width, plane length,
        bytes per complex value); see monc_spectral_layout."""
        row, blk, plane, eb = ctypes.c_int(), ctypes.c_int(), ctypes.c_longlong(), ctypes.c_int()
        n = lib().monc_spectral_layout(self._h, ctypes.byref(row), ctypes.byref(blk), ctypes.byref(plane),
                                       ctypes.byref(eb))
        return int(n), row.value, blk.value, plane.value, eb.value

    def spectral_buffer(self):
        """A zeroed device buffer with the spectral layout, shape (nz, plane)."""
        import torch
        n, row, blk, plane, eb = self.spectral_layout()
        dt = torch.complex128 if self.dtype == FP64 else torch.complex64
        return torch.zeros((self.nz, plane), dtype=dt, device="cuda")

    def _blocks(self, buf):
        # (nz, ny, row/blk, blk) strided view of the column blocks
        import torch
        n, row, blk, plane, eb = self.spectral_layout()
        return torch.as_strided(buf, (self.nz, self.ny, row // blk, blk),
                                (plane, blk, self.ny * blk, 1), buf.storage_offset())

    def spectral_get(self, buf):
        """Copy of the (nz, ny, nx/2+1) half spectrum held in a spectral buffer."""
        v = self._blocks(buf)
        return v.reshape(self.nz, self.ny, -1)[:, :, : self.nx // 2 + 1]

    def spectral_set(self, buf, values):
        """Write a (nz, ny, nx/2+1) half spectrum into a spectral buffer."""
        import torch
        v = self._blocks(buf)
        full = torch.zeros((self.nz, self.ny, v.shape[2] * v.shape[3]), dtype=buf.dtype, device=buf.device)
        full[:, :, : self.nx // 2 + 1] = torch.as_tensor(values).to(device=buf.device, dtype=buf.dtype)
        v.copy_(full.view(v.shape))

    def debug_stage(self, stage: int, bufs, stream=None):
        arr = (ctypes.c_void_p * len(bufs))(*[ctypes.c_void_p(b.data_ptr()) for b in bufs])
        _check(lib().monc_debug_stage(self._h, stage, arr, len(bufs), ctypes.c_void_p(_stream_handle(stream))))

    def profile_enable(self, mask: int):
        _check(lib().monc_profile_enable(self._h, mask))

    def profile_read(self):
        ms = (ctypes.c_double * len(KERNELS))()
        cnt = (ctypes.c_int * len(KERNELS))()
        _check(lib().monc_profile_read(self._h, ms, cnt))
        return {KERNELS[i]: (ms[i], cnt[i]) for i in range(len(KERNELS)) if cnt[i]}

    def autotune(self, stream=None):
        """Tune this plan's tile parameters (monc_autotune of one plan)."""
        arr = (ctypes.c_void_p * 1)(self._h)
        _check(lib().monc_autotune(arr, 1, ctypes.c_void_p(_stream_handle(stream))))

    @property
    def params(self):
        out = (ctypes.c_int * NPARAMS)()
        _check(lib().monc_plan_params(self._h, out))
        return list(out)

    @params.setter
    def params(self, vals):
        vals = list(vals) + [0] * (NPARAMS - len(vals))
        if len(vals) != NPARAMS:
            raise ValueError(f"expected at most {NPARAMS} tile parameters")
        arr = (ctypes.c_int * NPARAMS)(*[int(x) for x in vals])
        _check(lib().monc_plan_set_params(self._h, arr))


def autotune_batched(plans: Sequence[Plan], stream=None):
    """Tune the tile parameters of every distinct grid and the batch schedule
    (member order, grouping) of these plans (monc_autotune)."""
    arr = (ctypes.c_void_p * len(plans))(*[pl.handle for pl in plans])
    _check(lib().monc_autotune(arr, len(plans), ctypes.c_void_p(_stream_handle(stream))))


def batch_schedule(plans: Sequence[Plan]):
    """(order, budget_mb, groups, branches) of the batch schedule of these plans."""
    arr = (ctypes.c_void_p * len(plans))(*[pl.handle for pl in plans])
    out = (ctypes.c_int * 4)()
    _check(lib().monc_batch_schedule(arr, len(plans), out))
    return tuple(out)


def set_batch_schedule(plans: Sequence[Plan], order: int, budget_mb: int, branches: int = 1):
    """Set the batch schedule of these plans by hand (monc_batch_set_schedule)."""
    arr = (ctypes.c_void_p * len(plans))(*[pl.handle for pl in plans])
    _check(lib().monc_batch_set_schedule(arr, len(plans), int(order), int(budget_mb), int(branches)))


PROBES = {"read": 0, "write": 1, "copy": 2, "update": 3}


def stream_probe(kind: str, bufs, stream=None):
    """One launch of a streaming-bandwidth probe (see monc_stream_probe) over
    equally sized contiguous CUDA tensors: "read" (data, 16-byte sink),
    "write" (out), "copy" (src, dst), "update" (p, u, v, w)."""
    need = {"read": 2, "write": 1, "copy": 2, "update": 4}[kind]
    if len(bufs) != need:
        raise ValueError(f"probe {kind!r} takes {need} buffers")
    nbytes = bufs[0].numel() * bufs[0].element_size()
    for t in bufs:
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("probe buffers must be contiguous CUDA tensors")
    for t in bufs[1:]:
        if kind != "read" and t.numel() * t.element_size() != nbytes:
            raise ValueError("probe buffers must have equal sizes")
    ptrs = [ctypes.c_void_p(t.data_ptr()) for t in bufs] + [None] * (4 - len(bufs))
    _check(lib().monc_stream_probe(PROBES[kind], *ptrs, nbytes, ctypes.c_void_p(_stream_handle(stream))))


def project_batched(plans: Sequence[Plan], us, vs, ws, ps, stream=None):
    """Project every member in one graph launch (see include/monc.h)."""
    n = len(plans)
    VP = ctypes.c_void_p * n
    hs = VP(*[pl.handle for pl in plans])
    fields = []
    for name, ts in (("u", us), ("v", vs), ("w", ws), ("p", ps)):
        fields.append(VP(*[pl._field(t, f"{name}[{i}]") for i, (pl, t) in enumerate(zip(plans, ts))]))
    _check(lib().monc_project_batched(hs, n, *fields, ctypes.c_void_p(_stream_handle(stream))))
