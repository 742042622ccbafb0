"""The C ABI on the host (no GPU needed): the library loads, exports every
function include/monc.h declares, and rejects bad plan arguments before any
HIP call."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2009_12849_amd as monc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "monc.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(monc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("monc_plan_create", "monc_project", "monc_project_batched",
                     "monc_plan_destroy", "monc_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = monc.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def _create(nx=8, ny=8, nz=4, dx=10.0, dy=10.0, dz=None, rho0=None, dtype=0):
    L = monc.lib()
    dz = np.full(max(nz, 1), 5.0) if dz is None else np.asarray(dz, dtype=np.float64)
    rho0 = np.ones(max(nz, 1)) if rho0 is None else np.asarray(rho0, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    h = L.monc_plan_create(nx, ny, nz, dx, dy, dz.ctypes.data_as(dp), rho0.ctypes.data_as(dp), dtype)
    return h, monc.last_error()


@pytest.mark.parametrize("kw,needle", [
    (dict(nx=0), "grid size"),
    (dict(nz=-3), "grid size"),
    (dict(nx=10), "prime factor"),
    (dict(ny=14), "prime factor"),
    (dict(nx=9000), "limits"),
    (dict(nz=2000, dz=np.ones(2000), rho0=np.ones(2000)), "limits"),
    (dict(dx=0.0), "dx and dy"),
    (dict(dy=math.nan), "dx and dy"),
    (dict(dx=math.inf), "dx and dy"),
    (dict(dz=[5.0, 5.0, -1.0, 5.0]), "dz[2]"),
    (dict(dz=[5.0, math.nan, 5.0, 5.0]), "dz[1]"),
    (dict(rho0=[1.0, 1.0, 1.0, 0.0]), "rho0[3]"),
    (dict(rho0=[1.0, math.inf, 1.0, 1.0]), "rho0[1]"),
    (dict(dtype=7), "dtype"),
])
def test_plan_create_rejects_bad_arguments(kw, needle):
    h, err = _create(**kw)
    assert not h
    assert needle in err, err


def test_null_profile_arrays_rejected():
    L = monc.lib()
    dp = ctypes.POINTER(ctypes.c_double)
    h = L.monc_plan_create(8, 8, 4, 1.0, 1.0, None, None, 0)
    assert not h and "non-null" in monc.last_error()


def test_null_plan_calls_are_errors():
    L = monc.lib()
    assert L.monc_project(None, None, None, None, None, None) == monc.EINVAL
    assert L.monc_project_reduce(None, None, None, None, None, None, None) == monc.EINVAL
    assert L.monc_project_noalloc(None, None, None, None, None, None) == monc.EINVAL
    assert L.monc_project_var(None, None, None, None, None, None, 1e-10, 10, None, None, None) == monc.EINVAL
    assert "plan is null" in monc.last_error()
    assert L.monc_spectral_layout(None, None, None, None, None) == 0
    assert L.monc_profile_enable(None, 1) == monc.EINVAL
    L.monc_plan_destroy(None)  # ignored


def test_batch_argument_checks_run_before_the_device():
    L = monc.lib()
    VP = ctypes.c_void_p * 1
    z = VP(None)
    assert L.monc_project_batched(z, 0, z, z, z, z, None) == monc.EINVAL
    assert "count" in monc.last_error()
    assert L.monc_project_batched(z, 1, z, z, z, z, None) == monc.EINVAL
    assert "null" in monc.last_error()


def test_kernel_names():
    L = monc.lib()
    names = [L.monc_kernel_name(i).decode() for i in range(len(monc.KERNELS))]
    assert names == monc.KERNELS
    assert L.monc_kernel_name(99) == b""


def test_stream_probe_argument_checks_run_before_the_device():
    L = monc.lib()
    vp = ctypes.c_void_p
    fake = vp(1 << 20)  # aligned, never dereferenced: every call below fails its checks first
    assert L.monc_stream_probe(9, fake, fake, fake, fake, 1024, None) == monc.EINVAL    # unknown kind
    assert L.monc_stream_probe(2, fake, None, None, None, 1024, None) == monc.EINVAL    # copy needs b
    assert L.monc_stream_probe(1, fake, None, None, None, 1000, None) == monc.EINVAL    # not a multiple of 16
    assert L.monc_stream_probe(1, vp((1 << 20) + 8), None, None, None, 1024, None) == monc.EINVAL  # misaligned
    assert L.monc_stream_probe(0, fake, None, None, None, 1024, None) == monc.EINVAL    # read needs its sink


def test_batch_schedule_argument_checks_run_before_the_device():
    L = monc.lib()
    VP = ctypes.c_void_p * 1
    z = VP(None)
    out = (ctypes.c_int * 4)()
    assert L.monc_batch_schedule(z, 0, out) == monc.EINVAL
    assert L.monc_batch_set_schedule(z, 1, 0, 0, 1) == monc.EINVAL
    assert L.monc_autotune(z, 0, None) == monc.EINVAL
    assert "count" in monc.last_error()
