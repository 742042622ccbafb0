"""Benchmark of the MI355X pressure projection (one GPU).

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

A step is one whole projection (divergence, forward FFTs, FP64 tridiagonal
solves, inverse FFTs, gradient correction) of the workload's fields, already
resident in HBM; the projection re-projects its own output in place, which
costs exactly the same kernels and bytes as the first pass.

Workloads (seeded synthetic stand-ins for the paper's dry boundary-layer
case, see synth/):
  2048x2048x160  k^-5/3 spectra, one GPU's share of a large run; headline =
                 the mixed path, the plain FP64 path beside it (default)
  1024x1024x256  stretched anelastic grid; headline = mixed, FP64 beside it
  ensemble48     48-member ensemble of uneven grids, one batched call (HIP
                 graph); headline = mixed, FP64 beside it
  256x256x128    headline = plain FP64 path, mixed beside it
  4096x4096x64   the paper's 1.07e9-point global problem; headline = mixed
`value` is the warm rate (K projections back to back); `cold` times single
projections after a 1 GiB write has flushed the 256 MB Infinity Cache.
Single grids up to 3e8 points also time the variable-density projection
(conjugate gradients with the spectral solve as preconditioner, a seeded
density rho0(z)(1 + 0.2 f(x, y, z))) under "variable_density".
Prints one JSON line.

Counter profiles (rocprofv3 --pmc, one pass per counter set):
  python bench.py --pmc-run [--workload NAME]      short run to profile
  python bench.py --summarize-counters RD_CSV WR_CSV [DRAM_CSV] [--workload NAME]
                                                   per-kernel HBM bytes
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-points/s full projection (mixed vs FP64 GPU) at rel err ≤1e-6, %HBM roofline"
HBM_PEAK_GBS = 8000.0
KERNEL_DIR = os.path.join(ROOT, "paper_2009_12849_amd", "csrc")
WORKLOADS = ["2048x2048x160", "1024x1024x256", "ensemble48", "256x256x128", "4096x4096x64"]
KERNELS = ["div_fftx", "ffty_fwd", "tridiag", "ffty_inv", "ifftx", "grad", "resid_fftx", "grad_final"]


def spectral_words(nx):
    """Real words per grid point of one spectral field (nx/2+1 complex per row)."""
    return 2.0 * (nx // 2 + 1) / nx


def kernel_bytes_per_point(kernel, nx, mixed):
    """Algorithmic (compulsory) HBM bytes per grid point of one launch: the
    inputs it must read and the outputs it must write, each once."""
    f = spectral_words(nx)
    wb = 4.0 if mixed else 8.0
    table = {
        "div_fftx": (3 + f) * wb,               # read u, v, w; write spectrum
        "ffty_fwd": 2 * f * wb,                 # read + write spectrum
        "tridiag": 2 * f * wb,
        "ffty_inv": 2 * f * wb,
        # read spectrum, write p (mixed: p1, then the correction delta)
        "ifftx": (f + 1) * wb,
        "grad": 7 * wb,                         # read p, u, v, w; write u, v, w
        "resid_fftx": (4 + f) * wb,             # read u, v, w, p1; write spectrum
        "grad_final": 9 * wb,                   # read p1, delta, u, v, w; write u, v, w, p
    }
    return table[kernel]


def path_bytes_per_point(nx, mixed):
    """Minimum HBM traffic of the whole path as built (inputs once, one round
    trip of the spectrum per global-dependency boundary, outputs once): FP64
    10 + 4f words; mixed 16 + 8f words: first solve 3 + f, 2f, f + 1 (p1);
    residual 4 + f; correction 2f; final f + 1 (delta) + 2 (p1, delta) + 3
    + 3 + 1 (p)."""
    f = spectral_words(nx)
    return (16 + 8 * f) * 4.0 if mixed else (10 + 4 * f) * 8.0


def kernel_path_bytes_per_point(nx, mixed):
    """What the kernels of one projection move, each launch at its
    algorithmic bytes: FP64 11 + 8f words (div-FFT 3 + f, four spectral
    passes 2f each, inverse f + 1, gradient 7), mixed 18 + 16f words
    (div-FFT 3 + f, two solves' spectral passes, two inverses f + 1, the
    residual 4 + f, the final gradient 9)."""
    f = spectral_words(nx)
    return (18 + 16 * f) * 4.0 if mixed else (11 + 8 * f) * 8.0


def strip_comments(src):
    """C++ source without its comments, runs of whitespace collapsed to one
    space (string and character literals kept as written)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash():
    """Hash of every kernel source, comments and layout aside (a counter
    summary taken on other code is stale; one taken before a comment changed
    is not)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(KERNEL_DIR)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(KERNEL_DIR, name), encoding="utf-8") as fh:
                h.update(name.encode() + b"\0" + strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")


def read_traffic(workload, kernel, mixed):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    the workload, or None if it is missing or was taken on another version of
    the kernels."""
    path = traffic_file(workload)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernels_sha256_16") != kernel_source_hash():
        return None
    key = f"{'mixed' if mixed else 'fp64'}.{kernel}.bytes_per_launch"
    return float(vals[key]) if key in vals else None


TUNING_FILE = os.path.join(ROOT, "paper_2009_12849_amd", "tuning", "gfx950.json")


def use_tuning_cache():
    """Point MONC_TUNE_CACHE at a private copy of the committed tuning table
    (tile parameters the library's autotuner chose on an MI355X for the
    benchmark grids) unless the caller named a cache. Plans created
    afterwards start from the cached parameters of their grid; grids missing
    from it are autotuned by the Runner. Returns the cache's path."""
    if os.environ.get("MONC_TUNE_CACHE"):
        return os.environ["MONC_TUNE_CACHE"]
    import shutil
    import tempfile
    fd, path = tempfile.mkstemp(prefix="monc_tune_", suffix=".json")
    os.close(fd)
    if os.path.exists(TUNING_FILE):
        shutil.copyfile(TUNING_FILE, path)
    else:
        with open(path, "w") as fh:
            fh.write("{}\n")
    os.environ["MONC_TUNE_CACHE"] = path
    return path


def cached_params(nx, ny, nz, dtype):
    path = os.environ.get("MONC_TUNE_CACHE")
    if not path or not os.path.exists(path):
        return None
    with open(path) as fh:
        try:
            data = json.load(fh)
        except ValueError:
            return None
    val = data.get(f"gfx950:{nx},{ny},{nz}:{'fp64' if dtype == 'f64' else 'mixed'}")
    return val if isinstance(val, list) and len(val) in (6, 7) else None   # as the library reads them


def cached_batch(count, dtype):
    """Whether the tuning cache holds a batch schedule for `count` members of
    this dtype."""
    path = os.environ.get("MONC_TUNE_CACHE")
    if not path or not os.path.exists(path):
        return False
    with open(path) as fh:
        try:
            data = json.load(fh)
        except ValueError:
            return False
    tag = "fp64" if dtype == "f64" else "mixed"
    return any(k.startswith(f"gfx950:batch:{count}:") and k.endswith(tag) for k in data)


class Runner:
    """Owns the plans and device fields of one path (FP64 or mixed) of a
    workload and runs whole projections on them."""

    def __init__(self, monc, torch, members, dtype, tune=True, retune=False):
        self.torch = torch
        self.monc = monc
        self.mixed = dtype == "mixed"
        cast = np.float32 if self.mixed else np.float64
        self.plans = [monc.Plan.from_grid(m.grid, dtype) for m in members]
        self.tuned = {}
        self.tuning = {}
        self.schedule = None
        # tile parameters: the tuning cache's (read by the library at plan
        # creation), else the library's autotuner once per distinct grid
        # (untimed); plans of the same grid share them. A batch is tuned as a
        # whole (tile parameters of its grids, then its member order and
        # grouping) unless the cache holds it.
        missing = any(cached_params(pl.nx, pl.ny, pl.nz, dtype) is None for pl in self.plans)
        if len(self.plans) > 1:
            if tune and (retune or missing or not cached_batch(len(self.plans), dtype)):
                monc.autotune_batched(self.plans)
                for pl in self.plans:
                    self.tuning[(pl.nx, pl.ny, pl.nz)] = "autotuned"
            for pl in self.plans:
                self.tuned.setdefault((pl.nx, pl.ny, pl.nz), pl.params)
                self.tuning.setdefault((pl.nx, pl.ny, pl.nz), "cache")
            self.schedule = dict(zip(("order", "budget_mb", "groups", "branches"), monc.batch_schedule(self.plans)))
        else:
            for pl in self.plans:
                key = (pl.nx, pl.ny, pl.nz)
                if tune and (retune or cached_params(pl.nx, pl.ny, pl.nz, dtype) is None):
                    pl.autotune()
                    self.tuning[key] = "autotuned"
                else:
                    self.tuning[key] = "cache" if cached_params(pl.nx, pl.ny, pl.nz, dtype) else "default"
                self.tuned[key] = pl.params
        self.fields = []
        for m in members:
            f = [torch.from_numpy(a.astype(cast, copy=False)).to("cuda:0") for a in (m.u, m.v, m.w)]
            f.append(torch.empty_like(f[0]))
            self.fields.append(f)
        self.batched = len(members) > 1
        self.points = sum(m.grid.points for m in members)
        self.stats = None   # per-level reductions buffer (single grids), when timed with them

    def step(self, stream=None):
        if self.batched:
            f = self.fields
            self.monc.project_batched(self.plans, [x[0] for x in f], [x[1] for x in f], [x[2] for x in f],
                                      [x[3] for x in f], stream)
        else:
            self.plans[0].project(*self.fields[0], stream, stats=self.stats)

    def breakdown(self, steps):
        """Average ms per launch of every kernel (HIP events per launch)."""
        torch = self.torch
        self.plans[0].profile_read()
        self.plans[0].profile_enable((1 << len(KERNELS)) - 1)
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        prof = self.plans[0].profile_read()
        self.plans[0].profile_enable(0)
        return {k: (ms / n, n // steps) for k, (ms, n) in prof.items()}

    def timed(self, steps, warmup, profile_kernel=None):
        """Wall-clock time of `steps` projections back to back (synchronised
        before and after); with profile_kernel, HIP events on the launch
        stream bracket every launch of that kernel."""
        torch = self.torch
        stream = torch.cuda.current_stream()
        for _ in range(warmup):
            self.step(stream)
        torch.cuda.synchronize()
        if profile_kernel is not None:
            self.plans[0].profile_read()
            self.plans[0].profile_enable(1 << KERNELS.index(profile_kernel))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = None
        if profile_kernel is not None:
            prof = self.plans[0].profile_read()
            self.plans[0].profile_enable(0)
        return wall, prof

    def cold(self, steps, flush):
        """Median time (ms, HIP events) of single projections, each after a
        write of the `flush` buffer (outside the events) has replaced the
        Infinity Cache's contents."""
        torch = self.torch
        stream = torch.cuda.current_stream()
        pairs = []
        for _ in range(steps):
            self.monc.stream_probe("write", [flush], stream)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            self.step(stream)
            b.record(stream)
            pairs.append((a, b))
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in pairs]))


def measure(runner, steps, warmup, workload, cold_steps, flush):
    """Throughput (warm and cold), kernel breakdown and dominant-kernel
    roofline of a path."""
    bd = runner.breakdown(3)
    dom = max(bd, key=lambda k: bd[k][0] * bd[k][1])
    wall, _ = runner.timed(steps, warmup)                    # clean timing
    _, prof = runner.timed(steps, 0, profile_kernel=dom)     # events around the dominant kernel
    cold_ms = runner.cold(cold_steps, flush) if cold_steps > 0 else None
    value = runner.points * steps / wall
    dom_ms, dom_n = prof[dom]
    dom_avg_s = dom_ms / dom_n / 1e3
    # bytes per launch: the kernel's bytes per step (it runs once per step, the
    # spectral phases twice on the mixed path) over its launches per step
    # (one, or one per group of batch members that share a kernel instance)
    occ = 2 if (runner.mixed and dom in ("ffty_fwd", "tridiag", "ffty_inv", "ifftx")) else 1
    per_step = occ * sum(kernel_bytes_per_point(dom, p.nx, runner.mixed) * p.nx * p.ny * p.nz
                         for p in runner.plans)
    per_launch = per_step / max(1, dom_n // steps)
    achieved = per_launch / dom_avg_s / 1e9
    path_bytes = sum(path_bytes_per_point(p.nx, runner.mixed) * p.nx * p.ny * p.nz for p in runner.plans)
    kernel_bytes = sum(kernel_path_bytes_per_point(p.nx, runner.mixed) * p.nx * p.ny * p.nz for p in runner.plans)
    traffic = read_traffic(workload, dom, runner.mixed)
    out = {
        "value": value,
        "ms_per_step": 1e3 * wall / steps,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_over_algorithmic": (traffic / per_launch) if traffic else None,
                     "avg_launch_ms": dom_avg_s * 1e3, "algorithmic_bytes_per_launch": per_launch},
        "path": {"algorithmic_bytes_per_point": path_bytes / runner.points,
                 "kernel_bytes_per_point": kernel_bytes / runner.points,
                 "end_to_end_hbm_frac": path_bytes * steps / wall / 1e9 / HBM_PEAK_GBS,
                 "kernels_ms": {k: round(v[0], 5) for k, v in bd.items()},
                 "launches_per_step": {k: v[1] for k, v in bd.items()}},
    }
    if cold_ms is not None:
        out["cold"] = {"ms_per_step": cold_ms, "value": runner.points / (cold_ms * 1e-3),
                       "end_to_end_hbm_frac": path_bytes / (cold_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "steps": cold_steps,
                       "what": "median of single projections, each after a 1 GiB write (outside the timed "
                               "events) has flushed the 256 MB Infinity Cache"}
    return out


def streaming_ceilings(monc, torch, mib=1024, reps=5):
    """Bandwidth of the library's streaming probes (read only, write only,
    copy, and the 4-read 3-write pointwise update of the gradient's access
    mix) over `mib` MiB buffers: what a plain streaming kernel reaches on
    this device, next to the vendor peak."""
    n = mib * (1 << 20) // 4
    bufs = [torch.zeros(n, dtype=torch.float32, device="cuda:0") for _ in range(4)]
    sink = torch.zeros(4, dtype=torch.float32, device="cuda:0")
    nbytes = n * 4
    cases = {"read": ([bufs[0], sink], 1), "write": ([bufs[0]], 1), "copy": (bufs[:2], 2),
             "update_4r3w": (bufs, 7)}
    out = {}
    stream = torch.cuda.current_stream()
    for name, (b, mult) in cases.items():
        kind = name.split("_")[0]
        for _ in range(2):
            monc.stream_probe(kind, b, stream)
        evs = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            monc.stream_probe(kind, b, stream)
            e1.record(stream)
            evs.append((e0, e1))
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(c) for a, c in evs]))
        out[name] = mult * nbytes / (ms * 1e-3) / 1e9
    del bufs, sink
    torch.cuda.empty_cache()
    return out


def _max_abs_diff(a, b, chunk=8):
    """max |a - b| in FP64, a level chunk at a time (bounded host memory)."""
    m = 0.0
    for k0 in range(0, a.shape[0], chunk):
        d = np.abs(a[k0:k0 + chunk].astype(np.float64) - b[k0:k0 + chunk].astype(np.float64))
        m = max(m, float(d.max()) if d.size else 0.0)
    return m


def max_errors(out, ref, members_in):
    """Normwise errors of u, v, w (relative to the input velocity scale) and p."""
    u, v, w = members_in
    vs = max(float(np.abs(u).max()), float(np.abs(v).max()), float(np.abs(w).max()))
    errs = [_max_abs_diff(out[t], ref[t]) / vs for t in range(3)]
    errs.append(_max_abs_diff(out[3], ref[3]) / float(np.abs(ref[3]).max()))
    return errs
def var_iteration_bytes_per_point(nx, mixed):
    """Algorithmic HBM bytes per grid point of one conjugate-gradient
    iteration of the variable-density projection: the operator (read d and
    rho, write q), the update (read p, d, r, q; write p, r), the spectral
    preconditioner (read r, the spectrum's four round trips, write z in the
    plan's storage type), the inner products (read r and z; with the FP32
    preconditioner's flexible update also q) and the direction update (read
    z, d; write d). FP64 128 + 64f, mixed 124 + 32f."""
    f = spectral_words(nx)
    wb = 4.0 if mixed else 8.0
    dots = (8 + wb + 8) if mixed else (8 + wb)
    return 24 + 48 + (8 + 8 * f * wb + wb) + dots + (16 + wb)


def variable_density(monc, torch, member, reps=3, tol=1e-10, amp=0.2, strong=0.5):
    """The variable-density projection (conjugate gradients, the spectral
    solve as preconditioner) on the workload's grid and fields with a
    density rho0(z) (1 + amp f(x, y, z)), |f| <= 1: per preconditioner
    precision the median wall time of `reps` solves from the same inputs
    (inputs copied in before each, outside the timing), iterations,
    relative residual and the per-iteration HBM fraction; then the same
    with a stronger contrast (amp = `strong`) under "stronger_contrast"."""
    out = _variable_density_case(monc, torch, member, reps, tol, amp)
    out["stronger_contrast"] = _variable_density_case(monc, torch, member, reps, tol, strong)
    return out


def _variable_density_case(monc, torch, member, reps, tol, amp):
    import synth
    g = member.grid
    rho_np = synth.density_field(np.random.default_rng(6100), g, amp)
    dev = "cuda:0"
    rho = torch.from_numpy(rho_np).to(dev)
    del rho_np
    src = [torch.from_numpy(a.astype(np.float64, copy=False)).to(dev) for a in (member.u, member.v, member.w)]
    work = [torch.empty_like(src[0]) for _ in range(4)]
    out = {"what": f"D_rho(G p) = D_rho(u*) with rho = rho0(z)(1 + {amp} f(x,y,z)), FP64 conjugate gradients, "
                   f"the spectral solve as preconditioner, stop at relative residual {tol}",
           "tol": tol, "amp": amp}
    for dtype in ("f64", "mixed"):
        plan = monc.Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, rho.mean(dim=(1, 2)).cpu().numpy(), dtype)
        plan.autotune()
        times, it, rel = [], 0, 0.0
        for r in range(reps + 1):
            for a, b in zip(work[:3], src):
                a.copy_(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it, rel = plan.project_var(rho, *work, tol=tol, maxit=500)
            torch.cuda.synchronize()
            if r > 0:
                times.append(time.perf_counter() - t0)
        plan.close()
        ms = 1e3 * float(np.median(times))
        ms_it = ms / max(it, 1)
        gbs = var_iteration_bytes_per_point(g.nx, dtype == "mixed") * g.points / (ms_it * 1e-3) / 1e9
        out["fp64_preconditioner" if dtype == "f64" else "fp32_preconditioner"] = {
            "ms_per_solve": ms, "iterations": it, "relres": rel, "ms_per_iteration": ms_it,
            "grid_points_per_s": g.points / (ms * 1e-3),
            "iteration_hbm_frac": gbs / HBM_PEAK_GBS}
    del rho, src, work
    torch.cuda.empty_cache()
    return out


def cpu_baseline(members, min_s=10.0, budget_s=25.0):
    """The FP64 oracle timed on this host: whole projections of the workload's
    members in order, pass after pass, until at least min_s seconds are timed
    (a pass stops early once budget_s is exceeded). Returns the timing record
    and the oracle's output for each member reached in the first pass."""
    import oracle
    workers = len(os.sched_getaffinity(0))
    times, outs, pts, passes = [], [], 0, 0
    while True:
        for m in members:
            g = m.grid
            t0 = time.perf_counter()
            out = oracle.project(m.u, m.v, m.w, g.dx, g.dy, g.dz, g.rho0, workers=workers)
            times.append(time.perf_counter() - t0)
            if passes == 0:
                outs.append(out)
            pts += g.points
            if sum(times) > budget_s:
                break
        passes += 1
        if sum(times) >= min_s or sum(times) > budget_s:
            break
    tot = sum(times)
    g0 = members[0].grid
    if len(members) == 1:
        what = f"{len(times)} whole FP64 projection(s) of the {g0.nx}x{g0.ny}x{g0.nz} grid"
    else:
        what = f"{len(times)} whole member projections ({pts} points) over {passes} pass(es) of the ensemble"
    rec = {"value": pts / tot, "unit": "grid-points/s", "cores": workers, "kind": "oracle",
           "sample": f"{what}, {tot:.2f} s (scipy.fft workers={workers}, NumPy elsewhere), "
                     f"host {platform.processor() or platform.machine()}"}
    return rec, outs


def variable_cpu_baseline(min_s=3.0, amp=0.2):
    """The variable-density oracle (a direct sparse solve) timed on this host.
    It cannot solve the benchmark grid (8e6 unknowns and up), so the sample is
    a 32 x 32 x 16 grid with the same density recipe, solved repeatedly until
    min_s seconds are timed: the oracle's rate on a problem it can do, not a
    rate at the benchmark's size."""
    import oracle
    import synth
    rng = np.random.default_rng(6101)
    g = synth.random_grid(rng, 32, 32, 16, stretch=(1.0, 1.1))
    rho = synth.density_field(np.random.default_rng(6100), g, amp)
    u, v, w = synth.random_fields(rng, g)
    times = []
    while sum(times) < min_s:
        t0 = time.perf_counter()
        oracle.project_var(u, v, w, g.dx, g.dy, g.dz, rho)
        times.append(time.perf_counter() - t0)
    tot = sum(times)
    return {"value": len(times) * g.points / tot, "unit": "grid-points/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(times)} direct sparse solves (SciPy SuperLU) of a {g.nx}x{g.ny}x{g.nz} grid with "
                      f"rho0(z)(1 + {amp} f), {tot:.2f} s, host {platform.processor() or platform.machine()}"}




# ---------------------------------------------------------------------------
# hardware counters: a short run to profile, and its per-kernel summary
# ---------------------------------------------------------------------------
CALIB_MIB = 1024   # probe buffers of the counter calibration


def pmc_run(monc, torch, members, head, other):
    """What the counter passes profile: the probes over CALIB_MIB MiB (copy
    twice, then read and write once each: known bytes that calibrate the
    counters), then two projections of each path with the tuning cache's
    tile parameters (no autotuning, so every launch of a kernel has the
    shape the benchmark times)."""
    n = CALIB_MIB * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.zeros_like(a)
    sink = torch.zeros(4, dtype=torch.float32, device="cuda:0")
    for _ in range(2):
        monc.stream_probe("copy", [a, b])
    monc.stream_probe("read", [a, sink])
    monc.stream_probe("write", [b])
    torch.cuda.synchronize()
    del a, b, sink
    torch.cuda.empty_cache()
    for dtype in (head, other):
        r = Runner(monc, torch, members, dtype, tune=False)
        for _ in range(2):
            r.step()
        torch.cuda.synchronize()
        print(f"pmc-run: {dtype} path, 2 projections, tile params {r.tuned}", flush=True)
        del r
        torch.cuda.empty_cache()


_MODES_X = {"0": "div_fftx", "1": "resid_fftx", "2": "precond_fftx"}


def classify_kernel(name):
    """(path, kernel) of a library kernel from its demangled name, e.g.
    'void monc::k_xfwd_ct<float, 1, 2048>(monc::LaunchArgs)' -> ('mixed',
    'resid_fftx'); probes give ('probe', kind); None for anything else."""
    import re
    if "k_probe_" in name:
        return ("probe", name.split("k_probe_", 1)[1].split("(", 1)[0].split("<", 1)[0])
    m = re.search(r"k_(xfwd|ffty|xinv|tridiag|grad)(?:_ct|_gen|_pp)?<([^>]*)>", name)
    if not m:
        return None
    kind, args = m.group(1), [x.strip() for x in m.group(2).split(",")]
    if kind == "ffty" and args[0] in ("true", "false"):  # the persistent FP32 y kernel <INV, N>
        return ("mixed", "ffty_inv" if args[0] == "true" else "ffty_fwd")
    path = "fp64" if args[0] == "double" else "mixed"
    if kind == "xfwd":
        return (path, _MODES_X.get(args[1], "xfwd"))
    if kind == "ffty":
        return (path, "ffty_inv" if args[1] == "true" else "ffty_fwd")
    if kind == "xinv":
        return (path, "ifftx_corr" if args[1] == "1" else "ifftx")
    if kind == "tridiag":
        return (path, "tridiag")
    return (path, "grad" if path == "fp64" else "grad_final")


def _read_counter_csv(path):
    """{dispatch id: (kernel name, {counter: value})} of a rocprofv3
    counter-collection CSV (one row per counter and dispatch)."""
    import csv
    out = {}
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            did = row.get("Dispatch_Id") or row.get("Correlation_Id")
            name = row.get("Kernel_Name", "")
            ent = out.setdefault(int(did), (name, {}))
            ent[1][row["Counter_Name"]] = ent[1].get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
    return out


def read_bytes(c):
    """Bytes the L2 read from the memory side: 32, 64 and 128-byte requests."""
    return 32.0 * c.get("TCC_EA0_RDREQ_32B_sum", 0.0) + 64.0 * c.get("TCC_EA0_RDREQ_64B_sum", 0.0) \
        + 128.0 * c.get("TCC_EA0_RDREQ_128B_sum", 0.0)


def write_bytes(c):
    """Bytes the L2 wrote to the memory side: 64-byte and 32-byte requests."""
    n64 = c.get("TCC_EA0_WRREQ_64B_sum", 0.0)
    return 64.0 * n64 + 32.0 * (c.get("TCC_EA0_WRREQ_sum", 0.0) - n64)


def kernel_launch_bytes(kernel, nx, points, mixed):
    """Algorithmic bytes of one launch of a kernel as the counters see it
    (ifftx and its correction pass separately)."""
    f = spectral_words(nx)
    wb = 4.0 if mixed else 8.0
    per = {"ifftx": (f + 1) * wb, "ifftx_corr": (f + 1) * wb}.get(kernel)
    if per is None:
        per = kernel_bytes_per_point(kernel, nx, mixed)
    return per * points


def summarize_counters(rd_csv, wr_csv, workload, command, dram_csv=None):
    """Per-kernel HBM traffic from two counter passes over `pmc_run`: read
    bytes from the L2's 32/64/128-byte read requests, write bytes from its
    64/32-byte write requests, each scaled by the factor that makes the
    calibration copy (CALIB_MIB MiB read, CALIB_MIB MiB written) exact. The
    median over a kernel's launches; all launches of a kernel have one shape
    (no autotuning in the profiled run). With a third pass (dram_csv:
    TCC_EA0_RDREQ_DRAM, TCC_EA0_WRREQ_DRAM, the requests addressed to local
    memory), a cross-check: those request counts in bytes, each scaled by the
    bytes per request of the calibration copy."""
    import synth
    rd, wr = _read_counter_csv(rd_csv), _read_counter_csv(wr_csv)
    dr = _read_counter_csv(dram_csv) if dram_csv else None
    known = CALIB_MIB * float(1 << 20)

    def collect(table, fn):
        per = {}
        for did in sorted(table):
            name, c = table[did]
            cls = classify_kernel(name)
            if cls is not None:
                per.setdefault(cls, []).append(fn(c))
        return per

    r_all, w_all = collect(rd, read_bytes), collect(wr, write_bytes)
    copy_r = r_all.get(("probe", "copy"), [])
    copy_w = w_all.get(("probe", "copy"), [])
    if not copy_r or not copy_w:
        raise SystemExit("no calibration copy dispatch in the counter data")
    fr = known / float(np.median(copy_r))
    fw = known / float(np.median(copy_w))
    g = synth.make_grid(workload)
    lines = [f"# HBM traffic per kernel launch, {workload} ({g.nx}x{g.ny}x{g.nz} = {g.points} points)",
             f"# command: {command}",
             "# read bytes  = 32 TCC_EA0_RDREQ_32B + 64 TCC_EA0_RDREQ_64B + 128 TCC_EA0_RDREQ_128B (sums over",
             "#               the L2 channels), write bytes = 64 TCC_EA0_WRREQ_64B + 32 (TCC_EA0_WRREQ -",
             "#               TCC_EA0_WRREQ_64B); L2-to-memory-side traffic, Infinity Cache hits included",
             f"# calibration: the probe copy of {CALIB_MIB} MiB reads and writes {int(known)} bytes; raw counters",
             f"#   read {np.median(copy_r):.0f} and write {np.median(copy_w):.0f} bytes, so factors "
             f"read {fr:.4f}, write {fw:.4f}",
             f"kernels_sha256_16: {kernel_source_hash()}",
             f"calibration.read_factor: {fr:.6f}",
             f"calibration.write_factor: {fw:.6f}"]
    for probe in ("read", "write"):
        rr = r_all.get(("probe", probe))
        ww = w_all.get(("probe", probe))
        if rr and ww:
            lines.append(f"probe.{probe}.read_bytes: {np.median(rr) * fr:.0f}   # expected "
                         f"{known if probe == 'read' else 0:.0f}")
            lines.append(f"probe.{probe}.write_bytes: {np.median(ww) * fw:.0f}   # expected "
                         f"{known if probe == 'write' else 0:.0f}")
    for key in sorted(k for k in r_all if k[0] != "probe"):
        path, kern = key
        rr = float(np.median(r_all[key])) * fr
        ww = float(np.median(w_all.get(key, [0.0]))) * fw
        alg = kernel_launch_bytes(kern, g.nx, g.points, path == "mixed")
        lines.append(f"{path}.{kern}.read_bytes_per_launch: {rr:.0f}")
        lines.append(f"{path}.{kern}.write_bytes_per_launch: {ww:.0f}")
        lines.append(f"{path}.{kern}.bytes_per_launch: {rr + ww:.0f}   # algorithmic {alg:.0f}, "
                     f"ratio {(rr + ww) / alg:.3f}, launches {len(r_all[key])}")
    if dr is not None:
        def cnt(name):
            return lambda c: float(c.get(name, 0.0))
        dr_r = collect(dr, cnt("TCC_EA0_RDREQ_DRAM_sum"))
        dr_w = collect(dr, cnt("TCC_EA0_WRREQ_DRAM_sum"))
        cr, cw = dr_r.get(("probe", "copy"), []), dr_w.get(("probe", "copy"), [])
        if cr and cw and np.median(cr) > 0 and np.median(cw) > 0:
            br, bw = known / float(np.median(cr)), known / float(np.median(cw))
            lines.append("# cross-check: TCC_EA0_RDREQ_DRAM / TCC_EA0_WRREQ_DRAM (requests addressed to local "
                         "memory) in bytes,")
            lines.append(f"#   at the calibration copy's {br:.1f} read and {bw:.1f} written bytes per request")
            for key in sorted(k for k in dr_r if k[0] != "probe"):
                path, kern = key
                rr = float(np.median(dr_r[key])) * br
                ww = float(np.median(dr_w.get(key, [0.0]))) * bw
                alg = kernel_launch_bytes(kern, g.nx, g.points, path == "mixed")
                lines.append(f"dram.{path}.{kern}.bytes_per_launch: {rr + ww:.0f}   # read {rr:.0f}, "
                             f"write {ww:.0f}, ratio to algorithmic {(rr + ww) / alg:.3f}")
    return "\n".join(lines) + "\n"


def summarize_trace(stats_csv, workload, command, bench_log=None):
    """Per-kernel summary of a rocprofv3 --kernel-trace --stats run of
    bench.py (its kernel_stats CSV): calls, average and total time per
    kernel instance, the library's kernel name beside it; with the bench's
    JSON line (bench_log), the event-timed average of its dominant kernels
    for comparison."""
    import csv
    rows = list(csv.DictReader(open(stats_csv, newline="")))
    lines = [f"# rocprofv3 kernel statistics, {workload}",
             f"# command: {command}",
             "# kernel instance | library kernel (path) | calls | average us | total ms | share of GPU time",
             f"kernels_sha256_16: {kernel_source_hash()}"]
    for r in rows:
        cls = classify_kernel(r["Name"])
        tag = f"{cls[1]} ({cls[0]})" if cls else "-"
        lines.append(f"{r['Name']} | {tag} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} %")
    if bench_log:
        with open(bench_log) as fh:
            txt = fh.read()
        start = txt.find('{"metric"')
        if start >= 0:
            d = json.loads(txt[start:txt.index("\n", start)] if "\n" in txt[start:] else txt[start:])
            for path in (d, d.get("fp64") or {}, d.get("mixed") or {}):
                rf = path.get("roofline") if isinstance(path, dict) else None
                if rf:
                    lines.append(f"# bench events, same run: {rf['kernel']} average {rf['avg_launch_ms'] * 1e3:.1f} us "
                                 f"per launch ({rf['achieved']:.0f} GB/s algorithmic)")
    return "\n".join(lines) + "\n"


# ---------------------------------------------------------------------------
DESCRIPTIONS = {
    "256x256x128": "plain FP64 projection 256x256x128, dx=dy=25 m, dz=min(10*1.015^k,60) m, rho0=1.2exp(-z/8 km), "
                   "periodic x,y, rigid lids",
    "1024x1024x256": "mixed FP32/FP64 projection with one FP64 refinement step, 1024x1024x256, "
                     "dz=min(10*1.015^k,60) m, rho0=1.2exp(-z/8 km)",
    "ensemble48": "batched ensemble of 48 uneven grids (64^2x64..256^2x128), one graph launch, mixed",
    "2048x2048x160": "mixed FP32/FP64 projection with one FP64 refinement step, 2048x2048x160, dx=dy=25 m, "
                     "dz=5*20^(k/159) m, rho0=1.2exp(-z/8 km), k^-5/3 horizontal spectra",
    "4096x4096x64": "mixed projection 4096x4096x64 (the paper's 1.07e9-point global problem on one GPU), "
                    "dz=min(10*1.015^k,60) m, rho0=1.2exp(-z/8 km)",
}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cold-steps", type=int, default=5, help="single projections timed after a cache flush")
    ap.add_argument("--workload", default="2048x2048x160", choices=WORKLOADS)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs (CPU baseline and accuracy)")
    ap.add_argument("--no-other", action="store_true", help="time only the headline path")
    ap.add_argument("--retune", action="store_true", help="autotune every grid, ignoring the tuning cache")
    ap.add_argument("--no-var", action="store_true", help="skip the variable-density solve")
    ap.add_argument("--pmc-run", action="store_true", help="the short run that the counter passes profile")
    ap.add_argument("--summarize-counters", nargs="+", metavar="CSV",
                    help="print the per-kernel traffic summary of two counter passes over --pmc-run")
    ap.add_argument("--summarize-trace", nargs="+", metavar=("STATS_CSV", "BENCH_LOG"),
                    help="print the per-kernel summary of a rocprofv3 --kernel-trace --stats run")
    ap.add_argument("--command", default="", help="command line recorded in the counter summary")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the projection is built and measured on a single "
              "MI355X (sharding across GPUs is described, not built). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.summarize_counters:
        sc = args.summarize_counters
        if len(sc) not in (2, 3):
            ap.error("--summarize-counters takes RD_CSV WR_CSV [DRAM_CSV]")
        sys.stdout.write(summarize_counters(sc[0], sc[1], args.workload, args.command,
                                            sc[2] if len(sc) == 3 else None))
        return
    if args.summarize_trace:
        sys.stdout.write(summarize_trace(args.summarize_trace[0], args.workload, args.command,
                                         args.summarize_trace[1] if len(args.summarize_trace) > 1 else None))
        return

    import torch
    import synth
    import paper_2009_12849_amd as monc

    use_tuning_cache()
    wl = synth.make_workload(args.workload)
    members = wl.members
    head = "f64" if args.workload == "256x256x128" else "mixed"
    other = "mixed" if head == "f64" else "f64"
    if args.pmc_run:
        pmc_run(monc, torch, members, head, other)
        return

    ceilings = streaming_ceilings(monc, torch)
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0")   # 1 GiB
    nchk = 1 if len(members) == 1 else 3      # members whose outputs the oracle checks

    def run_path(dtype):
        r = Runner(monc, torch, members, dtype, retune=args.retune)
        r.step()
        torch.cuda.synchronize()
        first = None
        if not args.no_cpu:
            first = [[t.cpu().numpy() for t in f] for f in r.fields[:nchk]]
        res = measure(r, args.steps, args.warmup, args.workload, args.cold_steps, flush)
        res["tile_params"] = {f"{k[0]}x{k[1]}x{k[2]}": v for k, v in r.tuned.items()}
        res["tuning"] = {f"{k[0]}x{k[1]}x{k[2]}": v for k, v in r.tuning.items()}
        if r.schedule is not None:
            res["batch_schedule"] = r.schedule
        extra = {}
        if not r.batched:
            # the same projections with the per-level horizontal reductions fused in
            r.stats = torch.empty(8 * r.plans[0].nz, dtype=torch.float64, device="cuda:0")
            wall_r, _ = r.timed(args.steps, args.warmup)
            r.stats = None
            ms_r = 1e3 * wall_r / args.steps
            extra["with_reductions"] = {"ms_per_step": ms_r, "overhead_frac": ms_r / res["ms_per_step"] - 1.0,
                                        "what": "per-level horizontal mean and max of u, v, w, p "
                                                "(monc_project_reduce)"}
        del r
        torch.cuda.empty_cache()
        return res, first, extra

    res, first, extra = run_path(head)
    g = members[0].grid
    result = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "grid-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "f64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": DESCRIPTIONS[args.workload], "grid_points": sum(m.grid.points for m in members),
                   "members": len(members), "path": "fp64" if head == "f64" else "mixed",
                   "tile_params": res.pop("tile_params"), "tuning": res.pop("tuning"),
                   "batch_schedule": res.pop("batch_schedule", None)},
        "roofline": res.pop("roofline"),
        "cold": res.pop("cold", None),
        "path": res.pop("path"),
        "streaming_ceiling_GBps": ceilings,
    }
    result.update(extra)
    if not args.no_var and len(members) == 1 and g.points <= 300_000_000:
        result["variable_density"] = variable_density(monc, torch, members[0])
        if not args.no_cpu:
            result["variable_density"]["cpu_baseline"] = variable_cpu_baseline()
    ofirst = None
    if not args.no_other:
        ores, ofirst, oextra = run_path(other)
        key = "mixed" if other == "mixed" else "fp64"
        result[key] = dict(ores, **oextra)
        head_cold = result["cold"]
        mixed_v, fp64_v = (result, ores) if head == "mixed" else (ores, result)
        result["mixed_speedup_vs_fp64"] = mixed_v["value"] / fp64_v["value"]
        if head_cold and ores.get("cold"):
            mc, fc = (head_cold, ores["cold"]) if head == "mixed" else (ores["cold"], head_cold)
            result["mixed_speedup_vs_fp64_cold"] = fc["ms_per_step"] / mc["ms_per_step"]
    del flush
    torch.cuda.empty_cache()

    if not args.no_cpu:
        import oracle
        base, refs = cpu_baseline(members)
        result["cpu_baseline"] = base
        acc = {}
        n = min(len(refs), nchk)
        for path, outs in ((head, first), (other, ofirst)):
            if outs is None:
                continue
            errs, divs = [], []
            for i in range(n):
                m = members[i]
                ins = (m.u, m.v, m.w)
                ref = refs[i]
                if path == "mixed":   # the oracle on the FP32-rounded inputs
                    ins = tuple(a.astype(np.float32).astype(np.float64) for a in ins)
                    ref = oracle.project(*ins, m.grid.dx, m.grid.dy, m.grid.dz, m.grid.rho0)
                errs.append(max_errors(outs[i], ref, ins))
                del ref
                o64 = [x.astype(np.float64, copy=False) for x in outs[i][:3]]
                divs.append(float(np.abs(oracle.divergence(*o64, m.grid.dx, m.grid.dy, m.grid.dz,
                                                           m.grid.rho0)).max()))
                del o64
            worst = [max(e[t] for e in errs) for t in range(4)]
            rec = {"max_rel_err": max(worst), "rel_err_u_v_w_p": worst, "max_abs_divergence": max(divs),
                   "members_checked": n,
                   "reference": "the FP64 oracle" + (" on the FP32-rounded inputs" if path == "mixed" else "")}
            if path == "f64" and len(members) == 1:
                # the round-off floor of p on this input: the spread of two
                # FP64 column solves (bottom-up and top-down elimination) of
                # the oracle's spectrum
                from tests.tolerances import reference_noise
                m = members[0]
                b_spec = oracle.forward_spectrum(oracle.divergence(m.u, m.v, m.w, m.grid.dx, m.grid.dy,
                                                                   m.grid.dz, m.grid.rho0))
                floor = reference_noise(b_spec, refs[0][3], m.grid)
                del b_spec
                rec["p_roundoff_floor"] = floor
                rec["p_err_over_floor"] = worst[3] / floor if floor > 0 else None
            acc["fp64" if path == "f64" else "mixed"] = rec
        result["accuracy"] = acc
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
