"""Benchmark of the MI355X pressure projection (one GPU).

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

A step is one whole projection (divergence, forward FFTs, FP64 tridiagonal
solves, inverse FFTs, gradient correction) of the workload's fields, already
resident in HBM; the projection re-projects its own output in place, which
costs exactly the same kernels and bytes as the first pass.

Workloads (seeded synthetic stand-ins for the paper's dry boundary-layer
case, see synth/):
  256x256x128    stretched anelastic grid; headline = plain FP64 path, the
                 mixed FP32/FP64 path (one FP64 refinement step) timed
                 beside it (default)
  1024x1024x256  same vertical profiles; headline = mixed, FP64 beside it
  ensemble48     48-member ensemble of uneven grids, one batched call (HIP
                 graph); headline = mixed, FP64 beside it
  2048x2048x160  k^-5/3 spectra; headline = mixed, FP64 beside it
Single grids up to 3e8 points also time the variable-density projection
(conjugate gradients with the spectral solve as preconditioner, a seeded
density rho0(z)(1 + 0.2 f(x, y, z))) under "variable_density".
Prints one JSON line.
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
KERNEL_SRC = os.path.join(ROOT, "paper_2009_12849_amd", "csrc", "kernels.hip")
WORKLOADS = ["256x256x128", "1024x1024x256", "ensemble48", "2048x2048x160", "4096x4096x64"]
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
        # read spectrum, write p; on the mixed path the mean of its two
        # launches: p1 (f + 1 words), then the correction (read spectrum and
        # p1, write p and the remainder: f + 3 words)
        "ifftx": (f + 2) * wb if mixed else (f + 1) * wb,
        "grad": 7 * wb,                         # read p, u, v, w; write u, v, w
        "resid_fftx": (4 + f) * wb,             # read u, v, w, p1; write spectrum
        "grad_final": 8 * wb,                   # read p and remainder; read/write u, v, w
    }
    return table[kernel]


def path_bytes_per_point(nx, mixed):
    """Minimum HBM traffic of the whole path (inputs once, one round trip of
    the spectrum per global-dependency boundary, outputs once): FP64
    10 + 4f words, mixed with one refinement step 16 + 8f words."""
    f = spectral_words(nx)
    return (16 + 8 * f) * 4.0 if mixed else (10 + 4 * f) * 8.0


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


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


class Runner:
    """Owns the plans and device fields of one path (FP64 or mixed) of a
    workload and runs whole projections on them."""

    def __init__(self, monc, torch, members, dtype, tune=True):
        self.torch = torch
        self.monc = monc
        self.mixed = dtype == "mixed"
        cast = np.float32 if self.mixed else np.float64
        self.plans = [monc.Plan.from_grid(m.grid, dtype) for m in members]
        self.tuned = {}
        if tune:
            # the library's autotuner picks the tile parameters once per
            # distinct grid (untimed); plans of the same grid reuse them
            for pl in self.plans:
                key = (pl.nx, pl.ny, pl.nz)
                if key not in self.tuned:
                    pl.autotune()
                    self.tuned[key] = pl.params
                else:
                    pl.params = self.tuned[key]
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
        """Wall-clock time of `steps` projections; with profile_kernel, HIP
        events on the launch stream bracket every launch of that kernel."""
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


def measure(runner, steps, warmup, workload, nx_bytes):
    """Throughput, kernel breakdown and dominant-kernel roofline of a path."""
    bd = runner.breakdown(3)
    dom = max(bd, key=lambda k: bd[k][0] * bd[k][1])
    wall, _ = runner.timed(steps, warmup)                    # clean timing
    _, prof = runner.timed(steps, 0, profile_kernel=dom)     # events around the dominant kernel
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
    return {
        "value": value,
        "ms_per_step": 1e3 * wall / steps,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": read_traffic(workload, dom, runner.mixed),
                     "avg_launch_ms": dom_avg_s * 1e3, "algorithmic_bytes_per_launch": per_launch},
        "path": {"algorithmic_bytes_per_point": path_bytes / runner.points,
                 "end_to_end_hbm_frac": path_bytes * steps / wall / 1e9 / HBM_PEAK_GBS,
                 "kernels_ms": {k: round(v[0], 5) for k, v in bd.items()},
                 "launches_per_step": {k: v[1] for k, v in bd.items()}},
    }


def var_iteration_bytes_per_point(nx, mixed):
    """Algorithmic HBM bytes per grid point of one conjugate-gradient
    iteration of the variable-density projection: the operator (read d and
    rho, write q), the update (read p, d, r, q and the FP32 scaling s; write
    p, r), the spectral preconditioner (read r, the spectrum's four round
    trips, write z in the plan's storage type), the inner products (read r
    and z; with the FP32 preconditioner's flexible update also q and s) and
    the direction update (read z, d, s; write d). FP64 136 + 64f, mixed
    136 + 32f."""
    f = spectral_words(nx)
    wb = 4.0 if mixed else 8.0
    dots = (8 + wb + 8 + 4) if mixed else (8 + wb)
    return 24 + (48 + 4) + (8 + 8 * f * wb + wb) + dots + (16 + wb + 4)


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


def device_copy_gbps(torch, mb=2048, reps=10):
    """Read+write bandwidth of a plain device-to-device copy (context for the
    HBM peak)."""
    n = mb * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del src, dst
    return 2 * n * 4 / dt / 1e9


def max_errors(out, ref, members_in):
    """Normwise errors of u, v, w (relative to the input velocity scale) and p."""
    u, v, w = members_in
    vs = max(np.abs(u).max(), np.abs(v).max(), np.abs(w).max())
    errs = [float(np.abs(out[t] - ref[t]).max() / vs) for t in range(3)]
    errs.append(float(np.abs(out[3] - ref[3]).max() / np.abs(ref[3]).max()))
    return errs


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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="256x256x128", choices=WORKLOADS)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline leg")
    ap.add_argument("--no-other", action="store_true", help="time only the headline path")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile parameters")
    ap.add_argument("--no-var", action="store_true", help="skip the variable-density solve")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="also run a device copy of this many MB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the projection is built and measured on a single "
              "MI355X (sharding across GPUs is described, not built). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2009_12849_amd as monc

    wl = synth.make_workload(args.workload)
    members = wl.members
    head = "f64" if args.workload == "256x256x128" else "mixed"
    other = "mixed" if head == "f64" else "f64"
    g = members[0].grid
    desc = {
        "256x256x128": f"plain FP64 projection {g.nx}x{g.ny}x{g.nz}, dx=dy=25 m, dz=min(10*1.015^k,60) m, "
              f"rho0=1.2exp(-z/8 km), periodic x,y, rigid lids",
        "1024x1024x256": f"mixed FP32/FP64 projection with one FP64 refinement step, {g.nx}x{g.ny}x{g.nz}, "
              f"dz=min(10*1.015^k,60) m, rho0=1.2exp(-z/8 km)",
        "ensemble48": f"batched ensemble of {len(members)} uneven grids (64^2x64..256^2x128), one graph launch, mixed",
        "2048x2048x160": f"mixed projection {g.nx}x{g.ny}x{g.nz}, dz=5*20^(k/159) m, rho0=1.2exp(-z/8 km), "
              f"k^-5/3 horizontal spectra",
        "4096x4096x64": f"mixed projection {g.nx}x{g.ny}x{g.nz} (the paper's 1.07e9-point global problem on one "
              f"GPU), dz=min(10*1.015^k,60) m, rho0=1.2exp(-z/8 km)",
    }[args.workload]

    copy_gbps = device_copy_gbps(torch)
    runner = Runner(monc, torch, members, head, tune=not args.no_tune)
    runner.step()
    torch.cuda.synchronize()
    nchk = 1 if len(members) == 1 else 3      # members whose outputs the oracle checks
    first = ([[t.cpu().numpy().astype(np.float64) for t in f] for f in runner.fields[:nchk]]
             if not args.no_cpu else None)
    res = measure(runner, args.steps, args.warmup, args.workload, None)
    reductions = None
    if not runner.batched:
        # the same projections with the per-level horizontal reductions fused in
        runner.stats = torch.empty(8 * runner.plans[0].nz, dtype=torch.float64, device="cuda:0")
        wall_r, _ = runner.timed(args.steps, args.warmup)
        runner.stats = None
        ms_r = 1e3 * wall_r / args.steps
        reductions = {"ms_per_step": ms_r, "overhead_frac": ms_r / res["ms_per_step"] - 1.0,
                      "what": "per-level horizontal mean and max of u, v, w, p (monc_project_reduce)"}
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
        "config": {"workload": desc, "grid_points": runner.points, "members": len(members),
                   "path": "fp64" if head == "f64" else "mixed",
                   "tile_params": {f"{k[0]}x{k[1]}x{k[2]}": v for k, v in runner.tuned.items()}},
        "roofline": res["roofline"],
        "path": res["path"],
        "device_copy_GBps": copy_gbps,
        "with_reductions": reductions,
    }
    if not args.no_var and not runner.batched and runner.points <= 300_000_000:
        result["variable_density"] = variable_density(monc, torch, members[0])
        if not args.no_cpu:
            result["variable_density"]["cpu_baseline"] = variable_cpu_baseline()
    if not args.no_other:
        del runner
        torch.cuda.empty_cache()
        orun = Runner(monc, torch, members, other, tune=not args.no_tune)
        orun.step()
        torch.cuda.synchronize()
        ofirst = ([[t.cpu().numpy().astype(np.float64) for t in f] for f in orun.fields[:nchk]]
                  if not args.no_cpu else None)
        ores = measure(orun, args.steps, args.warmup, args.workload, None)
        key = "mixed" if other == "mixed" else "fp64"
        result[key] = {"value": ores["value"], "ms_per_step": ores["ms_per_step"],
                       "roofline": ores["roofline"], "path": ores["path"],
                       "tile_params": {f"{k[0]}x{k[1]}x{k[2]}": v for k, v in orun.tuned.items()}}
        sp = res["value"] / ores["value"] if head == "mixed" else ores["value"] / res["value"]
        result["mixed_speedup_vs_fp64"] = sp
        del orun
    else:
        ofirst = None

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["calibration_copy_bytes"] = 2 * n * 4

    if not args.no_cpu:
        base, refs = cpu_baseline(members)
        result["cpu_baseline"] = base
        acc = {}
        import oracle
        n = min(len(refs), nchk)
        for name, outs in (("head", first), ("other", ofirst)):
            if outs is None:
                continue
            path = head if name == "head" else other
            errs = []
            for i in range(n):
                m = members[i]
                ins = (m.u, m.v, m.w)
                ref = refs[i]
                if path == "mixed":   # the oracle on the FP32-rounded inputs
                    g_ = m.grid
                    ins = tuple(a.astype(np.float32).astype(np.float64) for a in ins)
                    ref = oracle.project(*ins, g_.dx, g_.dy, g_.dz, g_.rho0)
                errs.append(max_errors(outs[i], ref, ins))
            worst = [max(e[t] for e in errs) for t in range(4)]
            div = max(float(np.abs(oracle.divergence(outs[i][0], outs[i][1], outs[i][2], members[i].grid.dx,
                                                     members[i].grid.dy, members[i].grid.dz,
                                                     members[i].grid.rho0)).max()) for i in range(n))
            acc["fp64" if path == "f64" else "mixed"] = {"max_rel_err": max(worst), "rel_err_u_v_w_p": worst,
                                                         "max_abs_divergence": div, "members_checked": n}
        result["accuracy"] = acc
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
