"""Benchmark of the MI355X pressure projection (one GPU).

    python bench.py [--steps K] [--warmup W] [--workload c1] [--no-cpu]

A step is one whole projection (divergence, forward FFTs, FP64 tridiagonal
solves, inverse FFTs, gradient correction) of the workload's fields, already
resident in HBM; the projection re-projects its own output in place, which
costs exactly the same kernels and bytes as the first pass. The headline is the
plain FP64 path on the 256^2 x 128 stretched anelastic grid; the mixed
FP32/FP64 path (with its FP64 refinement step) is timed on the same grid and
reported beside it. Prints one JSON line.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_c1.txt")


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
        "ifftx": (f + 1) * wb,                  # read spectrum; write p
        "grad": 7 * wb,                         # read p, u, v, w; write u, v, w
        "resid_fftx": (4 + f) * wb,             # read u, v, w, p1; write spectrum
        "grad_final": 8 + 6 * wb,               # read FP64 p; read/write u, v, w
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


def read_traffic(kernel, mixed):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if it is missing or was taken on another version of the kernels."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernels_sha256_16") != kernel_source_hash():
        return None
    key = f"{'mixed' if mixed else 'fp64'}.{kernel}.bytes_per_launch"
    return float(vals[key]) if key in vals else None


def time_path(plan, fields, steps, warmup, torch, profile_kernel=None):
    u, v, w, p = fields
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.project(u, v, w, p, stream)
    torch.cuda.synchronize()
    if profile_kernel is not None:
        plan.profile_read()
        from paper_2009_12849_amd import KERNELS
        plan.profile_enable(1 << KERNELS.index(profile_kernel))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        plan.project(u, v, w, p, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = None
    if profile_kernel is not None:
        prof = plan.profile_read()
        plan.profile_enable(0)
    return wall, e0.elapsed_time(e1) / 1e3, prof


def kernel_breakdown(plan, fields, steps, torch):
    u, v, w, p = fields
    plan.profile_read()
    plan.profile_enable((1 << 8) - 1)
    for _ in range(steps):
        plan.project(u, v, w, p)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile_enable(0)
    return {k: (ms / n, n // steps) for k, (ms, n) in prof.items()}


def cpu_baseline(member, gpu_out, budget_s=25.0):
    """The FP64 oracle timed on this host (whole projections of the same
    workload, as many as fit the budget, at least one)."""
    import oracle
    g = member.grid
    workers = len(os.sched_getaffinity(0))
    times = []
    out = None
    while True:
        t0 = time.perf_counter()
        out = oracle.project(member.u, member.v, member.w, g.dx, g.dy, g.dz, g.rho0, workers=workers)
        times.append(time.perf_counter() - t0)
        if sum(times) + times[-1] > budget_s or len(times) >= 5:
            break
    med = float(np.median(times))
    res = {"value": g.points / med, "unit": "grid-points/s", "cores": workers, "kind": "oracle",
           "sample": f"{len(times)} whole FP64 projections of the {g.nx}x{g.ny}x{g.nz} grid, median "
                     f"{med:.2f} s (scipy.fft workers={workers}, NumPy elsewhere), host {platform.processor() or platform.machine()}"}
    acc = None
    if gpu_out is not None:
        vs = max(np.abs(member.u).max(), np.abs(member.v).max(), np.abs(member.w).max())
        errs = [float(np.abs(gpu_out[t] - out[t]).max() / vs) for t in range(3)]
        errs.append(float(np.abs(gpu_out[3] - out[3]).max() / np.abs(out[3]).max()))
        div = oracle.divergence(gpu_out[0], gpu_out[1], gpu_out[2], g.dx, g.dy, g.dz, g.rho0)
        acc = {"max_rel_err": max(errs), "rel_err_u_v_w_p": errs, "max_abs_divergence": float(np.abs(div).max())}
    return res, acc, out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c1", choices=["c1"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline leg")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
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

    dev = torch.device("cuda:0")
    wl = synth.make_workload(args.workload)
    m = wl.members[0]
    g = m.grid
    npts = g.points

    # ---- FP64 path ----------------------------------------------------------
    plan = monc.Plan.from_grid(g, "f64")
    fields = [torch.from_numpy(a).to(dev) for a in (m.u, m.v, m.w)]
    fields.append(torch.empty_like(fields[0]))
    plan.project(*fields)
    torch.cuda.synchronize()
    first_out = [t.cpu().numpy() for t in fields]
    breakdown = kernel_breakdown(plan, fields, 5, torch)
    dom = max(breakdown, key=lambda k: breakdown[k][0] * breakdown[k][1])
    wall, ev_s, prof = time_path(plan, fields, args.steps, args.warmup, torch, profile_kernel=dom)
    ms_step = 1e3 * wall / args.steps
    value = npts * args.steps / wall
    dom_ms, dom_n = prof[dom]
    dom_avg_s = dom_ms / dom_n / 1e3
    dom_bytes = kernel_bytes_per_point(dom, g.nx, False) * npts
    achieved = dom_bytes / dom_avg_s / 1e9
    traffic = read_traffic(dom, False)

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: plain FP64 projection {g.nx}x{g.ny}x{g.nz}, dx=dy={g.dx:g} m, "
                               f"dz=min(10*1.015^k,60) m, rho0=1.2exp(-z/8 km), periodic x,y, rigid lids",
                   "grid_points": npts, "fields": "u,v ~ N(0,4)+8 modes, w ~ N(0,0.25), seed 2000"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "avg_launch_ms": dom_avg_s * 1e3,
                     "algorithmic_bytes_per_launch": dom_bytes},
        "path": {"event_ms_per_step": 1e3 * ev_s / args.steps,
                 "algorithmic_bytes_per_point": path_bytes_per_point(g.nx, False),
                 "end_to_end_hbm_frac": path_bytes_per_point(g.nx, False) * value / 1e9 / HBM_PEAK_GBS,
                 "kernels_ms": {k: round(v[0], 5) for k, v in breakdown.items()}},
    }

    # ---- mixed path on the same grid ------------------------------------------
    if not args.no_mixed:
        mplan = monc.Plan.from_grid(g, "mixed")
        mf = [torch.from_numpy(a.astype(np.float32)).to(dev) for a in (m.u, m.v, m.w)]
        mf.append(torch.empty_like(mf[0]))
        mplan.project(*mf)
        torch.cuda.synchronize()
        mixed_out = [t.cpu().numpy().astype(np.float64) for t in mf]
        mbreak = kernel_breakdown(mplan, mf, 5, torch)
        mwall, mev, _ = time_path(mplan, mf, args.steps, args.warmup, torch)
        mvalue = npts * args.steps / mwall
        result["mixed"] = {"value": mvalue, "ms_per_step": 1e3 * mwall / args.steps,
                           "speedup_vs_fp64": mvalue / value,
                           "algorithmic_bytes_per_point": path_bytes_per_point(g.nx, True),
                           "end_to_end_hbm_frac": path_bytes_per_point(g.nx, True) * mvalue / 1e9 / HBM_PEAK_GBS,
                           "kernels_ms": {k: round(v[0], 5) for k, v in mbreak.items()}}

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["calibration_copy_bytes"] = 2 * n * 4

    # ---- CPU baseline (oracle) and accuracy ------------------------------------
    if not args.no_cpu:
        base, acc, ref = cpu_baseline(m, first_out)
        result["cpu_baseline"] = base
        result["accuracy"] = {"fp64": acc}
        if not args.no_mixed:
            import oracle
            ref32 = oracle.project(*(a.astype(np.float32).astype(np.float64) for a in (m.u, m.v, m.w)),
                                   g.dx, g.dy, g.dz, g.rho0)
            vs = max(np.abs(m.u).max(), np.abs(m.v).max(), np.abs(m.w).max())
            errs = [float(np.abs(mixed_out[t] - ref32[t]).max() / vs) for t in range(3)]
            errs.append(float(np.abs(mixed_out[3] - ref32[3]).max() / np.abs(ref32[3]).max()))
            result["accuracy"]["mixed"] = {"max_rel_err": max(errs), "rel_err_u_v_w_p": errs}
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
