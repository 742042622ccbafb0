"""Parity of the HIP path (called through the C ABI) with the FP64 oracle.

Tolerances (errors are normwise: velocities relative to the input velocity
scale, p relative to max|p|):
  FP64 path   velocities within 1e-12 of the oracle; p within
              max(1e-12, 4 u kappa), where kappa is the infinity-norm condition
              number of the worst-conditioned wavenumber column (smallest
              nonzero lambda) and u = 2^-53: the GPU's partitioned elimination
              and the oracle's Thomas sweep are both backward stable, so each
              lies within about kappa u of the exact solution. The output's
              divergence stays below 1e-12 in SI units.
  mixed path  every field within 1e-6 of the FP64 oracle run on the FP32
              inputs upcast to FP64 (the accuracy target of the mixed path).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import relerr
from tests.tolerances import TOL64, TOL_MIXED, p_tolerance, worst_column_condition  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2009_12849_amd as monc  # noqa: E402

DEV = "cuda:0"


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def run_gpu(g, u, v, w, dtype="f64", plan=None):
    plan = plan or monc.Plan.from_grid(g, dtype)
    tdt = plan.torch_dtype
    tu, tv, tw = to_dev(u, tdt), to_dev(v, tdt), to_dev(w, tdt)
    tp = torch.empty_like(tu)
    plan.project(tu, tv, tw, tp)
    torch.cuda.synchronize()
    return [t.cpu().numpy().astype(np.float64) for t in (tu, tv, tw, tp)]


def field_errors(out, ref, u, v, w):
    vs = max(np.max(np.abs(u)), np.max(np.abs(v)), np.max(np.abs(w)))
    errs = [np.max(np.abs(out[t] - ref[t])) / vs for t in range(3)]
    errs.append(relerr(out[3], ref[3]))
    return errs


def check_fp64(g, u, v, w, tol=TOL64):
    print(f"case {g.nx}x{g.ny}x{g.nz} fp64", flush=True)
    ref = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0)
    out = run_gpu(g, u, v, w, "f64")
    errs = field_errors(out, ref, u, v, w)
    assert max(errs[:3]) <= tol, errs
    assert errs[3] <= max(tol, p_tolerance(g)), (errs, p_tolerance(g))
    assert np.all(out[2][-1] == 0.0)
    div = oracle.divergence(out[0], out[1], out[2], g.dx, g.dy, g.dz, g.rho0)
    assert np.max(np.abs(div)) <= 1e-12
    return errs


# ---------------------------------------------------------------------------
# stage-wise
# ---------------------------------------------------------------------------
STAGE_SHAPES = [(32, 32, 32), (48, 27, 13), (24, 18, 9), (1, 6, 5), (12, 1, 3), (64, 64, 130)]
# y-FFT columns per workgroup; the spectral column blocks follow it (1..8 wide)
STAGE_YMT = [1, 2, 4, 8]


def _with_ymt(plan, ymt):
    prm = list(plan.params)
    prm[2] = ymt
    plan.params = prm
    return plan


def _case(shape, seed):
    # dz grows by at most a factor 20 over the column (as 5 m -> 100 m)
    rng = np.random.default_rng(seed)
    g = synth.random_grid(rng, *shape, stretch=(1.0, min(1.1, 20.0 ** (1.0 / max(shape[2], 1)))))
    return (g,) + synth.random_fields(rng, g)


@pytest.mark.parametrize("ymt", STAGE_YMT)
@pytest.mark.parametrize("shape", STAGE_SHAPES)
def test_stage_forward_spectrum(shape, ymt):
    g, u, v, w = _case(shape, 1)
    ref = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0, intermediates=True)
    plan = _with_ymt(monc.Plan.from_grid(g, "f64"), ymt)
    spec = plan.spectral_buffer()
    bufs = [to_dev(a, torch.float64) for a in (u, v, w)] + [spec]
    plan.debug_stage(monc.STAGE_FORWARD, bufs)
    torch.cuda.synchronize()
    got = plan.spectral_get(spec).cpu().numpy()
    assert relerr(got, ref["B"]) <= 1e-13


@pytest.mark.parametrize("ymt", STAGE_YMT)
@pytest.mark.parametrize("shape", STAGE_SHAPES)
def test_stage_solve_columns(shape, ymt):
    g, u, v, w = _case(shape, 2)
    ref = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0, intermediates=True)
    plan = _with_ymt(monc.Plan.from_grid(g, "f64"), ymt)
    spec = plan.spectral_buffer()
    plan.spectral_set(spec, torch.from_numpy(ref["B"]))
    plan.debug_stage(monc.STAGE_SOLVE, [spec])
    torch.cuda.synchronize()
    got = plan.spectral_get(spec).cpu().numpy()
    assert relerr(got, ref["P"] / (g.nx * g.ny)) <= p_tolerance(g)


@pytest.mark.parametrize("ymt", [1, 8])
@pytest.mark.parametrize("shape", [(48, 27, 13), (64, 64, 130)])
def test_spectral_layout_formula(shape, ymt):
    # the buffer positions follow the documented formula (column blocks of B)
    g, u, v, w = _case(shape, 4)
    plan = _with_ymt(monc.Plan.from_grid(g, "f64"), ymt)
    n_el, row, blk, plane, eb = plan.spectral_layout()
    nxh = g.nx // 2 + 1
    assert eb == 16 and row >= nxh and row % 8 == 0 and blk in (1, 2, 4, 8) and row % blk == 0
    eff = plan.params[2]  # the tile width the plan kept (clamped to the grid)
    assert blk == min(8, 1 << (eff.bit_length() - 1)) and plane >= g.ny * row and n_el == g.nz * plane
    spec = plan.spectral_buffer()
    vals = np.arange(g.nz * g.ny * nxh, dtype=np.float64).reshape(g.nz, g.ny, nxh) + 1.0
    plan.spectral_set(spec, torch.from_numpy(vals.astype(np.complex128)))
    raw = spec.cpu().numpy().reshape(-1)
    k, n, m = np.meshgrid(np.arange(g.nz), np.arange(g.ny), np.arange(nxh), indexing="ij")
    pos = k * plane + (m // blk) * g.ny * blk + n * blk + (m % blk)
    assert np.array_equal(raw[pos].real, vals)
    assert np.count_nonzero(raw) == vals.size


@pytest.mark.parametrize("ymt", STAGE_YMT)
@pytest.mark.parametrize("shape", STAGE_SHAPES)
def test_stage_inverse_and_gradient(shape, ymt):
    g, u, v, w = _case(shape, 3)
    ref = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0, intermediates=True)
    plan = _with_ymt(monc.Plan.from_grid(g, "f64"), ymt)
    spec = plan.spectral_buffer()
    plan.spectral_set(spec, torch.from_numpy(ref["P"] / (g.nx * g.ny)))
    p = torch.empty((g.nz, g.ny, g.nx), dtype=torch.float64, device=DEV)
    plan.debug_stage(monc.STAGE_INVERSE, [spec, p])
    torch.cuda.synchronize()
    assert relerr(p.cpu().numpy(), ref["p"]) <= 1e-13
    tu, tv, tw = (to_dev(a, torch.float64) for a in (u, v, w))
    pp = to_dev(ref["p"], torch.float64)
    plan.debug_stage(monc.STAGE_GRADIENT, [pp, tu, tv, tw])
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in (tu, tv, tw)]
    for o, r in zip(out, (ref["u"], ref["v"], ref["w"])):
        assert np.max(np.abs(o - r)) <= 1e-14 * max(np.abs(u).max(), np.abs(w).max())


# ---------------------------------------------------------------------------
# end to end, FP64
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(4, 4, 3), (6, 3, 4), (6, 4, 5), (8, 8, 6), (1, 1, 4), (4, 4, 1),
                                   (3, 2, 2), (9, 6, 3), (2, 3, 5), (1, 1, 1)])
def test_fp64_tiny_grids(shape):
    g, u, v, w = _case(shape, sum(shape))
    check_fp64(g, u, v, w)


@pytest.mark.parametrize("shape", [(48, 27, 13), (192, 96, 40), (64, 1, 8), (3, 64, 7), (96, 72, 33),
                                   (256, 8, 17), (16, 16, 700), (8, 6, 1024), (2048, 4, 3), (6, 1536, 2),
                                   (768, 6, 4), (1536, 4, 3), (4096, 2, 3), (512, 6, 4)])
def test_fp64_ragged_and_extreme_shapes(shape):
    g, u, v, w = _case(shape, 7)
    check_fp64(g, u, v, w)


@pytest.mark.parametrize("shape", [(8192, 2, 3), (2, 8192, 2), (6561, 3, 2), (4, 6561, 3)])
@pytest.mark.parametrize("dtype", ["f64", "mixed"])
def test_size_limits(shape, dtype):
    # nx or ny = 8192 (the limit) and 3^8 take the runtime-length FFT kernels at
    # their largest LDS footprint. The layers are 1 km thick: with the ~10 m
    # layers of the other cases a 400 km long, 20 m deep domain has a longest
    # mode with kappa ~ 1e8, and the flat velocity tolerance would then test
    # the conditioning rather than the kernels.
    rng = np.random.default_rng(24)
    nx, ny, nz = shape
    g = synth.Grid(nx, ny, nz, 50.0, 40.0, 1000.0 * rng.uniform(0.8, 1.2, nz), rng.uniform(0.5, 1.5, nz))
    u, v, w = synth.random_fields(rng, g)
    if dtype == "f64":
        check_fp64(g, u, v, w)
    else:
        errs, out, ref = mixed_case(g, u, v, w)
        assert max(errs) <= TOL_MIXED, errs


def test_fp64_32x32x32():
    m = synth.make_workload("32x32x32").members[0]
    check_fp64(m.grid, m.u, m.v, m.w)


def test_fp64_256x256x128_full_size():
    m = synth.make_workload("256x256x128").members[0]
    errs = check_fp64(m.grid, m.u, m.v, m.w)
    print("256x256x128 fp64 errors u,v,w,p:", errs)


@pytest.mark.parametrize("shape,dtype", [((1024, 648, 11), "f64"), ((864, 648, 9), "f64"), ((1536, 864, 5), "mixed"),
                                         ((2048, 648, 6), "mixed")])
def test_large_levels_tiled_stencil_order(shape, dtype):
    # a level of one field above 4 MB switches the stencil kernels to
    # (8 level x J row pair) tiles (about 512 KB of rows: J = 16 to 64 at
    # these widths), and the gradient kernels to (8 level x 8 row) tiles where a
    # row is a whole number of blocks (nx = 1024 FP64, 2048 mixed); ragged in
    # both (324 or 432 pairs per level, 5..11 levels), compile-time (1024,
    # 1536, 2048) and runtime (864) x FFTs
    g, u, v, w = _case(shape, 21)
    if dtype == "f64":
        check_fp64(g, u, v, w)
    else:
        errs, out, ref = mixed_case(g, u, v, w)
        assert max(errs) <= TOL_MIXED, errs


def test_fp64_deterministic_and_bitwise_repeatable():
    g, u, v, w = _case((96, 72, 33), 9)
    plan = monc.Plan.from_grid(g, "f64")
    a = run_gpu(g, u, v, w, plan=plan)
    b = run_gpu(g, u, v, w, plan=plan)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("dtype", ["f64", "mixed"])
@pytest.mark.parametrize("lid", [123.0, np.nan, np.inf])
def test_lid_input_ignored(dtype, lid):
    # w[nz-1] is documented as ignored on input: no value there, not even a
    # NaN or an infinity, may reach any output
    g, u, v, w = _case((32, 24, 10), 10)
    cast = np.float64 if dtype == "f64" else np.float32
    u, v, w = (x.astype(cast).astype(np.float64) for x in (u, v, w))
    w2 = w.copy()
    w2[-1] = lid
    a = run_gpu(g, u, v, w, dtype)
    b = run_gpu(g, u, v, w2, dtype)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# ---------------------------------------------------------------------------
# mixed path
# ---------------------------------------------------------------------------
def mixed_case(g, u, v, w):
    u32, v32, w32 = (a.astype(np.float32) for a in (u, v, w))
    ref = oracle.project(u32.astype(np.float64), v32.astype(np.float64), w32.astype(np.float64),
                         g.dx, g.dy, g.dz, g.rho0)
    out = run_gpu(g, u32, v32, w32, "mixed")
    errs = field_errors(out, ref, u32, v32, w32)
    return errs, out, ref


@pytest.mark.parametrize("shape", [(32, 32, 32), (48, 27, 13), (192, 96, 40), (1, 1, 4), (64, 64, 130),
                                   (18, 12, 7), (27, 9, 6), (768, 12, 5), (1536, 9, 3), (3072, 4, 3)])
def test_mixed_small(shape):
    # nx = 18 and 27 take the 2- and 1-point gradient variants (4 otherwise);
    # nx = 768 and 1536 x-transforms have thread counts that are not
    # multiples of the wave size, so two transforms share a wave
    g, u, v, w = _case(shape, 11)
    errs, out, ref = mixed_case(g, u, v, w)
    print(f"mixed {shape}: {errs}")
    assert max(errs) <= TOL_MIXED, errs
    assert np.all(out[2][-1] == 0.0)


@pytest.mark.parametrize("nx,xpws", [(64, [1, 3, 12]), (128, [1, 5]), (192, [1, 9, 21]), (256, [1, 2, 3, 8]),
                                     (384, [1, 10]), (512, [1, 4]), (768, [1, 4, 9]), (1536, [1, 3])])
@pytest.mark.parametrize("ny", [6, 9])
def test_mixed_residual_whole_rows_per_wave(nx, xpws, ny):
    # at these lengths the residual's stencil walks whole rows per wave (in
    # runs of 64 chunks of 1, 2 or 4 points) and the host rounds its
    # transforms per workgroup to whole waves (up, or down where up passes
    # 512 threads: 21 x 24 -> 16 x 24, 10 x 48 -> 8 x 48, 9 x 48 -> 8 x 48);
    # each transform's arithmetic does not depend on the grouping, so every
    # value gives the same bits, within the oracle's bound. ny = 9: rows pair
    # across levels (single-row stencils) and the last pair has one row
    g, u, v, w = _case((nx, ny, 5), 23)
    u32, v32, w32 = (a.astype(np.float32) for a in (u, v, w))
    ref = oracle.project(u32.astype(np.float64), v32.astype(np.float64), w32.astype(np.float64),
                         g.dx, g.dy, g.dz, g.rho0)
    outs = []
    for xpw in xpws:
        print(f"case residual whole rows nx={nx} ny={ny} xpw={xpw}", flush=True)
        plan = monc.Plan.from_grid(g, "mixed")
        plan.params = [0, 0, 0, 0, 0, xpw, 0]
        assert plan.params[5] == xpw
        out = run_gpu(g, u32, v32, w32, "mixed", plan=plan)
        errs = field_errors(out, ref, u32, v32, w32)
        assert max(errs) <= TOL_MIXED, (xpw, errs)
        outs.append(out)
        plan.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_mixed_256x256x128_with_ir_gain():
    m = synth.make_workload("256x256x128").members[0]
    g = m.grid
    errs, out, ref = mixed_case(g, m.u, m.v, m.w)
    print("256x256x128 mixed errors u,v,w,p:", errs)
    assert max(errs) <= TOL_MIXED, errs
    # first pass alone (forward, solve, inverse stages) is clearly worse
    plan = monc.Plan.from_grid(g, "mixed")
    u32, v32, w32 = (to_dev(a.astype(np.float32), torch.float32) for a in (m.u, m.v, m.w))
    spec = plan.spectral_buffer()
    plan.debug_stage(monc.STAGE_FORWARD, [u32, v32, w32, spec])
    plan.debug_stage(monc.STAGE_SOLVE, [spec])
    p1 = torch.empty_like(u32)
    plan.debug_stage(monc.STAGE_INVERSE, [spec, p1])
    torch.cuda.synchronize()
    e1 = relerr(p1.cpu().numpy().astype(np.float64), ref[3])
    print("256x256x128 mixed p error before refinement:", e1, "after:", errs[3])
    assert errs[3] < e1


# ---------------------------------------------------------------------------
# batched
# ---------------------------------------------------------------------------
def _ensemble(n, shapes, seed):
    rng = np.random.default_rng(seed)
    mem = []
    for i in range(n):
        shp = shapes[rng.integers(len(shapes))]
        g = synth.random_grid(rng, *shp, stretch=(1.0, 1.02))
        mem.append((g,) + synth.random_fields(rng, g))
    return mem


@pytest.mark.parametrize("dtype", ["f64", "mixed"])
def test_batched_equals_members_and_oracle(dtype):
    mem = _ensemble(7, [(32, 32, 16), (48, 48, 24), (64, 32, 20), (24, 36, 12), (96, 96, 9)], 12)
    plans = [monc.Plan.from_grid(g, dtype) for g, *_ in mem]
    tdt = plans[0].torch_dtype
    cast = np.float64 if dtype == "f64" else np.float32
    fields = [[to_dev(a.astype(cast), tdt) for a in (u, v, w)] for _, u, v, w in mem]
    ps = [torch.empty_like(f[0]) for f in fields]
    monc.project_batched(plans, [f[0] for f in fields], [f[1] for f in fields], [f[2] for f in fields], ps)
    torch.cuda.synchronize()
    for i, (g, u, v, w) in enumerate(mem):
        single = run_gpu(g, u.astype(cast), v.astype(cast), w.astype(cast), dtype)
        got = [f.cpu().numpy().astype(np.float64) for f in fields[i]] + [ps[i].cpu().numpy().astype(np.float64)]
        for a, b in zip(got, single):
            assert np.array_equal(a, b), f"member {i} differs from its single projection"
        ref = oracle.project(u.astype(cast).astype(np.float64), v.astype(cast).astype(np.float64),
                             w.astype(cast).astype(np.float64), g.dx, g.dy, g.dz, g.rho0)
        errs = field_errors(got, ref, u, v, w)
        if dtype == "f64":
            assert max(errs[:3]) <= TOL64 and errs[3] <= p_tolerance(g), (i, errs)
        else:
            assert max(errs) <= TOL_MIXED, (i, errs)


@pytest.mark.parametrize("dtype", ["f64", "mixed"])
def test_batch_schedules_equal_member_projections(dtype):
    # every member order, grouping (one group; groups of about 1 MB, i.e.
    # one or two members each; 8 MB) and number of graph branches the groups
    # run on gives each member its single projection bit for bit
    mem = _ensemble(7, [(32, 32, 16), (48, 48, 24), (64, 32, 20), (24, 36, 12), (96, 96, 9)], 41)
    plans = [monc.Plan.from_grid(g, dtype) for g, *_ in mem]
    tdt = plans[0].torch_dtype
    cast = np.float64 if dtype == "f64" else np.float32
    singles = [run_gpu(g, u.astype(cast), v.astype(cast), w.astype(cast), dtype) for g, u, v, w in mem]
    for order, budget, branches in [(0, 0, 1), (0, 1, 1), (0, 8, 1), (1, 0, 1), (1, 1, 1), (1, 8, 1),
                                    (0, 1, 2), (1, 1, 4), (0, 8, 2)]:
        monc.set_batch_schedule(plans, order, budget, branches)
        o, b, ngroups, nb = monc.batch_schedule(plans)
        assert (o, b, nb) == (order, budget, branches)
        assert (ngroups == 1) if budget == 0 else (ngroups > 1), ngroups
        fields = [[to_dev(a.astype(cast), tdt) for a in (u, v, w)] for _, u, v, w in mem]
        ps = [torch.empty_like(f[0]) for f in fields]
        monc.project_batched(plans, [f[0] for f in fields], [f[1] for f in fields], [f[2] for f in fields], ps)
        torch.cuda.synchronize()
        for i in range(len(mem)):
            got = [t.cpu().numpy().astype(np.float64) for t in fields[i] + [ps[i]]]
            for a, ref in zip(got, singles[i]):
                assert np.array_equal(a, ref), (order, budget, branches, i)


def test_batch_with_whole_row_residual_equals_member_projections():
    # members whose residual walks whole rows per wave (nx = 256, 768, 192),
    # with transforms per workgroup that the host rounds to whole waves (3 ->
    # 4, 1 -> 2, 1 -> 4, 5 -> 8), beside one that takes the per-thread
    # mapping (96), in one grouped batch: each member's projection bit for bit
    mem = _ensemble(1, [(256, 6, 5)], 50) + _ensemble(1, [(256, 9, 4)], 51) + _ensemble(1, [(768, 4, 3)], 52) \
        + _ensemble(1, [(192, 6, 5)], 54) + _ensemble(1, [(96, 8, 6)], 53)
    xpws = [3, 1, 1, 5, 0]
    plans = []
    for (g, *_), xpw in zip(mem, xpws):
        pl = monc.Plan.from_grid(g, "mixed")
        pl.params = [0, 0, 0, 0, 0, xpw, 0]
        plans.append(pl)
    print("case batch with whole-row residual", flush=True)
    singles = [run_gpu(g, u.astype(np.float32), v.astype(np.float32), w.astype(np.float32), "mixed", plan=pl)
               for (g, u, v, w), pl in zip(mem, plans)]
    fields = [[to_dev(a.astype(np.float32), torch.float32) for a in (u, v, w)] for _, u, v, w in mem]
    ps = [torch.empty_like(f[0]) for f in fields]
    monc.project_batched(plans, [f[0] for f in fields], [f[1] for f in fields], [f[2] for f in fields], ps)
    torch.cuda.synchronize()
    for i in range(len(mem)):
        got = [t.cpu().numpy().astype(np.float64) for t in fields[i] + [ps[i]]]
        for a, ref in zip(got, singles[i]):
            assert np.array_equal(a, ref), i
    for pl in plans:
        pl.close()


def test_batch_autotune_picks_a_schedule_and_caches_it(tmp_path, monkeypatch):
    import json
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("MONC_TUNE_CACHE", str(cache))
    mem = _ensemble(6, [(32, 32, 16), (64, 64, 24), (48, 24, 12)], 42)
    plans = [monc.Plan.from_grid(g, "mixed") for g, *_ in mem]
    monc.autotune_batched(plans)
    order, budget, ngroups, branches = monc.batch_schedule(plans)
    data = json.loads(cache.read_text())
    keys = [k for k in data if k.startswith("gfx950:batch:6:") and k.endswith(":mixed")]
    assert len(keys) == 1 and data[keys[0]] == [order, budget, branches], data
    # plans of the same grid share the tuned tile parameters
    for i in range(len(mem)):
        for j in range(i):
            if mem[i][0].key() == mem[j][0].key():
                assert plans[i].params == plans[j].params
    # a fresh set of plans of the same grids reads the schedule back
    plans2 = [monc.Plan.from_grid(g, "mixed") for g, *_ in mem]
    assert monc.batch_schedule(plans2)[:2] == (order, budget) and monc.batch_schedule(plans2)[3] == branches
    fields = [[to_dev(a.astype(np.float32), torch.float32) for a in (u, v, w)] for _, u, v, w in mem]
    ps = [torch.empty_like(f[0]) for f in fields]
    monc.project_batched(plans2, [f[0] for f in fields], [f[1] for f in fields], [f[2] for f in fields], ps)
    torch.cuda.synchronize()
    for i, (g, u, v, w) in enumerate(mem):
        u32, v32, w32 = (a.astype(np.float32) for a in (u, v, w))
        ref = oracle.project(u32.astype(np.float64), v32.astype(np.float64), w32.astype(np.float64),
                             g.dx, g.dy, g.dz, g.rho0)
        got = [t.cpu().numpy().astype(np.float64) for t in fields[i] + [ps[i]]]
        assert max(field_errors(got, ref, u32, v32, w32)) <= TOL_MIXED, i


def test_batched_graph_replays():
    mem = _ensemble(5, [(32, 32, 16), (48, 24, 12), (64, 64, 8)], 13)
    plans = [monc.Plan.from_grid(g, "mixed") for g, *_ in mem]
    base = [[a.astype(np.float32) for a in (u, v, w)] for _, u, v, w in mem]
    fields = [[to_dev(a, torch.float32) for a in b] for b in base]
    ps = [torch.empty_like(f[0]) for f in fields]
    results = []
    for rep in range(3):
        for f, b in zip(fields, base):           # restore the inputs eagerly
            for t, a in zip(f, b):
                t.copy_(torch.from_numpy(a).to(DEV))
        torch.cuda.synchronize()
        monc.project_batched(plans, [f[0] for f in fields], [f[1] for f in fields],
                             [f[2] for f in fields], ps)
        torch.cuda.synchronize()
        results.append([[t.cpu().numpy().copy() for t in f + [p]] for f, p in zip(fields, ps)])
    for rep in (1, 2):
        for a, b in zip(results[0], results[rep]):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)


def test_batched_rejects_mixed_dtypes():
    g, u, v, w = _case((16, 16, 8), 14)
    p64 = monc.Plan.from_grid(g, "f64")
    p32 = monc.Plan.from_grid(g, "mixed")
    a = [to_dev(x, torch.float64) for x in (u, v, w)] + [torch.empty((8, 16, 16), dtype=torch.float64, device=DEV)]
    b = [to_dev(x, torch.float32) for x in (u, v, w)] + [torch.empty((8, 16, 16), dtype=torch.float32, device=DEV)]
    with pytest.raises(monc.MoncError, match="mixes dtypes"):
        monc.project_batched([p64, p32], [a[0], b[0]], [a[1], b[1]], [a[2], b[2]], [a[3], b[3]])


def test_plan_rejects_too_many_elements_per_thread():
    g, u, v, w = _case((96, 48, 16), 17)
    plan = monc.Plan.from_grid(g, "f64")
    with pytest.raises(monc.MoncError, match="elements per thread"):
        plan.params = [16, 16, 0, 0, 0]


def test_plan_rejects_prime_factor_5():
    with pytest.raises(monc.MoncError, match="prime factor"):
        monc.Plan(5, 3, 4, 10.0, 10.0, np.full(4, 10.0), np.ones(4))


def test_project_rejects_bad_pointers():
    g, u, v, w = _case((16, 16, 8), 15)
    plan = monc.Plan.from_grid(g, "f64")
    t = to_dev(u, torch.float64)
    L = monc.lib()
    import ctypes
    vp = ctypes.c_void_p
    rc = L.monc_project(plan.handle, vp(t.data_ptr()), vp(t.data_ptr()), vp(t.data_ptr() + 8 * 16),
                        vp(t.data_ptr()), None)
    assert rc == monc.EINVAL
    rc = L.monc_project(plan.handle, vp(t.data_ptr() + 8), vp(0), vp(0), vp(0), None)
    assert rc == monc.EINVAL


# ---------------------------------------------------------------------------
# tuning parameters keep results within tolerance
# ---------------------------------------------------------------------------
TILE_PARAMS = [[4, 4, 1, 0, 0], [2, 2, 4, 0, 0], [8, 8, 32, 0, 0], [8, 8, 8, 64, 0], [8, 8, 8, 32, 0],
               [8, 8, 8, 16, 32], [8, 8, 8, 32, 4], [8, 8, 8, 64, 8], [8, 8, 8, 32, 16]]


@pytest.mark.parametrize("params", TILE_PARAMS)
def test_tile_parameters_do_not_change_results(params):
    g, u, v, w = _case((96, 48, 130), 16)
    plan = monc.Plan.from_grid(g, "f64")
    plan.params = params
    assert all(e == p for e, p in zip(plan.params[3:], params[3:]) if p), (plan.params, params)
    ref = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0)
    out = run_gpu(g, u, v, w, plan=plan)
    errs = field_errors(out, ref, u, v, w)
    assert max(errs[:3]) <= TOL64 and errs[3] <= p_tolerance(g), errs


# y tile widths 1 and 2 set spectral column blocks of 1 and 2 bins: with 1
# the FP32 x kernels move one bin per lane, from 2 on two bins per 16-byte
# access
@pytest.mark.parametrize("params", [[8, 8, 8, 16, 32], [8, 8, 8, 32, 8], [8, 8, 8, 64, 4], [8, 8, 1, 0, 0],
                                    [8, 8, 2, 0, 0]])
def test_tile_parameters_mixed(params):
    g, u, v, w = _case((96, 48, 130), 18)
    errs_default, _, _ = mixed_case(g, u, v, w)
    plan = monc.Plan.from_grid(g, "mixed")
    plan.params = params
    u32, v32, w32 = (a.astype(np.float32) for a in (u, v, w))
    ref = oracle.project(u32.astype(np.float64), v32.astype(np.float64), w32.astype(np.float64),
                         g.dx, g.dy, g.dz, g.rho0)
    out = run_gpu(g, u32, v32, w32, "mixed", plan=plan)
    errs = field_errors(out, ref, u32, v32, w32)
    assert max(errs) <= TOL_MIXED, (errs, errs_default)


@pytest.mark.parametrize("nz,lanes", [(12, 4), (16, 4), (20, 4), (24, 4), (28, 4), (32, 4), (40, 4), (48, 4),
                                      (64, 4), (130, 16)])
def test_mixed_tridiagonal_tiles_give_identical_bits(nz, lanes):
    # rows per lane 3, 4, 5, 6, 7, 8, 10, 12, 16 and 10 (130 levels on 16
    # lanes: 9 rounded up, the last lane's rows partly past the top). FP32
    # storage with an even number and tiles of 8 or more columns takes the
    # kernel instance that moves column pairs with 16-byte accesses, other
    # tiles the single-column one; each column's solve does not depend on
    # how columns are grouped into tiles or staged, so every tile width
    # gives the same bits. nx = 48: 25 spectral columns per row, so one pair
    # holds a padding column; ny = 9 leaves the last tile ragged.
    g, u, v, w = _case((48, 9, nz), 29)
    u32, v32, w32 = (a.astype(np.float32) for a in (u, v, w))
    ref = oracle.project(u32.astype(np.float64), v32.astype(np.float64), w32.astype(np.float64),
                         g.dx, g.dy, g.dz, g.rho0)
    outs = []
    for cw in (1, 4, 8, 16):
        print(f"case tridiagonal tiles nz={nz} lanes={lanes} cw={cw}", flush=True)
        plan = monc.Plan.from_grid(g, "mixed")
        plan.params = [0, 0, 0, lanes, cw, 0, 0]
        assert plan.params[3:5] == [lanes, cw], plan.params
        out = run_gpu(g, u32, v32, w32, "mixed", plan=plan)
        errs = field_errors(out, ref, u32, v32, w32)
        assert max(errs) <= TOL_MIXED, (cw, errs)
        outs.append(out)
        plan.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("params", [[8, 8, 8, 16, 3], [8, 8, 8, 32, 32], [8, 8, 8, 64, 16], [8, 8, 8, 3, 0]])
def test_plan_rejects_bad_tridiagonal_tiles(params):
    g, u, v, w = _case((32, 16, 130), 19)
    plan = monc.Plan.from_grid(g, "f64")
    before = plan.params
    with pytest.raises(monc.MoncError, match="tridiagonal"):
        plan.params = params
    assert plan.params == before


def test_autotune_keeps_results():
    g, u, v, w = _case((64, 48, 40), 20)
    plan = monc.Plan.from_grid(g, "f64")
    plan.autotune()
    prm = plan.params
    assert len(prm) == monc.NPARAMS and prm[3] * prm[4] <= 512, prm
    ref = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0)
    out = run_gpu(g, u, v, w, plan=plan)
    errs = field_errors(out, ref, u, v, w)
    assert max(errs[:3]) <= TOL64 and errs[3] <= p_tolerance(g), errs


def test_autotune_cache_round_trip(tmp_path, monkeypatch):
    # the tuned parameters land in the JSON file named by MONC_TUNE_CACHE and
    # a later plan of the same grid and dtype starts from them
    import json
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("MONC_TUNE_CACHE", str(cache))
    g, u, v, w = _case((48, 32, 24), 22)
    plan = monc.Plan.from_grid(g, "mixed")
    plan.autotune()
    tuned = plan.params
    data = json.loads(cache.read_text())
    key = f"gfx950:{g.nx},{g.ny},{g.nz}:mixed"
    assert key in data and len(data[key]) == monc.NPARAMS, data
    assert data[key][2:] == tuned[2:], (data[key], tuned)
    # a different value in the cache is picked up by a new plan
    other = list(data[key])
    other[3] = 8 if tuned[3] != 8 else 16
    other[4] = 0
    data[key] = other
    cache.write_text(json.dumps(data))
    plan2 = monc.Plan.from_grid(g, "mixed")
    assert plan2.params[3] == other[3], (plan2.params, other)
    errs, out, ref = mixed_case(g, u, v, w)
    assert max(errs) <= TOL_MIXED, errs


def test_profiler_counts_every_kernel_launch():
    g, u, v, w = _case((64, 32, 16), 23)
    for dtype, kernels in (("f64", {"div_fftx": 1, "ffty_fwd": 1, "tridiag": 1, "ffty_inv": 1, "ifftx": 1, "grad": 1}),
                           ("mixed", {"div_fftx": 1, "ffty_fwd": 2, "tridiag": 2, "ffty_inv": 2, "ifftx": 2,
                                      "resid_fftx": 1, "grad_final": 1})):
        plan = monc.Plan.from_grid(g, dtype)
        tdt = plan.torch_dtype
        f = [to_dev(x, tdt) for x in (u, v, w)] + [torch.empty((g.nz, g.ny, g.nx), dtype=tdt, device=DEV)]
        plan.profile_enable((1 << len(monc.KERNELS)) - 1)
        for _ in range(3):
            plan.project(*f)
        torch.cuda.synchronize()
        rec = plan.profile_read()
        plan.profile_enable(0)
        assert {k: n for k, (ms, n) in rec.items()} == {k: 3 * n for k, n in kernels.items()}, rec
        assert all(ms > 0 for ms, _ in rec.values()), rec
        assert plan.profile_read() == {}
