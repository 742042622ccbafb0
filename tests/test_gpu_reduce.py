"""Per-level horizontal reductions folded into the projection
(monc_project_reduce): against their definition (oracle.level_stats) applied
to the projection's own outputs, and against the oracle's projection.

Grids cover both ways the gradient kernel reduces: workgroups whose points lie
in one level (256^2 levels) and workgroups that span levels (small or ragged
grids, down to one point per level)."""
import numpy as np
import pytest

import oracle
import synth
from tests.tolerances import TOL64, TOL_MIXED, p_tolerance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2009_12849_amd as monc  # noqa: E402

DEV = "cuda:0"
SHAPES = [(32, 32, 32), (48, 27, 13), (256, 256, 16), (64, 64, 130), (1, 1, 4), (96, 72, 33)]
EPS64 = 2.0 ** -53


def _run(g, u, v, w, dtype, with_stats):
    plan = monc.Plan.from_grid(g, dtype)
    tdt = plan.torch_dtype
    t = [torch.from_numpy(np.ascontiguousarray(a)).to(DEV, tdt) for a in (u, v, w)]
    p = torch.empty_like(t[0])
    st = torch.full((8 * g.nz,), float("nan"), dtype=torch.float64, device=DEV) if with_stats else None
    plan.project(*t, p, stats=st)
    torch.cuda.synchronize()
    outs = [x.cpu().numpy().astype(np.float64) for x in t + [p]]
    plan.close()
    return outs, (st.cpu().numpy().reshape(4, 2, g.nz) if with_stats else None)


@pytest.mark.parametrize("dtype", ["f64", "mixed"])
@pytest.mark.parametrize("shape", SHAPES)
def test_reductions_match_definition_and_oracle(shape, dtype):
    print(f"case {shape} {dtype}", flush=True)
    rng = np.random.default_rng(900 + sum(shape))
    # dz grows by at most a factor 20 over the column, as in the parity tests
    g = synth.random_grid(rng, *shape, stretch=(1.0, min(1.1, 20.0 ** (1.0 / max(shape[2], 1)))))
    u, v, w = synth.random_fields(rng, g)
    if dtype == "mixed":
        u, v, w = (a.astype(np.float32) for a in (u, v, w))
    outs, st = _run(g, u, v, w, dtype, True)
    plain, _ = _run(g, u, v, w, dtype, False)
    for a, b in zip(outs, plain):          # the reductions leave the fields alone
        assert np.array_equal(a, b)
    assert np.all(np.isfinite(st))

    # 1. the definition on the GPU's own outputs: maxima exact, means within
    #    the summation bound (nx ny terms in another order)
    nh = g.nx * g.ny
    mine = oracle.level_stats(*outs)
    for f in range(4):
        bound = nh * EPS64 * np.abs(outs[f]).max() + 1e-300
        if f == 3 and dtype == "mixed":
            # p1 + delta in FP64 against its stored FP32 rounding
            bound += 2.0 ** -24 * np.abs(outs[3]).max()
            assert np.max(np.abs(st[f, 1] - mine[f, 1])) <= bound, f
        else:
            assert np.array_equal(st[f, 1], mine[f, 1]), f
        assert np.max(np.abs(st[f, 0] - mine[f, 0])) <= bound, (f, np.max(np.abs(st[f, 0] - mine[f, 0])), bound)

    # 2. the oracle's projection of the same (rounded) inputs
    ins = [a.astype(np.float64) for a in (u, v, w)]
    ref = oracle.project(*ins, g.dx, g.dy, g.dz, g.rho0)
    want = oracle.level_stats(*ref)
    scale = max(np.abs(a).max() for a in ins)
    pscale = np.abs(ref[3]).max()
    tol_uvw = (TOL64 if dtype == "f64" else TOL_MIXED) * scale
    tol_p = (p_tolerance(g) if dtype == "f64" else TOL_MIXED) * pscale
    for f in range(4):
        tol = tol_p if f == 3 else tol_uvw
        assert np.max(np.abs(st[f] - want[f])) <= tol, (f, np.max(np.abs(st[f] - want[f])), tol)
    # the lid row of w is zero, so is its level's mean and max
    assert st[2, 0, -1] == 0.0 and st[2, 1, -1] == 0.0


def test_reductions_reject_bad_buffer():
    g = synth.random_grid(np.random.default_rng(5), 16, 16, 8)
    plan = monc.Plan.from_grid(g, "f64")
    f = [torch.zeros((8, 16, 16), dtype=torch.float64, device=DEV) for _ in range(4)]
    with pytest.raises(ValueError):
        plan.project(*f, stats=torch.zeros(8 * 8 - 1, dtype=torch.float64, device=DEV))
    with pytest.raises(ValueError):
        plan.project(*f, stats=torch.zeros(8 * 8, dtype=torch.float32, device=DEV))
    plan.close()
