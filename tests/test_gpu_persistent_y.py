"""The persistent FP32 y-FFT (32 elements per thread, tile parameter
out[6] = 32): one workgroup per CU walks the level tiles and loads its next
tile while transforming the current one.

Its radix plan is the one the 16-elements-per-thread kernel takes for the
same length (radix-16 passes while they fit, then the remaining factors), its
twiddles are an LDS copy of the same table and every value goes through the
same butterflies, so its spectra and projections agree with that kernel's to
a few FP32 roundings (the compiler may contract a product and a sum into one
FMA in one kernel and not in the other: 1e-6 of the norm, against FP32's
6e-8 unit roundoff); the projection is also held to the mixed path's bound
against the FP64 oracle on the FP32 inputs. Shapes cover every length the
kernel is built for and tiles whose last columns lie past nx/2+1 (ragged). A
batch of members sharing one launch runs the same kernel on the same tiles as
the single calls, so it must equal them bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import relerr
from tests.tolerances import TOL_MIXED

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2009_12849_amd as monc  # noqa: E402

DEV = "cuda:0"

# (nx, ny, nz): ny selects the kernel instance (8, 16, 10 and 4 columns per
# tile); nx/2+1 = 19, 13, 28, 17 leaves the last tile partial
SHAPES = [(36, 2048, 3), (24, 1024, 5), (54, 1536, 4), (32, 4096, 2)]


def _fields(shape, seed):
    rng = np.random.default_rng(seed)
    g = synth.random_grid(rng, *shape, stretch=(1.0, 1.1))
    u, v, w = synth.random_fields(rng, g)
    return g, u.astype(np.float32), v.astype(np.float32), w.astype(np.float32)


def _plan(g, yept):
    plan = monc.Plan.from_grid(g, "mixed")
    plan.params = [0, 0, 0, 0, 0, 0, yept]
    assert plan.params[6] == yept
    return plan


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _project(plan, u, v, w):
    t = [_dev(a) for a in (u, v, w)]
    t.append(torch.empty_like(t[0]))
    plan.project(*t)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in t]


@pytest.mark.parametrize("shape", SHAPES)
def test_persistent_forward_spectrum_equals_radix16_kernel(shape):
    g, u, v, w = _fields(shape, 31)
    print(f"case persistent forward {shape}", flush=True)
    specs = []
    for yept in (16, 32):
        plan = _plan(g, yept)
        spec = plan.spectral_buffer()
        plan.debug_stage(monc.STAGE_FORWARD, [_dev(u), _dev(v), _dev(w), spec])
        torch.cuda.synchronize()
        specs.append(plan.spectral_get(spec).cpu().numpy())
        plan.close()
    assert relerr(specs[1], specs[0]) <= 1e-6
    ref = oracle.project(u.astype(np.float64), v.astype(np.float64), w.astype(np.float64),
                         g.dx, g.dy, g.dz, g.rho0, intermediates=True)
    assert relerr(specs[1].astype(np.complex128), ref["B"]) <= 1e-5


@pytest.mark.parametrize("shape", SHAPES)
def test_persistent_projection_equals_radix16_kernel(shape):
    g, u, v, w = _fields(shape, 32)
    print(f"case persistent projection {shape}", flush=True)
    outs = []
    for yept in (16, 32):
        plan = _plan(g, yept)
        outs.append(_project(plan, u, v, w))
        plan.close()
    for a, b in zip(outs[0], outs[1]):
        assert relerr(b.astype(np.float64), a.astype(np.float64)) <= 1e-6
    ref = oracle.project(u.astype(np.float64), v.astype(np.float64), w.astype(np.float64),
                         g.dx, g.dy, g.dz, g.rho0)
    vs = max(float(np.abs(x).max()) for x in (u, v, w))
    errs = [float(np.abs(outs[1][t].astype(np.float64) - ref[t]).max()) / vs for t in range(3)]
    errs.append(relerr(outs[1][3].astype(np.float64), ref[3]))
    print(f"persistent {shape} errors u, v, w, p: {errs}", flush=True)
    assert max(errs) <= TOL_MIXED, errs


def test_persistent_batch_equals_single_calls():
    # three members with ny = 2048 share each persistent launch (different
    # nx and nz: their tiles interleave over the workgroups)
    shapes = [(36, 2048, 3), (16, 2048, 5), (72, 2048, 2)]
    members = [_fields(s, 40 + i) for i, s in enumerate(shapes)]
    plans = [_plan(m[0], 32) for m in members]
    print("case persistent batch", flush=True)
    single = [_project(pl, *m[1:]) for pl, m in zip(plans, members)]
    fields = []
    for m in members:
        t = [_dev(a) for a in m[1:]]
        t.append(torch.empty_like(t[0]))
        fields.append(t)
    monc.project_batched(plans, *[[f[t] for f in fields] for t in range(4)])
    torch.cuda.synchronize()
    for s, f in zip(single, fields):
        for a, b in zip(s, f):
            assert np.array_equal(a, b.cpu().numpy())
    for pl in plans:
        pl.close()


def test_persistent_kernel_rejected_where_it_does_not_exist():
    rng = np.random.default_rng(5)
    g64 = synth.random_grid(rng, 16, 2048, 3, stretch=(1.0, 1.1))
    plan = monc.Plan.from_grid(g64, "f64")
    with pytest.raises(monc.MoncError, match="persistent"):
        plan.params = [0, 0, 0, 0, 0, 0, 32]
    plan.close()
    g = synth.random_grid(rng, 16, 512, 3, stretch=(1.0, 1.1))
    plan = monc.Plan.from_grid(g, "mixed")
    with pytest.raises(monc.MoncError, match="persistent"):
        plan.params = [0, 0, 0, 0, 0, 0, 32]
    plan.close()


def test_persistent_kernel_in_the_variable_density_preconditioner():
    # the Krylov solve runs the plan's spectral solve as its preconditioner,
    # in batches of iterations whose launches return at once (a skip flag in
    # the descriptor) after convergence: with the persistent kernel the
    # solve converges in the same iterations, and the answers of the two
    # preconditioners meet the same residual, so they agree to about the
    # tolerance times the operator's condition. The grid keeps that condition
    # near 4e5 (dx = dy = 25 m over 1024 rows, dz ~ 20 m), where FP32
    # transforms still make a useful preconditioner (their rounding, amplified
    # by the lowest mode, stays well below 1)
    rng = np.random.default_rng(61)
    g = synth.Grid(16, 1024, 6, 25.0, 25.0, 20.0 * rng.uniform(0.9, 1.1, 6), rng.uniform(0.8, 1.2, 6))
    rho = synth.density_field(rng, g, 0.2)
    u, v, w = synth.random_fields(rng, g)
    tol = 1e-10
    outs, its = [], []
    print("case persistent preconditioner (16, 1024, 6)", flush=True)
    for yept in (16, 32):
        plan = monc.Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, rho.mean(axis=(1, 2)), "mixed")
        plan.params = [0, 0, 0, 0, 0, 0, yept]
        t = [torch.from_numpy(np.ascontiguousarray(a)).to(DEV, torch.float64) for a in (rho, u, v, w)]
        p = torch.empty_like(t[1])
        it, rel = plan.project_var(t[0], t[1], t[2], t[3], p, tol=tol)
        torch.cuda.synchronize()
        assert rel <= tol, (yept, it, rel)
        its.append(it)
        outs.append([x.cpu().numpy() for x in t[1:] + [p]])
        plan.close()
    assert abs(its[0] - its[1]) <= 1, its
    for a, b in zip(outs[0], outs[1]):
        assert relerr(b, a) <= 4e5 * tol
