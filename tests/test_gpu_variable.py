"""Variable-density projection (monc_project_var): conjugate gradients with
the plan's spectral solve as the preconditioner, against the oracle's direct
sparse solve of the same discrete problem (oracle.project_var), and against
properties that hold at any size.

Tolerances. The solver stops at a relative residual tol = 1e-12 (dz-weighted
2-norms). The outputs' own divergence D_rho(u) is that residual up to the
rounding of the FP64 recurrences, so it is held to 100 tol. The pressure error
e solves D_rho(G e) = residual, so |e| <= cond * tol * |p|; the condition of
these small operators (stretched dz, density contrast 1.3/0.7) stays below
1e3, which bounds p to 1e-8 relative and u, v, w (G e, one difference of e)
to 1e-9 of the input scale with room to spare."""
import numpy as np
import pytest

import oracle
import synth
from tests.tolerances import TOL64

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2009_12849_amd as monc  # noqa: E402

DEV = "cuda:0"
TOL = 1e-12
# odd nx (27, 81) takes the one-point operator kernel with real x neighbours;
# nx = 384 leaves a partial 256-point x tile in every stencil kernel
SHAPES = [(32, 32, 16), (48, 27, 13), (24, 18, 9), (4, 4, 1), (1, 6, 5), (1, 1, 4), (27, 9, 6), (81, 6, 4),
          (384, 4, 3)]


def _case(shape, seed, amp=0.3):
    rng = np.random.default_rng(seed)
    g = synth.random_grid(rng, *shape, stretch=(1.0, min(1.1, 20.0 ** (1.0 / max(shape[2], 1)))))
    rho = synth.density_field(rng, g, amp)
    u, v, w = synth.random_fields(rng, g)
    return g, rho, u, v, w


def _plan(g, rho, dtype):
    """Plan whose reference density is the horizontal mean of rho."""
    return monc.Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, rho.mean(axis=(1, 2)), dtype)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, torch.float64)


def _wnorm(x, dz):
    return np.sqrt(np.sum(np.asarray(dz)[:, None, None] * x * x))


def _cond_estimate(nx, ny, dx, dy, dz, contrast=1.5):
    """Condition number of D_rho G estimated from the grid: largest
    eigenvalue 4/dx^2 + 4/dy^2 + 4/(min dz min dzc), smallest that of the
    longest horizontal or vertical mode, times the density contrast. Two
    solutions that meet a relative residual tol differ by at most about
    tol times this, relative to the solution."""
    dz = np.asarray(dz, dtype=np.float64)
    dzc = 0.5 * (dz[:-1] + dz[1:]) if dz.size > 1 else dz
    lmax = 4 / dx ** 2 + 4 / dy ** 2 + 4 / (dz.min() * dzc.min())
    modes = [(np.pi / dz.sum()) ** 2]
    if nx > 1:
        modes.append((2 * np.pi / (nx * dx)) ** 2)
    if ny > 1:
        modes.append((2 * np.pi / (ny * dy)) ** 2)
    return contrast * lmax / min(modes)


def _run(g, rho, u, v, w, dtype, tol=TOL, maxit=200):
    plan = _plan(g, rho, dtype)
    t = [_t(a) for a in (u, v, w)]
    p = torch.empty_like(t[0])
    it, rel = plan.project_var(_t(rho), *t, p, tol=tol, maxit=maxit)
    torch.cuda.synchronize()
    plan.close()
    return [x.cpu().numpy() for x in t + [p]], it, rel


@pytest.mark.parametrize("dtype", ["f64", "mixed"])
@pytest.mark.parametrize("shape", SHAPES)
def test_variable_density_matches_direct_solve(shape, dtype):
    print(f"case {shape} {dtype}", flush=True)
    g, rho, u, v, w = _case(shape, 1200 + sum(shape))
    outs, it, rel = _run(g, rho, u, v, w, dtype)
    print(f"  iterations {it}, relative residual {rel:.3e}", flush=True)
    assert rel <= TOL and it < 200
    # the outputs' own divergence, recomputed by the oracle
    b = oracle.divergence_var(u, v, w, g.dx, g.dy, g.dz, rho)
    res = oracle.divergence_var(*outs[:3], g.dx, g.dy, g.dz, rho)
    nb = _wnorm(b, g.dz)
    if nb > 0:
        assert _wnorm(res, g.dz) <= 100 * TOL * nb, _wnorm(res, g.dz) / nb
    assert np.all(outs[2][-1] == 0.0)
    # gauge: sum_k dz_k sum_ij p = 0 up to rounding
    dz = np.asarray(g.dz)
    pw = np.abs(outs[3]).max() * np.sum(dz) * g.nx * g.ny
    assert abs(np.sum(dz[:, None, None] * outs[3])) <= 1e-12 * max(pw, 1e-300)
    # the direct solve
    ref = oracle.project_var(u, v, w, g.dx, g.dy, g.dz, rho)
    scale = max(np.abs(a).max() for a in (u, v, w))
    for f in range(3):
        err = np.abs(outs[f] - ref[f]).max()
        assert err <= 1e-9 * scale, (f, err / scale)
    perr = np.abs(outs[3] - ref[3]).max()
    assert perr <= 1e-8 * max(np.abs(ref[3]).max(), 1e-300), perr / np.abs(ref[3]).max()


def test_separable_density_is_one_spectral_solve():
    """rho = rho0(z): the preconditioner is the exact inverse, CG stops after
    one iteration (two at most, from rounding) with monc_project's answer."""
    rng = np.random.default_rng(77)
    g = synth.random_grid(rng, 32, 24, 12, stretch=(1.0, 1.1))
    u, v, w = synth.random_fields(rng, g)
    rho = np.broadcast_to(np.asarray(g.rho0)[:, None, None], (g.nz, g.ny, g.nx)).copy()
    outs, it, rel = _run(g, rho, u, v, w, "f64")
    assert it <= 2 and rel <= TOL
    plan = monc.Plan.from_grid(g, "f64")
    t = [_t(a) for a in (u, v, w)]
    p = torch.empty_like(t[0])
    plan.project(*t, p)
    torch.cuda.synchronize()
    plan.close()
    scale = max(np.abs(a).max() for a in (u, v, w))
    for f in range(3):
        assert np.abs(outs[f] - t[f].cpu().numpy()).max() <= TOL64 * scale
    assert np.abs(outs[3] - p.cpu().numpy()).max() <= 1e-9 * np.abs(outs[3]).max()


def test_divergence_free_input_takes_no_iteration():
    g = synth.random_grid(np.random.default_rng(3), 16, 16, 6)
    rho = synth.density_field(np.random.default_rng(4), g, 0.2)
    z = np.zeros((g.nz, g.ny, g.nx))
    outs, it, rel = _run(g, rho, z, z, z, "f64")
    assert it == 0 and rel == 0.0
    assert all(np.all(o == 0.0) for o in outs)


def test_iteration_cap_is_reported():
    g, rho, u, v, w = _case((32, 32, 16), 5)
    outs, it, rel = _run(g, rho, u, v, w, "f64", tol=0.0, maxit=3)
    assert it == 3 and 0.0 < rel < 1.0


def test_bad_arguments_are_rejected():
    g, rho, u, v, w = _case((16, 16, 4), 6)
    plan = _plan(g, rho, "f64")
    f = [_t(a) for a in (rho, u, v, w, np.zeros_like(u))]
    with pytest.raises(monc.MoncError):
        plan.project_var(*f, tol=-1.0)
    with pytest.raises(monc.MoncError):
        plan.project_var(*f, maxit=0)
    with pytest.raises(ValueError):
        plan.project_var(f[0].float(), *f[1:])
    with pytest.raises(monc.MoncError):      # p aliases u
        plan.project_var(f[0], f[1], f[2], f[3], f[1])
    plan.close()


@pytest.mark.parametrize("name", ["256x256x128", "1024x1024x256"])
def test_full_size_variable_density(name):
    """The benchmark's grid, fields and density (rho0(z)(1 + 0.2 f), seed
    6100) with both preconditioners, as bench.py runs them: the direct
    solve is out of reach at 8.4e6 and 2.7e8 unknowns, so the checks are the ones that
    hold at any size: the outputs' own divergence recomputed by the oracle,
    the gauge, the lid, and the two preconditioners agreeing with each other
    (both stop at the same FP64 residual)."""
    wl = synth.make_workload(name)
    m = wl.members[0]
    g = m.grid
    rho = synth.density_field(np.random.default_rng(6100), g, 0.2)
    u, v, w = (a.astype(np.float64) for a in (m.u, m.v, m.w))
    b = oracle.divergence_var(u, v, w, g.dx, g.dy, g.dz, rho)
    nb = _wnorm(b, g.dz)
    dz = np.asarray(g.dz)
    outs = {}
    for dtype in ("f64", "mixed"):
        print(f"case {name} {dtype}", flush=True)
        o, it, rel = _run(g, rho, u, v, w, dtype, tol=1e-10, maxit=500)
        print(f"  iterations {it}, relative residual {rel:.3e}", flush=True)
        assert rel <= 1e-10 and it < 500
        res = oracle.divergence_var(*o[:3], g.dx, g.dy, g.dz, rho)
        assert _wnorm(res, g.dz) <= 1e-8 * nb, _wnorm(res, g.dz) / nb
        assert np.all(o[2][-1] == 0.0)
        pw = np.abs(o[3]).max() * np.sum(dz) * g.nx * g.ny
        assert abs(np.sum(dz[:, None, None] * o[3])) <= 1e-12 * pw
        outs[dtype] = o
    # Both stop at relative residual 1e-10. A tighter FP64 solve (1e-12)
    # serves as the reference: the FP64-preconditioned answer's distance from
    # it measures the error a 1e-10 stop leaves on this input, and the FP32-
    # preconditioned answer must lie within a small multiple of that.
    o, it, rel = _run(g, rho, u, v, w, "f64", tol=1e-12, maxit=500)
    print(f"  tight FP64 reference: iterations {it}, relative residual {rel:.3e}", flush=True)
    assert rel <= 1e-11
    scale = max(np.abs(a).max() for a in (u, v, w))
    pref = np.abs(o[3]).max()
    dist = {}
    for dtype in ("f64", "mixed"):
        du = max(np.abs(outs[dtype][f] - o[f]).max() for f in range(3)) / scale
        dp = np.abs(outs[dtype][3] - o[3]).max() / pref
        dist[dtype] = (du, dp)
    print(f"  distance from the tight solve (u, v, w; p): FP64 preconditioner {dist['f64']}, "
          f"FP32 preconditioner {dist['mixed']}", flush=True)
    for i in range(2):
        assert dist["mixed"][i] <= 10.0 * dist["f64"][i] + 1e-13, dist


@pytest.mark.parametrize("dtype", ["f64", "mixed"])
@pytest.mark.parametrize("shape", [(48, 1, 1), (96, 8, 5)])
def test_x_only_density_closed_form(shape, dtype):
    """rho and u* of x alone: u = C / rx (harmonic-mean flux) and p in
    closed form (see tests/test_oracle_pins.py, _x_only_case)."""
    from tests.test_oracle_pins import _x_only_case
    dx, dy, dz, rho, u, z, uo, po = _x_only_case(*shape, seed=36)
    nz, ny, nx = rho.shape
    plan = monc.Plan(nx, ny, nz, dx, dy, dz, rho.mean(axis=(1, 2)), dtype)
    t = [_t(a) for a in (u, z, z)]
    p = torch.empty_like(t[0])
    it, rel = plan.project_var(_t(rho), *t, p, tol=TOL, maxit=200)
    torch.cuda.synchronize()
    plan.close()
    outs = [x.cpu().numpy() for x in t + [p]]
    assert rel <= TOL
    # within TOL times the condition estimate (density contrast 1.5/0.5);
    # v and w are zero up to that and the rounding of the transforms of row-
    # and level-constant fields
    bound = max(TOL * _cond_estimate(nx, ny, dx, dy, dz, contrast=3.0), 1e-12)
    print(f"  bound {bound:.1e}: u {np.abs(outs[0] - uo).max() / np.abs(uo).max():.1e}, "
          f"v {np.abs(outs[1]).max() / np.abs(uo).max():.1e}, w {np.abs(outs[2]).max() / np.abs(uo).max():.1e}, "
          f"p {np.abs(outs[3] - po).max() / np.abs(po).max():.1e}", flush=True)
    assert np.abs(outs[0] - uo).max() <= bound * np.abs(uo).max()
    assert np.abs(outs[1]).max() <= bound * np.abs(uo).max()
    assert np.abs(outs[2]).max() <= bound * np.abs(uo).max()
    assert np.abs(outs[3] - po).max() <= bound * np.abs(po).max()


@pytest.mark.parametrize("dtype", ["f64", "mixed"])
def test_strong_contrast_matches_direct_solve(dtype):
    """Density varying by +-60 %: more iterations, the same answer."""
    shape = (32, 24, 12)
    g, rho, u, v, w = _case(shape, 1300, amp=0.6)
    outs, it, rel = _run(g, rho, u, v, w, dtype)
    print(f"  iterations {it}, relative residual {rel:.3e}", flush=True)
    assert rel <= TOL and it < 200
    ref = oracle.project_var(u, v, w, g.dx, g.dy, g.dz, rho)
    scale = max(np.abs(a).max() for a in (u, v, w))
    bound = TOL * _cond_estimate(g.nx, g.ny, g.dx, g.dy, g.dz, contrast=1.6 / 0.4)
    for f in range(3):
        assert np.abs(outs[f] - ref[f]).max() <= bound * scale, f
    assert np.abs(outs[3] - ref[3]).max() <= bound * np.abs(ref[3]).max()


@pytest.mark.parametrize("dtype", ["f64", "mixed"])
def test_solve_is_deterministic(dtype):
    """The inner products add per-workgroup partials in a fixed order (no
    atomics): two solves of the same input on one plan are bitwise equal."""
    g, rho, u, v, w = _case((64, 48, 20), 1400)
    plan = _plan(g, rho, dtype)
    r = _t(rho)
    res = []
    for _ in range(2):
        t = [_t(a) for a in (u, v, w)]
        p = torch.empty_like(t[0])
        it, rel = plan.project_var(r, *t, p, tol=TOL, maxit=200)
        torch.cuda.synchronize()
        res.append(([x.cpu().numpy() for x in t + [p]], it, rel))
    plan.close()
    (o0, i0, r0), (o1, i1, r1) = res
    assert i0 == i1 and r0 == r1
    for a, b in zip(o0, o1):
        assert np.array_equal(a, b)


def test_non_finite_input_is_reported():
    g, rho, u, v, w = _case((16, 16, 4), 7)
    u = u.copy()
    u[1, 2, 3] = np.nan
    plan = _plan(g, rho, "f64")
    f = [_t(a) for a in (rho, u, v, w, np.zeros_like(u))]
    with pytest.raises(monc.MoncError, match="not finite"):
        plan.project_var(*f)
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "mixed"])
def test_plan_density_far_from_rho(dtype):
    """A plan whose rho0 is not the level mean of rho (here uniform 1 while
    rho decays with height and varies by +-30 %): the scaling S = sqrt(rho0 /
    rho) absorbs the mismatch, the solve converges to the same answer."""
    g, rho, u, v, w = _case((32, 24, 12), 1500)
    plan = monc.Plan(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, np.ones(g.nz), dtype)
    t = [_t(a) for a in (u, v, w)]
    p = torch.empty_like(t[0])
    it, rel = plan.project_var(_t(rho), *t, p, tol=TOL, maxit=400)
    torch.cuda.synchronize()
    plan.close()
    print(f"  iterations {it}, relative residual {rel:.3e}", flush=True)
    assert rel <= TOL and it < 400
    outs = [x.cpu().numpy() for x in t + [p]]
    ref = oracle.project_var(u, v, w, g.dx, g.dy, g.dz, rho)
    scale = max(np.abs(a).max() for a in (u, v, w))
    bound = TOL * _cond_estimate(g.nx, g.ny, g.dx, g.dy, g.dz, contrast=1.3 / 0.7)
    for f in range(3):
        assert np.abs(outs[f] - ref[f]).max() <= bound * scale, f
    assert np.abs(outs[3] - ref[3]).max() <= bound * np.abs(ref[3]).max()


def test_side_stream_and_retuned_plan():
    """The solve on a non-default stream (its kernels and its status reads
    follow the caller's stream) gives bitwise the default stream's answer;
    after the plan's tiles change (autotune, or explicit parameters) the
    preconditioner's descriptor follows them and the answer is the same to
    the solver tolerance."""
    g, rho, u, v, w = _case((64, 48, 20), 1600)
    plan = _plan(g, rho, "f64")
    r = _t(rho)

    def solve(stream=None):
        t = [_t(a) for a in (u, v, w)]
        p = torch.empty_like(t[0])
        if stream is None:
            it, rel = plan.project_var(r, *t, p, tol=TOL)
        else:
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                it, rel = plan.project_var(r, *t, p, tol=TOL, stream=stream)
            stream.synchronize()
        torch.cuda.synchronize()
        return [x.cpu().numpy() for x in t + [p]], it, rel

    ref, it0, _ = solve()
    side, it1, _ = solve(torch.cuda.Stream())
    assert it0 == it1
    for a, b in zip(ref, side):
        assert np.array_equal(a, b)
    params = plan.params
    alt = list(params)
    alt[3] = 8 if params[3] != 8 else 16        # tridiagonal lanes per column
    alt[4] = 0                                  # columns per workgroup: automatic
    plan.params = alt
    assert plan.params[3] == alt[3]
    out, it2, rel2 = solve()
    plan.close()
    assert rel2 <= TOL
    scale = max(np.abs(a).max() for a in (u, v, w))
    bound = TOL * _cond_estimate(g.nx, g.ny, g.dx, g.dy, g.dz, contrast=1.3 / 0.7)
    for f in range(3):
        assert np.abs(out[f] - ref[f]).max() <= bound * scale
    assert np.abs(out[3] - ref[3]).max() <= bound * np.abs(ref[3]).max()


@pytest.mark.parametrize("dtype", ["f64", "mixed"])
def test_long_domain_converges_like_a_square_one(dtype):
    """A domain 16 cells wide and 1024 long (dy = 57 m): its lowest mode is
    far below the density's horizontal scales. The preconditioned condition
    number is still bounded by the face-density contrast, so the solve takes
    as many iterations as on square grids (a symmetric density scaling of the
    preconditioner lost that bound here and stagnated near 2e-4). Checked
    against the oracle's direct solve: velocities to 1e-9 of the input scale,
    p to the tolerance times the operator's condition estimate."""
    rng = np.random.default_rng(61)
    g = synth.random_grid(rng, 16, 1024, 6, stretch=(1.0, 1.1), dx=11.1, dy=56.8)
    rho = synth.density_field(rng, g, 0.3)
    u, v, w = synth.random_fields(rng, g)
    print(f"case long domain {dtype}", flush=True)
    outs, it, rel = _run(g, rho, u, v, w, dtype)
    print(f"  iterations {it}, relative residual {rel:.3e}", flush=True)
    assert rel <= TOL and it <= 30, (it, rel)
    ref = oracle.project_var(u, v, w, g.dx, g.dy, g.dz, rho)
    scale = max(np.abs(a).max() for a in (u, v, w))
    for f in range(3):
        assert np.abs(outs[f] - ref[f]).max() <= 1e-9 * scale, f
    cond = _cond_estimate(g.nx, g.ny, g.dx, g.dy, g.dz, contrast=1.3 / 0.7)
    pmax = np.abs(ref[3]).max()
    assert np.abs(outs[3] - ref[3]).max() <= 10 * cond * TOL * pmax, (np.abs(outs[3] - ref[3]).max() / pmax, cond)
