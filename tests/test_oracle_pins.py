"""Pins of the FP64 oracle against things other than itself.

The paper (Sec. 4) says only that the pressure solve is a forward horizontal
FFT, a vertical ODE per wavenumber and a backward FFT; it prints no equation,
worked example or value. The oracle is therefore pinned against:

  P-brute  dense matrices of D and G assembled cell by cell from the
           C-grid definitions (code separate from the spectral oracle) and a
           dense gauge-constrained solve, on tiny grids;
  P-DCT    uniform dz and constant rho0: the operator is diagonalised by
           DFT x DFT x DCT-II, solved with scipy's dct;
  P-mfg    manufactured solutions (known p plus a discretely divergence-free
           part built from a streamfunction);
  P-inv    invariants (divergence-free output, gauge, per-level means, energy
           identity, idempotence, linearity, lid);
  P-conv   second-order convergence to a continuum closed form;
  P-2D     nz = 1 reduces to the textbook periodic Poisson solve;
  P-col    nx = ny = 1 reduces to a cumulative sum in z (plus a hand-derived
           golden fixture).
"""
import os

import numpy as np
import pytest
import scipy.fft as sfft

import oracle
import oracle.projection as op
import synth
from tests.helpers import relerr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# Dense assembly from the definitions (independent of oracle/)
# ----------------------------------------------------------------------------
def _face_density(dz, rho0):
    # rho0 on the face between cells k and k+1, linear in z: the weights are
    # the distances to the two centres, dz_{k+1}/2 and dz_k/2.
    return (dz[1:] * rho0[:-1] + dz[:-1] * rho0[1:]) / (dz[:-1] + dz[1:])


def dense_operators(g):
    nx, ny, nz = g.nx, g.ny, g.nz
    N = nx * ny * nz
    cell = lambda k, j, i: (k * ny + (j % ny)) * nx + (i % nx)
    rw = _face_density(g.dz, g.rho0)
    dzc = 0.5 * (g.dz[:-1] + g.dz[1:])
    D = np.zeros((N, 3 * N))
    G = np.zeros((3 * N, N))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = cell(k, j, i)
                D[r, cell(k, j, i)] += g.rho0[k] / g.dx
                D[r, cell(k, j, i - 1)] -= g.rho0[k] / g.dx
                D[r, N + cell(k, j, i)] += g.rho0[k] / g.dy
                D[r, N + cell(k, j - 1, i)] -= g.rho0[k] / g.dy
                if k <= nz - 2:
                    D[r, 2 * N + cell(k, j, i)] += rw[k] / g.dz[k]
                if k >= 1:
                    D[r, 2 * N + cell(k - 1, j, i)] -= rw[k - 1] / g.dz[k]
                G[cell(k, j, i), cell(k, j, i + 1)] += 1.0 / g.dx
                G[cell(k, j, i), cell(k, j, i)] -= 1.0 / g.dx
                G[N + cell(k, j, i), cell(k, j + 1, i)] += 1.0 / g.dy
                G[N + cell(k, j, i), cell(k, j, i)] -= 1.0 / g.dy
                if k <= nz - 2:
                    G[2 * N + cell(k, j, i), cell(k + 1, j, i)] += 1.0 / dzc[k]
                    G[2 * N + cell(k, j, i), cell(k, j, i)] -= 1.0 / dzc[k]
    return D, G


def dense_project(g, u, v, w):
    """Gauge-constrained dense solve: [L 1; g^T 0][p; mu] = [b; 0] with
    L = D G and g the cell volumes dz_k (so sum dz p = 0)."""
    N = g.points
    D, G = dense_operators(g)
    L = D @ G
    ustar = np.concatenate([u.ravel(), v.ravel(), w.ravel()])
    b = D @ ustar
    vol = np.repeat(g.dz, g.nx * g.ny)
    K = np.zeros((N + 1, N + 1))
    K[:N, :N] = L
    K[:N, N] = 1.0
    K[N, :N] = vol
    sol = np.linalg.solve(K, np.concatenate([b, [0.0]]))
    p = sol[:N]
    uo = ustar - G @ p
    shp = (g.nz, g.ny, g.nx)
    wo = uo[2 * N:].reshape(shp).copy()
    wo[-1] = 0.0
    return uo[:N].reshape(shp), uo[N:2 * N].reshape(shp), wo, p.reshape(shp), b.reshape(shp)


BRUTE_GRIDS = [(4, 4, 3), (5, 3, 4), (6, 4, 5), (8, 8, 6), (1, 1, 4), (4, 4, 1),
               (3, 2, 2), (9, 6, 3), (2, 3, 5)]


def brute_error(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    g = synth.random_grid(rng, nx, ny, nz, stretch=(1.0, 1.3))
    u, v, w = synth.random_fields(rng, g)
    ref = dense_project(g, u, v, w)
    out = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0)
    # velocities relative to the input scale (an output field can be ~0, e.g.
    # w on a single column); p relative to itself
    vscale = max(np.max(np.abs(u)), np.max(np.abs(v)), np.max(np.abs(w)))
    errs = [np.max(np.abs(out[t] - ref[t])) / vscale for t in range(3)]
    return max(errs + [relerr(out[3], ref[3])])


@pytest.mark.parametrize("shape", BRUTE_GRIDS)
def test_brute_force_dense_solve(shape):
    assert brute_error(*shape, seed=sum(shape)) <= 1e-12


def test_brute_force_divergence_matches_dense():
    rng = np.random.default_rng(7)
    g = synth.random_grid(rng, 5, 4, 6)
    u, v, w = synth.random_fields(rng, g)
    D, _ = dense_operators(g)
    b_ref = (D @ np.concatenate([u.ravel(), v.ravel(), w.ravel()])).reshape(u.shape)
    assert relerr(oracle.divergence(u, v, w, g.dx, g.dy, g.dz, g.rho0), b_ref) <= 1e-14


# ----------------------------------------------------------------------------
# Library closed form: uniform dz, constant rho0 -> DFT x DFT x DCT-II
# ----------------------------------------------------------------------------
def dct_solve(b, dx, dy, dz, rho):
    nz, ny, nx = b.shape
    m = np.arange(nx // 2 + 1)
    n = np.arange(ny)
    q = np.arange(nz)
    ev = ((4 / dx ** 2) * np.sin(np.pi * m / nx) ** 2)[None, None, :] \
        + ((4 / dy ** 2) * np.sin(np.pi * n / ny) ** 2)[None, :, None] \
        + ((4 / dz ** 2) * np.sin(np.pi * q / (2 * nz)) ** 2)[:, None, None]
    spec = sfft.dct(np.fft.rfft2(b, axes=(1, 2)), type=2, axis=0, norm="ortho")
    ev[0, 0, 0] = 1.0
    spec = -spec / (rho * ev)
    spec[0, 0, 0] = 0.0
    return np.fft.irfft2(sfft.idct(spec, type=2, axis=0, norm="ortho"), s=(ny, nx), axes=(1, 2))


def test_dct_closed_form_at_32x32x32():
    wl = synth.make_workload("32x32x32")
    m = wl.members[0]
    g = m.grid
    out = oracle.project(m.u, m.v, m.w, g.dx, g.dy, g.dz, g.rho0, intermediates=True)
    p_ref = dct_solve(out["b"], g.dx, g.dy, 20.0, 1.0)
    assert relerr(out["p"], p_ref) <= 1e-12


def test_dct_closed_form_constant_rho():
    rng = np.random.default_rng(11)
    g = synth.Grid(12, 18, 10, 30.0, 45.0, np.full(10, 7.0), np.full(10, 1.7))
    u, v, w = synth.random_fields(rng, g)
    out = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0, intermediates=True)
    assert relerr(out["p"], dct_solve(out["b"], g.dx, g.dy, 7.0, 1.7)) <= 1e-12


# ----------------------------------------------------------------------------
# Manufactured solutions
# ----------------------------------------------------------------------------
def manufactured(g, m0, n0, seed, mean_mode=False):
    rng = np.random.default_rng(seed)
    zw = np.concatenate([[0.0], np.cumsum(g.dz)])
    zc = 0.5 * (zw[:-1] + zw[1:])
    H = zw[-1]
    prof = np.cos(2.3 * zc / H) + 0.4 * (zc / H) ** 2 - 0.1
    if mean_mode:
        prof = prof - np.sum(g.dz * prof) / H
        p_true = np.broadcast_to(prof[:, None, None], (g.nz, g.ny, g.nx)).copy()
    else:
        cx = np.cos(2 * np.pi * m0 * (np.arange(g.nx) + 0.5) / g.nx)
        cy = np.cos(2 * np.pi * n0 * (np.arange(g.ny) + 0.5) / g.ny)
        p_true = prof[:, None, None] * np.outer(cy, cx)[None]
    dzc = zc[1:] - zc[:-1]
    gx = (np.roll(p_true, -1, 2) - p_true) / g.dx
    gy = (np.roll(p_true, -1, 1) - p_true) / g.dy
    gz = np.zeros_like(p_true)
    gz[:-1] = np.diff(p_true, axis=0) / dzc[:, None, None]
    psi = rng.standard_normal((g.nz, g.ny, g.nx))        # at cell corners
    us = (psi - np.roll(psi, 1, 1)) / g.dy
    vs = -(psi - np.roll(psi, 1, 2)) / g.dx
    return p_true, us, vs, gx + us, gy + vs, gz


@pytest.mark.parametrize("m0,n0", [(1, 0), (3, 2), (0, 5)])
def test_manufactured_stretched_vertical_grid(m0, n0):
    base = synth.make_grid("256x256x128")
    g = synth.Grid(32, 24, base.nz, 40.0, 30.0, base.dz, base.rho0)
    p_true, us, vs, u, v, w = manufactured(g, m0, n0, seed=m0 * 10 + n0)
    uo, vo, wo, p = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0)
    assert relerr(p, p_true) <= 1e-12
    assert relerr(uo, us) <= 1e-12 and relerr(vo, vs) <= 1e-12
    assert np.max(np.abs(wo)) <= 1e-12 * np.max(np.abs(w))


def test_manufactured_mean_mode():
    base = synth.make_grid("256x256x128")
    g = synth.Grid(16, 16, base.nz, 25.0, 25.0, base.dz, base.rho0)
    p_true, us, vs, u, v, w = manufactured(g, 0, 0, seed=3, mean_mode=True)
    uo, vo, wo, p = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0)
    assert relerr(p, p_true) <= 1e-12
    assert relerr(uo, us) <= 1e-12
    assert np.max(np.abs(wo)) <= 1e-12 * np.max(np.abs(w))


def test_manufactured_2048_grid_worst_conditioned_column():
    # the 2048^2 x 160 vertical grid (5 m -> 100 m over 160 levels) and
    # horizontal length (2048 x 25 m), coarsely sampled in x and y: the (1, 0)
    # and (0, 1) columns have the same smallest lambda as at full size.
    base = synth.make_grid("2048x2048x160")
    g = synth.Grid(32, 32, base.nz, 2048 * 25.0 / 32, 2048 * 25.0 / 32, base.dz, base.rho0)
    for (m0, n0) in [(1, 0), (1, 1)]:
        p_true, us, vs, u, v, w = manufactured(g, m0, n0, seed=5)
        uo, vo, wo, p = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0)
        assert relerr(p, p_true) <= 1e-10
        assert relerr(uo, us) <= 1e-10


# ----------------------------------------------------------------------------
# Invariants
# ----------------------------------------------------------------------------
def _inv_case(name):
    if name in ("32x32x32", "256x256x128"):
        m = synth.make_workload(name).members[0]
        return m.grid, m.u, m.v, m.w
    rng = np.random.default_rng(99)
    g = synth.random_grid(rng, 27, 12, 9, stretch=(1.0, 1.2))
    return (g,) + synth.random_fields(rng, g)


@pytest.mark.parametrize("case", ["32x32x32", "256x256x128", "odd"])
def test_invariants(case):
    g, u, v, w = _inv_case(case)
    uo, vo, wo, p = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0)
    div = oracle.divergence(uo, vo, wo, g.dx, g.dy, g.dz, g.rho0)
    assert np.max(np.abs(div)) <= 1e-12
    # gauge: dz-weighted volume sum of p is zero
    assert abs(np.sum(g.dz[:, None, None] * p)) <= 1e-12 * np.sum(g.dz[:, None, None] * np.abs(p))
    # horizontal mean of w vanishes on every face; means of u and v unchanged
    assert np.max(np.abs(wo.mean(axis=(1, 2)))) <= 1e-13 * np.max(np.abs(w))
    assert np.allclose(uo.mean(axis=(1, 2)), u.mean(axis=(1, 2)), rtol=0, atol=1e-13 * np.abs(u).max())
    assert np.allclose(vo.mean(axis=(1, 2)), v.mean(axis=(1, 2)), rtol=0, atol=1e-13 * np.abs(v).max())
    assert np.all(wo[-1] == 0.0)
    # energy identity E(u*) = E(u) + E(u* - u): the projection is orthogonal
    e_in = oracle.weighted_energy(u, v, w, g.dz, g.rho0)
    e_out = oracle.weighted_energy(uo, vo, wo, g.dz, g.rho0)
    e_gp = oracle.weighted_energy(u - uo, v - vo, w - wo, g.dz, g.rho0)
    assert abs(e_in - e_out - e_gp) <= 1e-12 * e_in


def test_idempotence_and_linearity():
    g, u, v, w = _inv_case("odd")
    a = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0)
    b = oracle.project(a[0], a[1], a[2], g.dx, g.dy, g.dz, g.rho0)
    assert np.max(np.abs(b[3])) <= 1e-12 * np.max(np.abs(a[3]))
    for t in range(3):
        assert relerr(b[t], a[t]) <= 1e-13
    rng = np.random.default_rng(5)
    u2, v2, w2 = synth.random_fields(rng, g)
    c = oracle.project(u2, v2, w2, g.dx, g.dy, g.dz, g.rho0)
    d = oracle.project(2.0 * u - 3.0 * u2, 2.0 * v - 3.0 * v2, 2.0 * w - 3.0 * w2,
                       g.dx, g.dy, g.dz, g.rho0)
    for t in range(4):
        assert relerr(d[t], 2.0 * a[t] - 3.0 * c[t]) <= 1e-12


# ----------------------------------------------------------------------------
# Continuum convergence (second order)
# ----------------------------------------------------------------------------
def _continuum_errors(stretched):
    L, H = 1000.0, 1000.0
    kx, ky = 2 * np.pi / L, 4 * np.pi / L
    errs = []
    for n in (8, 16, 32, 64):
        nx = ny = 2 * n
        nz = n
        xi = np.linspace(0.0, 1.0, nz + 1)
        zw = H * (xi + 0.3 * xi * (1 - xi)) if stretched else H * xi
        dz = np.diff(zw)
        zc = 0.5 * (zw[:-1] + zw[1:])
        dx = L / nx
        xc = (np.arange(nx) + 0.5) * dx
        xf = xc + 0.5 * dx
        yc, yf = xc, xf
        P = lambda x, y, z: np.cos(kx * x)[None, None, :] * np.cos(ky * y)[None, :, None] \
            * np.cos(np.pi * z / H)[:, None, None]
        p_ex = P(xc, yc, zc)
        u = (-kx * np.sin(kx * xf))[None, None, :] * np.cos(ky * yc)[None, :, None] * np.cos(np.pi * zc / H)[:, None, None]
        v = np.cos(kx * xc)[None, None, :] * (-ky * np.sin(ky * yf))[None, :, None] * np.cos(np.pi * zc / H)[:, None, None]
        w = np.cos(kx * xc)[None, None, :] * np.cos(ky * yc)[None, :, None] \
            * (-np.pi / H * np.sin(np.pi * zw[1:] / H))[:, None, None]
        w[-1] = 0.0
        _, _, _, p = oracle.project(u, v, w, dx, dx, dz, np.ones(nz))
        errs.append(np.max(np.abs(p - p_ex)))
    return errs


@pytest.mark.parametrize("stretched", [False, True])
def test_second_order_convergence(stretched):
    errs = _continuum_errors(stretched)
    rates = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert min(rates) >= 3.5, (errs, rates)


# ----------------------------------------------------------------------------
# Reductions to textbook cases
# ----------------------------------------------------------------------------
def test_nz1_is_2d_poisson():
    rng = np.random.default_rng(21)
    g = synth.Grid(24, 18, 1, 20.0, 35.0, np.array([13.0]), np.array([0.8]))
    u, v, w = synth.random_fields(rng, g)
    out = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0, intermediates=True)
    bh = np.fft.fft2(out["b"][0])
    kx = np.fft.fftfreq(g.nx) * g.nx
    ky = np.fft.fftfreq(g.ny) * g.ny
    lam = (4 / g.dx ** 2) * np.sin(np.pi * kx / g.nx)[None, :] ** 2 \
        + (4 / g.dy ** 2) * np.sin(np.pi * ky / g.ny)[:, None] ** 2
    lam[0, 0] = 1.0
    ph = -bh / (0.8 * lam)
    ph[0, 0] = 0.0
    assert relerr(out["p"][0], np.fft.ifft2(ph).real) <= 1e-13


def test_single_column_cumulative_sum():
    # nx = ny = 1: D(u) = 0 forces every interior flux to 0, so w -> 0, u and
    # v are untouched and p_{k+1} - p_k = dzc_k w*_k, then the gauge.
    rng = np.random.default_rng(4)
    g = synth.random_grid(rng, 1, 1, 9)
    u, v, w = synth.random_fields(rng, g)
    uo, vo, wo, p = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0)
    zc = np.concatenate([[0.0], np.cumsum(g.dz)])[:-1] + 0.5 * g.dz
    pc = np.concatenate([[0.0], np.cumsum(np.diff(zc) * w[:-1, 0, 0])])
    pc -= np.sum(g.dz * pc) / g.dz.sum()
    assert relerr(p[:, 0, 0], pc) <= 1e-14
    assert np.array_equal(uo, u) and np.array_equal(vo, v)
    assert np.max(np.abs(wo)) <= 1e-14 * np.max(np.abs(w))


def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                key, rest = line.split("=", 1)
                vals[key.strip()] = np.array([float(t) for t in rest.split()])
    return vals


def test_golden_single_column():
    gd = _read_golden("single_column_nz3.txt")
    dz, rho0, w = gd["dz"], gd["rho0"], gd["w"]
    shape = (3, 1, 1)
    uo, vo, wo, p = oracle.project(np.zeros(shape), np.zeros(shape), w.reshape(shape),
                                   7.0, 9.0, dz, rho0)
    assert np.allclose(p.ravel(), gd["p"], rtol=0, atol=1e-14)
    assert np.allclose(wo.ravel(), 0.0, atol=1e-15)


def test_golden_face_density_column_pair():
    # the separable oracle and the variable-density oracle with rho = rho0(z)
    # both reproduce the hand-derived overturning cell, which depends on the
    # w-face density
    gd = _read_golden("face_density_column_pair.txt")
    dx, dy, dz, rho0 = float(gd["dx"][0]), float(gd["dy"][0]), gd["dz"], gd["rho0"]
    shape = (2, 1, 2)
    z = np.zeros(shape)
    w = gd["w_in"].reshape(shape)
    out_sep = oracle.project(z, z, w, dx, dy, dz, rho0)
    rho = np.broadcast_to(rho0[:, None, None], shape).copy()
    out_var = oracle.project_var(z, z, w, dx, dy, dz, rho)
    for uo, vo, wo, p in (out_sep, out_var):
        assert np.allclose(uo.ravel(), gd["u83"] / 83.0, rtol=0, atol=1e-14)
        assert np.allclose(vo, 0.0, atol=1e-15)
        assert np.allclose(wo.ravel(), gd["w83"] / 83.0, rtol=0, atol=1e-14)
        assert np.allclose(p.ravel(), gd["p83"] / 83.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("axis", ["x", "y"])
def test_golden_face_density_ring(axis):
    gd = _read_golden("face_density_x_ring.txt")
    shape = (1, 1, 3) if axis == "x" else (1, 3, 1)
    rho = gd["rho"].reshape(shape)
    z = np.zeros(shape)
    f_in = gd["u_in"].reshape(shape)
    u_in, v_in = (f_in, z) if axis == "x" else (z, f_in)
    uo, vo, wo, p = oracle.project_var(u_in, v_in, z, 1.0, 1.0, np.ones(1), rho)
    got = uo if axis == "x" else vo
    other = vo if axis == "x" else uo
    assert np.allclose(got.ravel(), gd["u21"] / 21.0, rtol=0, atol=1e-14)
    assert np.allclose(other, 0.0, atol=1e-15)
    assert np.allclose(p.ravel(), gd["p63"] / 63.0, rtol=0, atol=1e-14)


# ----------------------------------------------------------------------------
# The pins catch plausible mistakes planted in the oracle (CPU only)
# ----------------------------------------------------------------------------
def _spectral_k2(nx, ny, dx, dy):
    m = np.arange(nx // 2 + 1)
    n = np.fft.fftfreq(ny) * ny
    return (2 * np.pi * m / (nx * dx)) ** 2, (2 * np.pi * n / (ny * dy)) ** 2


def _swapped_coeffs(dz, rho0):
    a, c = _ORIG["tridiag_coefficients"](dz, rho0)
    return c, a


def _plain_mean_rhow(dz, rho0):
    vg = _ORIG["vertical_grid"](dz, rho0)
    vg["rhow"] = 0.5 * (vg["rho0"][:-1] + vg["rho0"][1:])
    return vg


def _no_rho_div(u, v, w, dx, dy, dz, rho0):
    b = _ORIG["divergence"](u, v, w, dx, dy, dz, rho0)
    hor = (u - np.roll(u, 1, 2)) / dx + (v - np.roll(v, 1, 1)) / dy
    return b - (np.asarray(rho0)[:, None, None] - 1.0) * hor


def _flipped_grad(p, dx, dy, dz):
    gx, gy, gz = _ORIG["gradient"](p, dx, dy, dz)
    return gx, gy, -gz


def _unnormalised_inverse(P, nx, ny, workers=None):
    return _ORIG["inverse_spectrum"](P, nx, ny, workers) * 2.0


def _no_gauge(B0, dz, rho0):
    P = _ORIG["solve_mean_column"](B0, dz, rho0)
    return P + 0.37


_ORIG = {k: getattr(op, k) for k in ("modified_wavenumbers", "tridiag_coefficients",
                                     "vertical_grid", "divergence", "gradient",
                                     "inverse_spectrum", "solve_mean_column")}

MUTANTS = {
    "spectral_k2": ("modified_wavenumbers", _spectral_k2),
    "swapped_a_c": ("tridiag_coefficients", _swapped_coeffs),
    "midpoint_face_density": ("vertical_grid", _plain_mean_rhow),
    "rho_dropped_horizontal": ("divergence", _no_rho_div),
    "flipped_vertical_gradient": ("gradient", _flipped_grad),
    "wrong_inverse_scale": ("inverse_spectrum", _unnormalised_inverse),
    "gauge_missing": ("solve_mean_column", _no_gauge),
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_planted_mistake(mutant, monkeypatch):
    name, fn = MUTANTS[mutant]
    monkeypatch.setattr(op, name, fn)
    worst = max(brute_error(6, 4, 5, seed=1), brute_error(5, 3, 4, seed=2))
    assert worst > 1e-6, f"planted mistake {mutant} went unnoticed ({worst})"


def test_golden_catches_midpoint_face_density(monkeypatch):
    # the hand-derived w-face fixture fails when rhow is the plain mean
    monkeypatch.setattr(op, "vertical_grid", _plain_mean_rhow)
    with pytest.raises(AssertionError):
        test_golden_face_density_column_pair()


import oracle.variable as _ov  # noqa: E402

_ORIG_FACES = _ov.face_densities


def _cell_value_faces(rho, dz):
    # a plausible slip: an x or y face takes the density of the cell on its
    # west / south side instead of the mean of the two cells
    rx, ry, rz = _ORIG_FACES(rho, dz)
    rho = np.asarray(rho, dtype=np.float64)
    return rho.copy(), rho.copy(), rz


@pytest.mark.parametrize("axis", ["x", "y"])
def test_golden_catches_cell_value_face_density(axis, monkeypatch):
    monkeypatch.setattr(_ov, "face_densities", _cell_value_faces)
    with pytest.raises(AssertionError):
        test_golden_face_density_ring(axis)


def test_level_stats_closed_form():
    """Per-level reductions on fields with known per-level mean and maximum:
    a level constant plus a periodic mode whose horizontal mean is zero and
    whose maximum over the grid is attained (cos at i = j = 0)."""
    nz, ny, nx = 5, 6, 8
    k = np.arange(nz, dtype=np.float64)[:, None, None]
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    mode = np.cos(2 * np.pi * i / nx) * np.cos(2 * np.pi * j / ny)
    amp = np.array([0.5, 1.0, 2.0, 0.25])
    fields = [(3.0 * f + 1.0) * k - 7.0 + a * mode for f, a in enumerate(amp)]
    st = oracle.level_stats(*fields)
    assert st.shape == (4, 2, nz)
    for f, a in enumerate(amp):
        base = (3.0 * f + 1.0) * np.arange(nz) - 7.0
        np.testing.assert_allclose(st[f, 0], base, rtol=0, atol=1e-14)
        np.testing.assert_allclose(st[f, 1], base + a, rtol=0, atol=1e-14)
    # a field that is one value everywhere except a single point
    p = np.zeros((nz, ny, nx))
    p[2, 3, 4] = 48.0
    st = oracle.level_stats(p, p, p, p)
    assert st[0, 0, 2] == 1.0 and st[0, 1, 2] == 48.0 and st[0, 1, 1] == 0.0


# ---------------------------------------------------------------------------
# horizontally varying density (the operator the Krylov path solves)
# ---------------------------------------------------------------------------
def _var_case(nx, ny, nz, seed, vary=0.3):
    rng = np.random.default_rng(seed)
    g = synth.random_grid(rng, nx, ny, nz, stretch=(1.0, 1.1))
    rho = g.rho0[:, None, None] * (1.0 + vary * rng.uniform(-1.0, 1.0, (nz, ny, nx)))
    u, v, w = synth.random_fields(rng, g)
    return g, rho, u, v, w


def test_variable_operator_matrix_is_the_stencil():
    """The assembled matrix equals D_rho(G p) evaluated by the stencil
    functions (separate code), is symmetric in the dz weights and annihilates
    constants."""
    g, rho, *_ = _var_case(5, 4, 6, seed=31)
    L = oracle.operator_matrix(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, rho)
    p = np.random.default_rng(32).standard_normal((g.nz, g.ny, g.nx))
    gx, gy, gz = oracle.gradient(p, g.dx, g.dy, g.dz)
    ref = oracle.divergence_var(gx, gy, gz, g.dx, g.dy, g.dz, rho)
    np.testing.assert_allclose((L @ p.ravel()).reshape(p.shape), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    W = np.broadcast_to(np.asarray(g.dz)[:, None, None], p.shape).ravel()
    A = (L.multiply(W[:, None])).toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(L @ np.ones(L.shape[0])).max() <= 1e-12 * np.abs(A).max()


def test_variable_projection_is_divergence_free_with_gauge():
    g, rho, u, v, w = _var_case(6, 5, 7, seed=33)
    uo, vo, wo, p = oracle.project_var(u, v, w, g.dx, g.dy, g.dz, rho)
    div = oracle.divergence_var(uo, vo, wo, g.dx, g.dy, g.dz, rho)
    scale = np.abs(oracle.divergence_var(u, v, w, g.dx, g.dy, g.dz, rho)).max()
    assert np.abs(div).max() <= 1e-12 * scale
    assert abs(np.sum(np.asarray(g.dz)[:, None, None] * p)) <= 1e-12 * np.abs(p).sum()
    assert np.all(wo[-1] == 0.0)


def test_variable_projection_reduces_to_separable():
    """A density of z alone gives the separable projection."""
    rng = np.random.default_rng(34)
    g = synth.random_grid(rng, 8, 6, 5, stretch=(1.0, 1.1))
    u, v, w = synth.random_fields(rng, g)
    rho = np.broadcast_to(np.asarray(g.rho0)[:, None, None], (g.nz, g.ny, g.nx)).copy()
    got = oracle.project_var(u, v, w, g.dx, g.dy, g.dz, rho)
    ref = oracle.project(u, v, w, g.dx, g.dy, g.dz, g.rho0)
    for a, b in zip(got, ref):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-11 * max(np.abs(b).max(), 1.0))


def _x_only_case(nx, ny, nz, seed):
    """rho and u* functions of x alone (the same on every row and level),
    v* = w* = 0. The projected flux rx_i u_i is then the same constant C on
    every east face: the periodic sum of the gradient vanishes, so
    C = sum_i u*_i / sum_i 1/rx_i and u_i = C / rx_i (a harmonic mean);
    p_{i+1} - p_i = dx (u*_i - u_i), with zero mean (the gauge)."""
    rng = np.random.default_rng(seed)
    dx, dy = 40.0, 30.0
    dz = 10.0 * 1.1 ** np.arange(nz)
    r1 = 1.0 + 0.5 * rng.uniform(-1.0, 1.0, nx)
    u1 = rng.standard_normal(nx)
    rho = np.broadcast_to(r1, (nz, ny, nx)).copy()
    u = np.broadcast_to(u1, (nz, ny, nx)).copy()
    z = np.zeros((nz, ny, nx))
    rx = 0.5 * (r1 + np.roll(r1, -1))
    C = u1.sum() / np.sum(1.0 / rx)
    uo = C / rx
    p1 = np.concatenate([[0.0], np.cumsum(dx * (u1 - uo))[:-1]])
    p1 -= p1.mean()
    return dx, dy, dz, rho, u, z, np.broadcast_to(uo, (nz, ny, nx)), np.broadcast_to(p1, (nz, ny, nx))


@pytest.mark.parametrize("shape", [(12, 1, 1), (9, 4, 3)])
def test_variable_projection_x_only_closed_form(shape):
    dx, dy, dz, rho, u, z, uo, po = _x_only_case(*shape, seed=35)
    got = oracle.project_var(u, z, z, dx, dy, dz, rho)
    np.testing.assert_allclose(got[0], uo, rtol=0, atol=1e-12 * np.abs(uo).max())
    assert np.abs(got[1]).max() <= 1e-12 and np.abs(got[2]).max() <= 1e-12
    np.testing.assert_allclose(got[3], po, rtol=0, atol=1e-11 * np.abs(po).max())
