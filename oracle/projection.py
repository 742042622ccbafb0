"""FP64 NumPy/SciPy reference of the pressure projection.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing on the product
path imports this module.

What the paper fixes (Sec. 4, "Performance and scaling", the paragraph on the
FFT pressure solver): the pressure terms come from a Poisson problem that the
model solves by a forward horizontal FFT, then a vertical ODE per horizontal
wavenumber in Fourier space, then a backward FFT. The paper gives no
discretisation, so this oracle takes the second-order Arakawa C-grid
finite-volume reading below; every choice the paper leaves open is stated
where it is made.

Grid and staggering (arrays are C-order (nz, ny, nx), periodic in x and y):
  p[k,j,i]   cell centre ((i+1/2)dx, (j+1/2)dy, zc_k)
  u[k,j,i]   east face  x = (i+1)dx
  v[k,j,i]   north face y = (j+1)dy
  w[k,j,i]   top face   z = zw_{k+1};  w[nz-1] is the rigid lid (0), and the
             bottom lid w = 0 at z = 0 is implicit.
  dz[k]      cell thickness; zw_0 = 0, zw_{k+1} = zw_k + dz_k,
             zc_k = zw_k + dz_k/2, dzc_k = zc_{k+1} - zc_k = (dz_k + dz_{k+1})/2
             (evaluated in that last form).
  rho0[k]    anelastic reference density at cell centres; on the face
             zw_{k+1} it is interpolated linearly in z (rhow_k).

Operators:
  D(u)_k = rho0_k [(u_i - u_{i-1})/dx + (v_j - v_{j-1})/dy]
           + (rhow_k w_k - rhow_{k-1} w_{k-1}) / dz_k     (flux 0 at both lids)
  G(p)   = ((p_{i+1}-p_i)/dx, (p_{j+1}-p_j)/dy, (p_{k+1}-p_k)/dzc_k)
  Projection: solve D(G p) = D(u*) with the gauge sum_k dz_k sum_ij p = 0,
  then u = u* - G p (dt folded into p), and w[nz-1] = 0.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

_F64 = np.float64


def _workers() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def vertical_grid(dz, rho0):
    """Vertical metrics from cell thicknesses dz[nz] and centre densities
    rho0[nz]: face heights zw[nz+1], centres zc[nz], centre spacings
    dzc[nz-1] and face densities rhow[nz-1] (at zw_1 .. zw_{nz-1})."""
    dz = np.asarray(dz, dtype=_F64)
    rho0 = np.asarray(rho0, dtype=_F64)
    zw = np.concatenate([[0.0], np.cumsum(dz)])
    zc = zw[:-1] + 0.5 * dz
    # centre spacing straight from the thicknesses (dzc_k = (dz_k + dz_{k+1})/2),
    # not as a difference of accumulated heights, which cancels at the top
    # of a tall column
    dzc = 0.5 * (dz[:-1] + dz[1:])
    # linear interpolation of rho0 from zc_k, zc_{k+1} to the face zw_{k+1},
    # which lies dz_k/2 above zc_k and dz_{k+1}/2 below zc_{k+1}
    rhow = (dz[1:] * rho0[:-1] + dz[:-1] * rho0[1:]) / (dz[:-1] + dz[1:])
    return {"zw": zw, "zc": zc, "dzc": dzc, "rhow": rhow, "dz": dz, "rho0": rho0}


def divergence(u, v, w, dx, dy, dz, rho0):
    """Anelastic C-grid divergence D(u) at cell centres (definition above)."""
    vg = vertical_grid(dz, rho0)
    nz = u.shape[0]
    hor = (u - np.roll(u, 1, axis=2)) / dx + (v - np.roll(v, 1, axis=1)) / dy
    flux = np.zeros((nz + 1,) + u.shape[1:], dtype=_F64)   # flux[k] at zw_k
    flux[1:nz] = vg["rhow"][:, None, None] * w[: nz - 1]
    vert = (flux[1:] - flux[:-1]) / vg["dz"][:, None, None]
    return vg["rho0"][:, None, None] * hor + vert


def gradient(p, dx, dy, dz):
    """Staggered gradient G(p) on the u, v, w points; the lid row of the
    vertical component is 0."""
    dz = np.asarray(dz, dtype=_F64)
    dzc = 0.5 * (dz[:-1] + dz[1:])                 # zc_{k+1} - zc_k, as in vertical_grid
    gx = (np.roll(p, -1, axis=2) - p) / dx
    gy = (np.roll(p, -1, axis=1) - p) / dy
    gz = np.zeros_like(p)
    gz[:-1] = (p[1:] - p[:-1]) / dzc[:, None, None]
    return gx, gy, gz


def tridiag_coefficients(dz, rho0):
    """Vertical part of D(G p) for one horizontal wavenumber:
    row k reads a_k P_{k-1} + (-a_k - c_k - rho0_k lam) P_k + c_k P_{k+1}."""
    vg = vertical_grid(dz, rho0)
    nz = len(vg["dz"])
    a = np.zeros(nz)
    c = np.zeros(nz)
    if nz > 1:
        a[1:] = vg["rhow"] / (vg["dz"][1:] * vg["dzc"])
        c[:-1] = vg["rhow"] / (vg["dz"][:-1] * vg["dzc"])
    return a, c


def modified_wavenumbers(nx, ny, dx, dy):
    """Eigenvalues of minus the discrete second differences:
    lam_x(m) = (4/dx^2) sin^2(pi m / nx) for m = 0..nx//2 and
    lam_y(n) = (4/dy^2) sin^2(pi n / ny) for n = 0..ny-1. The modified (not
    spectral) wavenumber makes the solve exact for the discrete operator."""
    m = np.arange(nx // 2 + 1, dtype=_F64)
    n = np.arange(ny, dtype=_F64)
    lamx = (4.0 / dx ** 2) * np.sin(np.pi * m / nx) ** 2
    lamy = (4.0 / dy ** 2) * np.sin(np.pi * n / ny) ** 2
    return lamx, lamy


def forward_spectrum(b, workers=None):
    """Unnormalised real 2-D FFT of every level: B[k, n, m], m = 0..nx//2."""
    return sfft.rfft2(b, axes=(1, 2), workers=workers or _workers())


def inverse_spectrum(P, nx, ny, workers=None):
    """Inverse of forward_spectrum with the 1/(nx*ny) factor; the imaginary
    parts of self-conjugate bins are ignored (c2r convention)."""
    return sfft.irfft2(P, s=(ny, nx), axes=(1, 2), workers=workers or _workers())


def _thomas(a, beta, c, d):
    """Thomas elimination without pivoting, vectorised over trailing axes.
    a, c: (n,) real; beta: (n, ...) real; d: (n, ...) complex."""
    n = d.shape[0]
    cp = np.empty(beta.shape, dtype=_F64)
    dp = np.empty(d.shape, dtype=d.dtype)
    den = beta[0]
    cp[0] = c[0] / den
    dp[0] = d[0] / den
    for k in range(1, n):
        den = beta[k] - a[k] * cp[k - 1]
        cp[k] = c[k] / den
        dp[k] = (d[k] - a[k] * dp[k - 1]) / den
    x = np.empty_like(dp)
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def solve_mean_column(B0, dz, rho0):
    """The (m, n) = (0, 0) column, whose operator is singular (constants).
    1. remove the dz-weighted mean of the right-hand side (its incompatible
       part, which is round-off for a divergence);
    2. pin P_{nz-1} = 0 and solve rows 0..nz-2 (the last row then holds);
    3. shift P so that sum_k dz_k P_k = 0 (the gauge)."""
    dz = np.asarray(dz, dtype=_F64)
    nz = len(dz)
    H = dz.sum()
    d = B0 - np.sum(dz * B0) / H
    P = np.zeros(nz, dtype=B0.dtype)
    if nz > 1:
        a, c = tridiag_coefficients(dz, rho0)
        m = nz - 1
        P[:m] = _thomas(a[:m], -(a[:m] + c[:m]), c[:m], d[:m])
    P = P - np.sum(dz * P) / H
    return P


def solve_columns(B, dz, rho0, dx, dy, nx, ny):
    """Vertical ODE of every horizontal wavenumber (m, n): a tridiagonal
    system in z with real coefficients and complex right-hand side B[:, n, m].
    The (0, 0) column takes solve_mean_column."""
    rho0 = np.asarray(rho0, dtype=_F64)
    a, c = tridiag_coefficients(dz, rho0)
    lamx, lamy = modified_wavenumbers(nx, ny, dx, dy)
    lam = lamy[:, None] + lamx[None, :]
    lam_safe = lam.copy()
    lam_safe[0, 0] = 1.0            # placeholder; the column is replaced below
    beta = (-(a + c))[:, None, None] - rho0[:, None, None] * lam_safe[None]
    P = _thomas(a, beta, c, B)
    P[:, 0, 0] = solve_mean_column(B[:, 0, 0], dz, rho0)
    return P


def project(u, v, w, dx, dy, dz, rho0, intermediates=False, workers=None):
    """Pressure projection of (u, v, w) in FP64.

    Returns (u, v, w, p) as new arrays, or a dict with the intermediates
    b = D(u*), B = its spectrum, P = the solved spectrum as well."""
    u = np.asarray(u, dtype=_F64)
    v = np.asarray(v, dtype=_F64)
    w = np.asarray(w, dtype=_F64)
    nz, ny, nx = u.shape
    b = divergence(u, v, w, dx, dy, dz, rho0)
    B = forward_spectrum(b, workers)
    P = solve_columns(B, dz, rho0, dx, dy, nx, ny)
    p = inverse_spectrum(P, nx, ny, workers)
    gx, gy, gz = gradient(p, dx, dy, dz)
    uo = u - gx
    vo = v - gy
    wo = w - gz
    wo[nz - 1] = 0.0
    if intermediates:
        return {"u": uo, "v": vo, "w": wo, "p": p, "b": b, "B": B, "P": P}
    return uo, vo, wo, p


def weighted_energy(u, v, w, dz, rho0):
    """E = sum rho0 dz (u^2 + v^2) + sum rhow dzc w^2 (interior faces): the
    weights under which -G is the adjoint of D, so the projection is
    orthogonal in this norm."""
    vg = vertical_grid(dz, rho0)
    wt = (vg["rho0"] * vg["dz"])[:, None, None]
    e = np.sum(wt * (u * u + v * v))
    if len(vg["dz"]) > 1:
        e += np.sum((vg["rhow"] * vg["dzc"])[:, None, None] * w[:-1] ** 2)
    return float(e)
