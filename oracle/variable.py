"""Projection with a horizontally varying density (the non-separable case).

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing on the product
path imports this module.

Sec. 4 of the paper sets the FFT solver beside an iterative Krylov solver
(ILU-preconditioned BiCGStab), and Sec. 5 proposes bespoke preconditioners and
a mixed-precision solver with a double-precision restart. The FFT solve is
exact only when the operator separates (density a function of z alone); with a
density rho(x, y, z) it is an approximate inverse, the natural preconditioner
of a Krylov solve. This module defines that operator and solves it directly.

Reading (the paper gives no discretisation): rho[k, j, i] at the cell
centres; on the faces the arithmetic mean of the two cells in x and y and, in
z, the linear interpolation used for rho0 on the w faces. With rho = rho0(z)
every face density equals the separable operator's, so the projection here
reduces to projection.project.

  D_rho(u)_k = (rx_i u_i - rx_{i-1} u_{i-1})/dx + (ry_j v_j - ry_{j-1} v_{j-1})/dy
               + (rz_k w_k - rz_{k-1} w_{k-1})/dz_k         (flux 0 at both lids)
  with rx = (rho_i + rho_{i+1})/2, ry = (rho_j + rho_{j+1})/2,
       rz_k = (dz_{k+1} rho_k + dz_k rho_{k+1})/(dz_k + dz_{k+1}).
  Projection: D_rho(G p) = D_rho(u*), sum_k dz_k sum_ij p = 0, u = u* - G p.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .projection import gradient

_F64 = np.float64


def face_densities(rho, dz):
    """(rx, ry, rz): densities on the east, north and top faces (rz has nz-1
    levels, the interior top faces)."""
    rho = np.asarray(rho, dtype=_F64)
    dz = np.asarray(dz, dtype=_F64)
    rx = 0.5 * (rho + np.roll(rho, -1, axis=2))
    ry = 0.5 * (rho + np.roll(rho, -1, axis=1))
    d0, d1 = dz[:-1, None, None], dz[1:, None, None]
    rz = (d1 * rho[:-1] + d0 * rho[1:]) / (d0 + d1)
    return rx, ry, rz


def divergence_var(u, v, w, dx, dy, dz, rho):
    """D_rho(u) at the cell centres (definition above)."""
    dz = np.asarray(dz, dtype=_F64)
    rx, ry, rz = face_densities(rho, dz)
    nz = u.shape[0]
    fx = rx * u
    fy = ry * v
    hor = (fx - np.roll(fx, 1, axis=2)) / dx + (fy - np.roll(fy, 1, axis=1)) / dy
    flux = np.zeros((nz + 1,) + u.shape[1:], dtype=_F64)
    flux[1:nz] = rz * w[: nz - 1]
    return hor + (flux[1:] - flux[:-1]) / dz[:, None, None]


def operator_matrix(nx, ny, nz, dx, dy, dz, rho):
    """Sparse L = D_rho G on the flattened (k, j, i) cell index."""
    dz = np.asarray(dz, dtype=_F64)
    rx, ry, rz = face_densities(rho, dz)
    idx = np.arange(nz * ny * nx).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []

    def add(r, c, v):
        rows.append(r.ravel())
        cols.append(c.ravel())
        vals.append(np.broadcast_to(v, r.shape).ravel())

    # x faces: flux rx (p_{i+1} - p_i)/dx leaves cell i, enters cell i+1
    e = np.roll(idx, -1, axis=2)
    cx = rx / (dx * dx)
    add(idx, e, cx); add(idx, idx, -cx); add(e, idx, cx); add(e, e, -cx)
    n = np.roll(idx, -1, axis=1)
    cy = ry / (dy * dy)
    add(idx, n, cy); add(idx, idx, -cy); add(n, idx, cy); add(n, n, -cy)
    if nz > 1:
        dzc = 0.5 * (dz[:-1] + dz[1:])
        lo, hi = idx[:-1], idx[1:]
        f = rz / dzc[:, None, None]
        add(lo, hi, f / dz[:-1, None, None]); add(lo, lo, -f / dz[:-1, None, None])
        add(hi, lo, f / dz[1:, None, None]); add(hi, hi, -f / dz[1:, None, None])
    N = nz * ny * nx
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def project_var(u, v, w, dx, dy, dz, rho):
    """Projection with density rho(x, y, z), solved directly. The operator
    times the cell weights dz is symmetric with the constants as its null
    space and the right-hand side (made exactly compatible by removing its
    dz-weighted mean) lies in its range, so: fix the first unknown at zero,
    solve the remaining nonsingular sparse system, and shift p by its
    dz-weighted mean to meet the gauge. Returns (u, v, w, p). For small
    grids (a sparse LU of nx ny nz - 1 unknowns)."""
    u = np.asarray(u, dtype=_F64)
    v = np.asarray(v, dtype=_F64)
    w = np.asarray(w, dtype=_F64)
    dz = np.asarray(dz, dtype=_F64)
    nz, ny, nx = u.shape
    N = nx * ny * nz
    L = operator_matrix(nx, ny, nz, dx, dy, dz, rho)
    wt = np.broadcast_to(dz[:, None, None], (nz, ny, nx)).ravel()
    A = (sp.diags(wt) @ L).tocsc()
    b = divergence_var(u, v, w, dx, dy, dz, rho).ravel()
    rhs = wt * (b - np.sum(wt * b) / np.sum(wt))   # compatible right-hand side
    x = np.zeros(N)
    if N > 1:
        x[1:] = spla.splu(A[1:, 1:], permc_spec="MMD_AT_PLUS_A").solve(rhs[1:])
    x -= np.sum(wt * x) / np.sum(wt)
    p = x.reshape(nz, ny, nx)
    gx, gy, gz = gradient(p, dx, dy, dz)
    wo = w - gz
    wo[nz - 1] = 0.0
    return u - gx, v - gy, wo, p
