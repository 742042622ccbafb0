"""Tolerances of the GPU parity tests (test infrastructure; uses the oracle's
coefficient definitions to bound the conditioning of the column systems)."""
import numpy as np

import oracle

TOL64 = 1e-12      # FP64 path: u, v, w relative to the input scale
TOL_MIXED = 1e-6   # mixed path: every field, normwise relative


def worst_column_condition(g):
    """kappa_inf of the worst-conditioned column system: the tridiagonal of
    the smallest nonzero horizontal eigenvalue, or the (0,0) column's system
    with the top unknown pinned (rows 0..nz-2)."""
    a, c = oracle.tridiag_coefficients(g.dz, g.rho0)
    cond = lambda T: float(np.linalg.norm(T, np.inf) * np.linalg.norm(np.linalg.inv(T), np.inf))
    kappa = 1.0
    if g.nz > 1:
        m = g.nz - 1
        T0 = np.diag(-(a[:m] + c[:m])) + np.diag(a[1:m], -1) + np.diag(c[:m - 1], 1)
        kappa = cond(T0)
    lamx, lamy = oracle.modified_wavenumbers(g.nx, g.ny, g.dx, g.dy)
    lam = (lamy[:, None] + lamx[None, :]).ravel()
    lam = lam[lam > 0]
    if lam.size:
        T = np.diag(-(a + c) - g.rho0 * lam.min()) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        kappa = max(kappa, cond(T))
    return kappa


def p_tolerance(g):
    return max(TOL64, 4 * 2.0 ** -53 * worst_column_condition(g))
