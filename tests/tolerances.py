"""Tolerances of the GPU parity tests (test infrastructure; uses the oracle's
coefficient definitions to bound the conditioning of the column systems)."""
import numpy as np

import oracle
import oracle.projection

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


def reference_noise(b_spec, p_ref, g, workers=None):
    """How far two correct FP64 answers for p lie apart on this input: the
    oracle's spectrum B solved column by column with Thomas elimination
    running from the lid down (rows reversed) instead of from the bottom up,
    transformed back, and compared normwise with the oracle's p. Both sweeps
    are backward stable, so their spread is the round-off the conditioning of
    this input's wavenumber columns allows; a correct FP64 solver (the GPU's
    partitioned elimination included) lands within a small multiple of it.
    The (0,0) column is solved the other way round as well: the bottom
    unknown pinned instead of the top one (rows 1..nz-1, which with a
    compatible right-hand side imply row 0), then the same gauge.""" 
    a, c = oracle.tridiag_coefficients(g.dz, g.rho0)
    rho0 = np.asarray(g.rho0, dtype=np.float64)
    lamx, lamy = oracle.modified_wavenumbers(g.nx, g.ny, g.dx, g.dy)
    lam = lamy[:, None] + lamx[None, :]
    lam[0, 0] = 1.0                                   # replaced below
    nz = len(rho0)
    beta = (-(a + c))[:, None, None] - rho0[:, None, None] * lam[None]
    # reversed system: row k' = nz-1-k, sub- and super-diagonals swap
    ar, cr = c[::-1].copy(), a[::-1].copy()
    br = beta[::-1]
    d = b_spec[::-1]
    cp = np.empty(br.shape)
    dp = np.empty(d.shape, dtype=d.dtype)
    cp[0] = cr[0] / br[0]
    dp[0] = d[0] / br[0]
    for k in range(1, nz):
        den = br[k] - ar[k] * cp[k - 1]
        cp[k] = cr[k] / den
        dp[k] = (d[k] - ar[k] * dp[k - 1]) / den
    x = np.empty_like(dp)
    x[nz - 1] = dp[nz - 1]
    for k in range(nz - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    del cp, dp
    P = x[::-1].copy()
    del x
    P[:, 0, 0] = _mean_column_bottom_pinned(b_spec[:, 0, 0], g.dz, g.rho0)
    p_alt = oracle.inverse_spectrum(P, g.nx, g.ny, workers)
    del P
    return float(np.abs(p_alt - p_ref).max() / np.abs(p_ref).max())


def _mean_column_bottom_pinned(B0, dz, rho0):
    """The singular (0,0) column with P_0 = 0 and rows 1..nz-1 (the oracle
    pins P_{nz-1} and keeps rows 0..nz-2), then the gauge sum dz P = 0."""
    dz = np.asarray(dz, dtype=np.float64)
    nz = len(dz)
    H = dz.sum()
    d = B0 - np.sum(dz * B0) / H
    P = np.zeros(nz, dtype=B0.dtype)
    if nz > 1:
        a, c = oracle.tridiag_coefficients(dz, rho0)
        sub, dia, sup, rhs = a[1:], -(a[1:] + c[1:]), c[1:], d[1:]
        n = nz - 1
        cp = np.empty(n)
        dp = np.empty(n, dtype=rhs.dtype)
        cp[0] = sup[0] / dia[0]
        dp[0] = rhs[0] / dia[0]
        for k in range(1, n):
            den = dia[k] - sub[k] * cp[k - 1]
            cp[k] = sup[k] / den
            dp[k] = (rhs[k] - sub[k] * dp[k - 1]) / den
        x = np.empty_like(dp)
        x[n - 1] = dp[n - 1]
        for k in range(n - 2, -1, -1):
            x[k] = dp[k] - cp[k] * x[k + 1]
        P[1:] = x
    return P - np.sum(dz * P) / H
