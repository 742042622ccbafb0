"""Seeded synthetic workloads for the anelastic pressure projection.

This module only draws grids and velocity fields. It holds none of the
projection's arithmetic (no divergence, transform or solve), so that both the
FP64 oracle and the HIP path can be fed from it without sharing any method
code.

The paper's own workload is the dry boundary-layer case (Sec. 4, "Performance
and scaling": z = 64 levels, horizontal grids of n^2 points, 32 x 32 x 64 points
per process in the weak-scaling runs). Its inputs need the whole model and are
not available, so the configurations below stand in for it:

  "32x32x32"       32^3, dx = dy = 50 m, uniform dz = 20 m, rho0 = 1
  "256x256x128"    256^2 x 128, dx = dy = 25 m, dz_k = min(10 * 1.015^k, 60) m,
                   rho0 = 1.2 exp(-zc / 8000 m)
  "1024x1024x256"  1024^2 x 256 with the same vertical profiles (stored FP32)
  "ensemble48"     48-member ensemble, grids drawn from {64^2x64, 128^2x96,
                   192^2x128, 256^2x128}, per member dz_k = 10 r^k
                   (r ~ U(1.00, 1.02)) and rho0 = 1.2 exp(-zc / H)
                   (H ~ U(6, 10) km) (stored FP32)
  "2048x2048x160"  2048^2 x 160, dz_k = 5 * 20^(k/159) m, rho0 as above,
                   horizontal k^-5/3 spectrum (stored FP32)

Field conventions (C-order arrays (nz, ny, nx), x fastest):
  u[k, j, i] sits at x = (i + 1) dx, y = (j + 1/2) dy  (east face)
  v[k, j, i] sits at x = (i + 1/2) dx, y = (j + 1) dy  (north face)
  w[k, j, i] sits at the top face of cell k; w[nz - 1] is the rigid lid and is 0.

All randomness comes from NumPy's PCG64 (``numpy.random.default_rng``).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

__all__ = ["Grid", "Member", "Workload", "CONFIGS", "make_workload",
           "make_grid", "mode_fields", "random_grid", "random_fields", "density_field"]


@dataclasses.dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: np.ndarray      # (nz,) cell thicknesses [m]
    rho0: np.ndarray    # (nz,) reference density at cell centres [kg m^-3]

    @property
    def points(self) -> int:
        return self.nx * self.ny * self.nz

    def key(self):
        return (self.nx, self.ny, self.nz)


@dataclasses.dataclass
class Member:
    grid: Grid
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray


@dataclasses.dataclass
class Workload:
    name: str
    dtype: str               # "f64" (plain) or "mixed" (FP32 storage)
    members: List[Member]
    description: str

    @property
    def points(self) -> int:
        return sum(m.grid.points for m in self.members)


CONFIGS = {
    "32x32x32": "FP64, 32x32x32, dx=dy=50 m, dz=20 m, rho0=1; u,v,w ~ N(0,1) + 2cos(2pi x/Lx)cos(2pi y/Ly)",
    "256x256x128": "FP64, 256x256x128, dx=dy=25 m, dz=min(10*1.015^k,60) m, rho0=1.2exp(-z/8 km); "
                   "u,v ~ N(0,4)+8 modes, w ~ N(0,0.25)",
    "1024x1024x256": "mixed (FP32 storage), 1024x1024x256, the 256x256x128 vertical profiles and field recipe",
    "ensemble48": "mixed, 48-member ensemble of uneven grids, per-member dz stretch and rho0 scale height",
    "2048x2048x160": "mixed, 2048x2048x160, dz=5*20^(k/159) m, rho0=1.2exp(-z/8 km), k^-5/3 horizontal spectra",
    "4096x4096x64": "mixed, 4096x4096x64 (the paper's 1.07e9-point global problem on one GPU), "
                    "dx=dy=25 m, dz=min(10*1.015^k,60) m, rho0=1.2exp(-z/8 km), the 256x256x128 field recipe",
}


def _zc(dz: np.ndarray) -> np.ndarray:
    zw = np.concatenate([[0.0], np.cumsum(dz)])
    return zw[:-1] + 0.5 * dz


def capped_geometric_dz(nz: int, dz0: float = 10.0, ratio: float = 1.015,
                        cap: float = 60.0) -> np.ndarray:
    """dz_k = min(dz0 * ratio^k, cap)."""
    return np.minimum(dz0 * ratio ** np.arange(nz, dtype=np.float64), cap)


def exp_rho0(dz: np.ndarray, scale_height: float = 8000.0) -> np.ndarray:
    """rho0 = 1.2 exp(-zc / H) evaluated at the cell centres."""
    return 1.2 * np.exp(-_zc(dz) / scale_height)


def make_grid(name: str) -> Grid:
    if name == "32x32x32":
        return Grid(32, 32, 32, 50.0, 50.0, np.full(32, 20.0), np.ones(32))
    if name == "256x256x128":
        dz = capped_geometric_dz(128)
        return Grid(256, 256, 128, 25.0, 25.0, dz, exp_rho0(dz))
    if name == "1024x1024x256":
        dz = capped_geometric_dz(256)
        return Grid(1024, 1024, 256, 25.0, 25.0, dz, exp_rho0(dz))
    if name == "2048x2048x160":
        dz = 5.0 * 20.0 ** (np.arange(160, dtype=np.float64) / 159.0)
        return Grid(2048, 2048, 160, 25.0, 25.0, dz, exp_rho0(dz))
    if name == "4096x4096x64":
        dz = capped_geometric_dz(64)
        return Grid(4096, 4096, 64, 25.0, 25.0, dz, exp_rho0(dz))
    raise KeyError(name)


def _staggered_coords(g: Grid):
    """1-D coordinates of cell centres and faces in x and y."""
    xc = (np.arange(g.nx) + 0.5) * g.dx
    xf = (np.arange(g.nx) + 1.0) * g.dx
    yc = (np.arange(g.ny) + 0.5) * g.dy
    yf = (np.arange(g.ny) + 1.0) * g.dy
    return xc, xf, yc, yf


def _mode_sum(rng, g: Grid, x: np.ndarray, y: np.ndarray, count: int = 8):
    """Sum of `count` plane waves A cos(2 pi (m x / Lx + n y / Ly) + phi),
    (m, n) uniform in [-4, 4]^2 minus the origin, A ~ U(0.5, 1.5),
    phi ~ U(0, 2 pi); constant in z. Returns a (ny, nx) array."""
    Lx, Ly = g.nx * g.dx, g.ny * g.dy
    out = np.zeros((g.ny, g.nx))
    drawn = 0
    while drawn < count:
        m, n = rng.integers(-4, 5, size=2)
        if m == 0 and n == 0:
            continue
        amp = rng.uniform(0.5, 1.5)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        ax = 2.0 * np.pi * m * x / Lx + phi
        by = 2.0 * np.pi * n * y / Ly
        # cos(ax + by) = cos(ax) cos(by) - sin(ax) sin(by), as an outer product
        out += amp * (np.outer(np.cos(by), np.cos(ax)) - np.outer(np.sin(by), np.sin(ax)))
        drawn += 1
    return out


def mode_fields(rng, g: Grid):
    """u, v ~ N(0, variance 4) + 8 low-wavenumber modes each; w ~ N(0, variance
    0.25); rigid lid w[nz-1] = 0."""
    xc, xf, yc, yf = _staggered_coords(g)
    shape = (g.nz, g.ny, g.nx)
    u = 2.0 * rng.standard_normal(shape)
    v = 2.0 * rng.standard_normal(shape)
    w = 0.5 * rng.standard_normal(shape)
    u += _mode_sum(rng, g, xf, yc)[None]
    v += _mode_sum(rng, g, xc, yf)[None]
    w[g.nz - 1] = 0.0
    return u, v, w


def _small_fields(rng, g: Grid):
    xc, xf, yc, yf = _staggered_coords(g)
    Lx, Ly = g.nx * g.dx, g.ny * g.dy
    shape = (g.nz, g.ny, g.nx)
    u = rng.standard_normal(shape)
    v = rng.standard_normal(shape)
    w = rng.standard_normal(shape)
    mode = lambda x, y: 2.0 * np.outer(np.cos(2 * np.pi * y / Ly), np.cos(2 * np.pi * x / Lx))
    u += mode(xf, yc)[None]
    v += mode(xc, yf)[None]
    w += mode(xc, yc)[None]
    w[g.nz - 1] = 0.0
    return u, v, w


def _spectral_field(rng, g: Grid, std: float, chunk: int = 8):
    """Real field whose horizontal spectrum has shell energy ~ kappa^(-5/3),
    i.e. 2-D amplitude ~ kappa^(-4/3) for 1 <= kappa <= Nyquist, random
    phases, independent per level; scaled to the given std per level."""
    m = np.arange(g.nx // 2 + 1, dtype=np.float64)
    n = np.fft.fftfreq(g.ny, d=1.0 / g.ny)
    kappa = np.sqrt(n[:, None] ** 2 + m[None, :] ** 2)
    kmax = min(g.nx, g.ny) / 2.0
    amp = np.where((kappa >= 1.0) & (kappa <= kmax), np.maximum(kappa, 1.0) ** (-4.0 / 3.0), 0.0)
    out = np.empty((g.nz, g.ny, g.nx))
    for k0 in range(0, g.nz, chunk):
        k1 = min(g.nz, k0 + chunk)
        phase = rng.uniform(0.0, 2.0 * np.pi, size=(k1 - k0,) + amp.shape)
        spec = amp[None] * np.exp(1j * phase)
        f = np.fft.irfft2(spec, s=(g.ny, g.nx), axes=(1, 2))
        f *= std / f.std(axis=(1, 2), keepdims=True)
        out[k0:k1] = f
    return out


def _spectral_fields(rng, g: Grid):
    u = _spectral_field(rng, g, 2.0)
    v = _spectral_field(rng, g, 2.0)
    w = _spectral_field(rng, g, 0.5)
    w[g.nz - 1] = 0.0
    return u, v, w


def density_field(rng, g: Grid, amp: float = 0.2):
    """Density varying in all three directions around the grid's rho0:
    rho[k, j, i] = rho0_k (1 + amp (c_k f1 + (1 - c_k) f2)) with f1, f2 two
    sums of 8 low-wavenumber plane waves at the cell centres (as in
    mode_fields) scaled to max |f| = 1, and c_k = zc_k / H the height
    fraction, so |rho/rho0 - 1| <= amp (positive for amp < 1)."""
    xc, _, yc, _ = _staggered_coords(g)
    dz = np.asarray(g.dz, dtype=np.float64)
    zc = _zc(dz)
    c = zc / dz.sum()
    f1 = _mode_sum(rng, g, xc, yc)
    f2 = _mode_sum(rng, g, xc, yc)
    f1 /= np.abs(f1).max()
    f2 /= np.abs(f2).max()
    shape = (g.nz, g.ny, g.nx)
    rho = np.empty(shape)
    for k in range(g.nz):
        rho[k] = g.rho0[k] * (1.0 + amp * (c[k] * f1 + (1.0 - c[k]) * f2))
    return rho


C3_SHAPES = [(64, 64, 64), (128, 128, 96), (192, 192, 128), (256, 256, 128)]


def ensemble_members(count: int = 48, shapes=None, seed: int = 4000):
    """Member grids of the ensemble: sizes drawn with `seed`, member m uses
    seed + 1 + m for its dz ratio, rho0 scale height and fields."""
    shapes = C3_SHAPES if shapes is None else shapes
    pick = np.random.default_rng(seed).integers(0, len(shapes), size=count)
    out = []
    for mi, s in enumerate(pick):
        nx, ny, nz = shapes[s]
        rng = np.random.default_rng(seed + 1 + mi)
        ratio = rng.uniform(1.00, 1.02)
        hs = rng.uniform(6000.0, 10000.0)
        dz = 10.0 * ratio ** np.arange(nz, dtype=np.float64)
        g = Grid(nx, ny, nz, 25.0, 25.0, dz, exp_rho0(dz, hs))
        out.append((g, rng))
    return out


def make_workload(name: str, members: Optional[int] = None) -> Workload:
    """Build one named configuration. Fields are drawn in FP64; the mixed
    configurations are meant to be rounded to FP32 by the caller."""
    if name == "ensemble48":
        mem = []
        for g, rng in ensemble_members(48 if members is None else members):
            mem.append(Member(g, *mode_fields(rng, g)))
        return Workload(name, "mixed", mem, CONFIGS[name])
    g = make_grid(name)
    seed = {"32x32x32": 1000, "256x256x128": 2000, "1024x1024x256": 3000, "2048x2048x160": 5000,
            "4096x4096x64": 6000}[name]
    rng = np.random.default_rng(seed)
    if name == "32x32x32":
        fields = _small_fields(rng, g)
    elif name == "2048x2048x160":
        fields = _spectral_fields(rng, g)
    else:
        fields = mode_fields(rng, g)
    dtype = "f64" if name in ("32x32x32", "256x256x128") else "mixed"
    return Workload(name, dtype, [Member(g, *fields)], CONFIGS[name])


def random_grid(rng, nx: int, ny: int, nz: int, stretch=(1.0, 1.3),
                dx=None, dy=None) -> Grid:
    """Small test grid: random positive dz (ratio of neighbours within
    `stretch`), random positive rho0, random dx, dy."""
    dz = 5.0 + 20.0 * rng.random(nz)
    if stretch is not None:
        r = rng.uniform(*stretch)
        dz = 10.0 * r ** np.arange(nz) * rng.uniform(0.8, 1.2, size=nz)
    rho0 = rng.uniform(0.3, 1.5, size=nz)
    dx = rng.uniform(10.0, 60.0) if dx is None else dx
    dy = rng.uniform(10.0, 60.0) if dy is None else dy
    return Grid(nx, ny, nz, float(dx), float(dy), dz.astype(np.float64), rho0)


def random_fields(rng, g: Grid, lid: bool = True):
    shape = (g.nz, g.ny, g.nx)
    u = rng.standard_normal(shape)
    v = rng.standard_normal(shape)
    w = rng.standard_normal(shape)
    if lid:
        w[g.nz - 1] = 0.0
    return u, v, w
