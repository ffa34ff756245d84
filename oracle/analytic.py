"""Closed forms and brute-force sums used to pin the oracle -- TEST INFRASTRUCTURE.

None of these is the method; they are independent references for it.
"""
from __future__ import annotations

import numpy as np
import scipy.special

from .core import Grid


def sphere_potential(r: np.ndarray, M: float, R: float, G: float = 1.0) -> np.ndarray:
    """Uniform sphere of mass M and radius R: -G M / r outside,
    -G M (3 R^2 - r^2) / (2 R^3) inside."""
    r = np.asarray(r, dtype=np.float64)
    out = np.where(r >= R, -G * M / np.maximum(r, 1e-300), -G * M * (3.0 * R * R - r * r) / (2.0 * R ** 3))
    return out


def gaussian_mass(A: float, sigma: float) -> float:
    return A * (2.0 * np.pi) ** 1.5 * sigma ** 3


def gaussian_potential(r: np.ndarray, A: float, sigma: float, G: float = 1.0) -> np.ndarray:
    """rho = A exp(-r^2 / (2 sigma^2)) has potential -G M erf(r / (sqrt(2) sigma)) / r."""
    r = np.asarray(r, dtype=np.float64)
    M = gaussian_mass(A, sigma)
    small = r < 1e-12
    rs = np.where(small, 1.0, r)
    val = -G * M * scipy.special.erf(rs / (np.sqrt(2.0) * sigma)) / rs
    centre = -G * M * np.sqrt(2.0 / np.pi) / sigma
    return np.where(small, centre, val)


# integral over the unit cube [-1/2, 1/2]^3 of 1/|x|: the potential of a
# uniform cube at its centre is -G rho a^2 times this number
CUBE_SELF = 3.0 * np.log(2.0 + np.sqrt(3.0)) - np.pi / 2.0


def cell_centres(g: Grid):
    x = g.x0 + (np.arange(g.nx) + 0.5) * g.dx
    y = g.y0 + (np.arange(g.ny) + 0.5) * g.dx
    z = g.z0 + (np.arange(g.nz) + 0.5) * g.dx
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def ghost_points(g: Grid):
    """Ghost-cell centres as six (N, 3) arrays in the face order x-, x+, y-, y+, z-, z+,
    each face flattened in C order of its 2D shape ((nz,ny), (nz,nx), (ny,nx))."""
    x = g.x0 + (np.arange(g.nx) + 0.5) * g.dx
    y = g.y0 + (np.arange(g.ny) + 0.5) * g.dx
    z = g.z0 + (np.arange(g.nz) + 0.5) * g.dx
    xm, xp = g.x0 - 0.5 * g.dx, g.x0 + (g.nx + 0.5) * g.dx
    ym, yp = g.y0 - 0.5 * g.dx, g.y0 + (g.ny + 0.5) * g.dx
    zm, zp = g.z0 - 0.5 * g.dx, g.z0 + (g.nz + 0.5) * g.dx
    out = []
    Zf, Yf = np.meshgrid(z, y, indexing="ij")
    for xv in (xm, xp):
        out.append(np.stack([np.full(Zf.size, xv), Yf.ravel(), Zf.ravel()], 1))
    Zf, Xf = np.meshgrid(z, x, indexing="ij")
    for yv in (ym, yp):
        out.append(np.stack([Xf.ravel(), np.full(Zf.size, yv), Zf.ravel()], 1))
    Yf, Xf = np.meshgrid(y, x, indexing="ij")
    for zv in (zm, zp):
        out.append(np.stack([Xf.ravel(), Yf.ravel(), np.full(Yf.size, zv)], 1))
    return out


def legendre_multipole(g: Grid, rho: np.ndarray, pts: np.ndarray, lmax: int, G: float = 1.0,
                       origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Multipole potential by the Legendre addition theorem, brute force over
    cells: phi(x) = -G sum_j m_j sum_{l<=lmax} r_j^l / r^{l+1} P_l(cos gamma_j)."""
    X, Y, Z = cell_centres(g)
    o = np.asarray(origin, dtype=np.float64)
    src = np.stack([X.ravel() - o[0], Y.ravel() - o[1], Z.ravel() - o[2]], 1)
    m = np.asarray(rho, dtype=np.float64).ravel() * g.dx ** 3
    keep = m != 0
    src, m = src[keep], m[keep]
    rj = np.linalg.norm(src, axis=1)
    out = np.zeros(len(pts))
    for n, p in enumerate(np.asarray(pts, dtype=np.float64) - o):
        r = np.linalg.norm(p)
        with np.errstate(invalid="ignore", divide="ignore"):
            cg = np.where(rj > 0, src @ p / (np.maximum(rj, 1e-300) * r), 1.0)
        tot = 0.0
        for l in range(lmax + 1):
            tot += np.sum(m * rj ** l * scipy.special.eval_legendre(l, cg)) / r ** (l + 1)
        out[n] = -G * tot
    return out


def direct_sum_points(g: Grid, rho: np.ndarray, pts: np.ndarray, G: float = 1.0) -> np.ndarray:
    """Free-space potential of the cell masses at points outside every cell."""
    X, Y, Z = cell_centres(g)
    src = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    m = np.asarray(rho, dtype=np.float64).ravel() * g.dx ** 3
    keep = m != 0
    src, m = src[keep], m[keep]
    out = np.zeros(len(pts))
    for n, p in enumerate(np.asarray(pts, dtype=np.float64)):
        out[n] = -G * np.sum(m / np.linalg.norm(src - p, axis=1))
    return out


def direct_sum_cells(g: Grid, rho: np.ndarray, G: float = 1.0) -> np.ndarray:
    """Free-space potential at every cell centre of the piecewise-constant
    density: point masses for the other cells plus the exact uniform-cube
    self term -G rho_i dx^2 CUBE_SELF (tiny grids only)."""
    X, Y, Z = cell_centres(g)
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    r = np.asarray(rho, dtype=np.float64).ravel()
    m = r * g.dx ** 3
    out = np.zeros(len(pos))
    for n in range(len(pos)):
        d = np.linalg.norm(pos - pos[n], axis=1)
        d[n] = np.inf
        out[n] = -G * (np.sum(m / d) + r[n] * g.dx ** 2 * CUBE_SELF)
    return out.reshape(g.shape)
