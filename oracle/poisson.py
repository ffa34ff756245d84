"""The limit the method converges to: the discrete Dirichlet Poisson problem
L_h phi = 4 pi G rho (Eq. (1) with the 7-point Laplacian), ghost values fixed.
TEST INFRASTRUCTURE.

With the ghosts moved to the right-hand side the interior system is
A phi = b,  b = 4 pi G rho - (sum of adjacent ghosts) / dx^2,
A = (D_x + D_y + D_z) / dx^2, each D the 1D second-difference matrix with zero
Dirichlet ends.  D has eigenvectors sin(pi k (i+1) / (n+1)) and eigenvalues
-4 sin^2(pi k / (2 (n+1))), k = 1..n, so the type-I discrete sine transform
diagonalises A and inverts it exactly (up to rounding).
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.sparse
import scipy.sparse.linalg

from .core import Grid, interior


def ghost_sum(g: Grid, P: np.ndarray) -> np.ndarray:
    """Sum of the ghost neighbours of each interior cell (zero in the bulk)."""
    out = np.zeros(g.shape)
    out[:, :, 0] += P[1:-1, 1:-1, 0]
    out[:, :, -1] += P[1:-1, 1:-1, -1]
    out[:, 0, :] += P[1:-1, 0, 1:-1]
    out[:, -1, :] += P[1:-1, -1, 1:-1]
    out[0, :, :] += P[0, 1:-1, 1:-1]
    out[-1, :, :] += P[-1, 1:-1, 1:-1]
    return out


def rhs(g: Grid, rho: np.ndarray, G: float, P: np.ndarray) -> np.ndarray:
    return 4.0 * np.pi * G * np.asarray(rho, dtype=np.float64) - ghost_sum(g, P) / g.dx ** 2


def eigenvalues_1d(n: int, dx: float) -> np.ndarray:
    k = np.arange(1, n + 1)
    return -(4.0 / dx ** 2) * np.sin(np.pi * k / (2.0 * (n + 1))) ** 2


def lambda_min(g: Grid) -> float:
    """Smallest magnitude eigenvalue of -A (slowest discrete mode)."""
    return float(sum((4.0 / g.dx ** 2) * np.sin(np.pi / (2.0 * (n + 1))) ** 2 for n in (g.nx, g.ny, g.nz)))


def lambda_max(g: Grid) -> float:
    return float(sum((4.0 / g.dx ** 2) * np.sin(np.pi * n / (2.0 * (n + 1))) ** 2 for n in (g.nx, g.ny, g.nz)))


def solve_dst(g: Grid, rho: np.ndarray, G: float, P: np.ndarray) -> np.ndarray:
    """Interior solution of the discrete Dirichlet Poisson problem (compact)."""
    b = rhs(g, rho, G, P)
    lx = eigenvalues_1d(g.nx, g.dx)
    ly = eigenvalues_1d(g.ny, g.dx)
    lz = eigenvalues_1d(g.nz, g.dx)
    lam = lz[:, None, None] + ly[None, :, None] + lx[None, None, :]
    bh = scipy.fft.dstn(b, type=1)
    return scipy.fft.idstn(bh / lam, type=1)


def solve_dense(g: Grid, rho: np.ndarray, G: float, P: np.ndarray) -> np.ndarray:
    """Same problem by a direct sparse LU factorisation (small grids only)."""
    assert g.nx * g.ny * g.nz <= 40 ** 3

    def d1(n):
        return scipy.sparse.diags([np.ones(n - 1), -2.0 * np.ones(n), np.ones(n - 1)], [-1, 0, 1])

    Ix, Iy, Iz = (scipy.sparse.identity(n) for n in (g.nx, g.ny, g.nz))
    # x fastest: kron(z, kron(y, x))
    A = (scipy.sparse.kron(Iz, scipy.sparse.kron(Iy, d1(g.nx)))
         + scipy.sparse.kron(Iz, scipy.sparse.kron(d1(g.ny), Ix))
         + scipy.sparse.kron(d1(g.nz), scipy.sparse.kron(Iy, Ix))) / g.dx ** 2
    b = rhs(g, rho, G, P).ravel()
    x = scipy.sparse.linalg.spsolve(A.tocsc(), b)
    return x.reshape(g.shape)


def with_solution(g: Grid, P: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Padded copy of P with its interior replaced by phi."""
    Q = P.copy()
    interior(Q)[...] = phi
    return Q


def mean_relative_error(phi_h: np.ndarray, phi_p: np.ndarray) -> float:
    """The paper's average relative error (Sec. 4, Eq. 6): the root mean square,
    over the volume, of the pointwise relative difference (Eq. 5)
    (phi_h - phi_p) / phi_p between the wave-equation potential and the
    Poisson solution of the same density.  On a uniform grid the volume
    integrals are sums over cells with equal weights."""
    h = np.asarray(phi_h, dtype=np.float64)
    p = np.asarray(phi_p, dtype=np.float64)
    d = (h - p) / p
    return float(np.sqrt(np.mean(d * d)))
