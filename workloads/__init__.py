"""Seeded synthetic inputs shared by the oracle checks and the HIP path.

This module holds input generators only -- none of the method's arithmetic.
Densities are evaluated in FP64 at cell centres and then cast to the storage
dtype.  Workload shapes follow the paper's setting of a smooth
self-gravitating density on a 3D Cartesian grid (Sec. 2): a uniform sphere,
single Gaussians and mixtures of Gaussian blobs (stand-ins for the stellar
models, which need a hydro code and are not reproduced).

Blob recipe (the paper gives none):
  rng = numpy.random.default_rng(seed)
  centres = rng.uniform(-0.6, 0.6, (K, 3)); sigma = rng.uniform(0.05, 0.2, K);
  amplitude = rng.lognormal(0.0, 1.0, K), drawn in that order;
  rho(x) = sum_k A_k exp(-|x - c_k|^2 / (2 sigma_k^2)).
A rigid rotation by angle theta about +z (counter-clockwise) moves the centres.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Blobs:
    centres: np.ndarray  # (K, 3)
    sigma: np.ndarray  # (K,)
    amp: np.ndarray  # (K,)

    def rotated(self, theta: float) -> "Blobs":
        c, s = np.cos(theta), np.sin(theta)
        x, y, z = self.centres[:, 0], self.centres[:, 1], self.centres[:, 2]
        cen = np.stack([c * x - s * y, s * x + c * y, z], 1)
        return Blobs(cen, self.sigma, self.amp)


def blob_params(seed: int, k: int) -> Blobs:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-0.6, 0.6, (k, 3))
    sigma = rng.uniform(0.05, 0.2, k)
    amp = rng.lognormal(0.0, 1.0, k)
    return Blobs(centres, sigma, amp)


def axis(n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    dx = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * dx


def blob_density_axes(x: np.ndarray, y: np.ndarray, z: np.ndarray, blobs: Blobs, dtype=np.float64) -> np.ndarray:
    """rho at the cell centres x (nx,), y (ny,), z (nz,); shape (nz, ny, nx).
    Each Gaussian is a product of three 1D factors."""
    rho = np.zeros((len(z), len(y), len(x)))
    for c, s, a in zip(blobs.centres, blobs.sigma, blobs.amp):
        fx = np.exp(-((x - c[0]) ** 2) / (2 * s * s))
        fy = np.exp(-((y - c[1]) ** 2) / (2 * s * s))
        fz = np.exp(-((z - c[2]) ** 2) / (2 * s * s))
        rho += a * fz[:, None, None] * (fy[:, None] * fx[None, :])[None, :, :]
    return rho.astype(dtype)


def centred_axes(shape, dx: float):
    """Cell-centre axes of a (nz, ny, nx) box of cell size dx centred on the origin."""
    nz, ny, nx = shape
    return tuple((np.arange(m) + 0.5) * dx - 0.5 * m * dx for m in (nx, ny, nz))


def blob_density(n, blobs: Blobs, lo: float = -1.0, hi: float = 1.0, dtype=np.float64) -> np.ndarray:
    """rho on an n^3 (or (nz,ny,nx) tuple) cell-centred grid with lower corner lo
    on every axis and dx = (hi - lo) / nx, shape (nz, ny, nx)."""
    nz, ny, nx = (n, n, n) if np.isscalar(n) else n
    dx = (hi - lo) / nx
    x = lo + (np.arange(nx) + 0.5) * dx
    y = lo + (np.arange(ny) + 0.5) * dx
    z = lo + (np.arange(nz) + 0.5) * dx
    return blob_density_axes(x, y, z, blobs, dtype)


def blob_density_torch(n: int, blobs: Blobs, device, dtype, lo: float = -1.0, hi: float = 1.0):
    """Same density built on a torch device (FP64 arithmetic, then cast)."""
    import torch

    dx = (hi - lo) / n
    ax = lo + (torch.arange(n, device=device, dtype=torch.float64) + 0.5) * dx
    rho = torch.zeros((n, n, n), device=device, dtype=torch.float64)
    for c, s, a in zip(blobs.centres, blobs.sigma, blobs.amp):
        f = [torch.exp(-((ax - float(cc)) ** 2) / (2 * float(s) ** 2)) for cc in c]
        rho += float(a) * f[2][:, None, None] * (f[1][:, None] * f[0][None, :])[None]
    return rho.to(dtype)


def sphere_density(n: int, radius: float = 0.25, rho0: float = 1.0, lo: float = -1.0, hi: float = 1.0,
                   dtype=np.float64) -> np.ndarray:
    """Uniform sphere point-sampled at cell centres, strict r < radius."""
    a = axis(n, lo, hi)
    Z, Y, X = np.meshgrid(a, a, a, indexing="ij")
    r2 = X * X + Y * Y + Z * Z
    return np.where(r2 < radius * radius, rho0, 0.0).astype(dtype)


def gaussian_density(n: int, sigma: float = 0.1, amp: float = 1.0, centre=(0.0, 0.0, 0.0),
                     lo: float = -1.0, hi: float = 1.0, dtype=np.float64) -> np.ndarray:
    b = Blobs(np.asarray([centre], dtype=np.float64), np.asarray([sigma]), np.asarray([amp]))
    return blob_density(n, b, lo, hi, dtype)


def random_field(shape, seed: int, lo: float = -1.0, hi: float = 1.0, dtype=np.float64) -> np.ndarray:
    """Uniform random values, for parity checks that need no structure."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, shape).astype(dtype)


@dataclass(frozen=True)
class BatchSpec:
    sizes: tuple  # per-grid N (cube N^3)
    nblobs: tuple  # per-grid blob count
    seeds: tuple  # per-grid blob seed


def batch_spec(seed: int = 2, count: int = 64, sizes=tuple(range(32, 161, 16)),
               kmin: int = 4, kmax: int = 12, seed_base: int = 1000) -> BatchSpec:
    """Uneven batch of cube grids: N_g drawn from `sizes`, K_g from [kmin, kmax],
    blob seeds seed_base + g."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.asarray(sizes), count)
    k = rng.integers(kmin, kmax + 1, count)
    return BatchSpec(tuple(int(v) for v in n), tuple(int(v) for v in k),
                     tuple(seed_base + g for g in range(count)))


def warmstart_blobs(seed: int) -> Blobs:
    """Density of the warm-start study: K in {4..12} blobs, K drawn from its own
    seeded stream, then the blob recipe above with the sample's seed."""
    k = int(np.random.default_rng(seed + 7_000_000).integers(4, 13))
    return blob_params(seed, k)
