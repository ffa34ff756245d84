"""Nested coarse outer level -- TEST INFRASTRUCTURE (see the package header).

Sec. 4 of the paper proposes moving the outer boundary far from the matter at
little cost, by an extended gravity-only grid and, as it notes, by nested
grids.  It gives no scheme for the latter; the reading taken here is:

* a coarse grid of twice the cell size covers the fine (hydrodynamics) grid
  and extends ``ext`` coarse cells beyond it on every side, with a local
  boundary (Robin or outgoing) at its own faces;
* per hydrodynamical step, the coarse source is the density averaged over the
  2 x 2 x 2 fine cells of each coarse cell, zero in the extension; the coarse
  grid advances ceil(nsub / 2) substeps spanning the same time nsub * dt;
* the fine ghosts are then the coarse potential interpolated trilinearly
  (between the nearest coarse cell centres) at the fine ghost centres, and
  stay fixed over the fine substeps, as the multipole ghosts do;
* the fine grid advances nsub substeps of dt.

More levels repeat this outwards: each level has twice the cell size of the
one inside it and extends ``ext`` of its cells beyond it; only the outermost
has the local boundary.  All levels share G, eta and the expansion centre
``origin`` (the Robin relation's centre).
"""
import numpy as np

from .analytic import ghost_points
from .core import Grid, Oracle
from .nn import restrict2


def coarse_grid(g: Grid, ext: int) -> Grid:
    """The grid of cell size 2 dx that covers g and ext coarse cells more on
    every side."""
    if g.nx % 2 or g.ny % 2 or g.nz % 2:
        raise ValueError("the fine grid needs even sizes")
    h = 2.0 * g.dx
    return Grid(g.nx // 2 + 2 * ext, g.ny // 2 + 2 * ext, g.nz // 2 + 2 * ext,
                g.x0 - ext * h, g.y0 - ext * h, g.z0 - ext * h, h)


def coarse_source(rho: np.ndarray, ext: int) -> np.ndarray:
    """2 x 2 x 2 means of rho, padded with ext zero cells on every side."""
    return np.pad(restrict2(np.asarray(rho, dtype=np.float64)), ext)


def trilinear(phi: np.ndarray, g: Grid, pts: np.ndarray) -> np.ndarray:
    """Cell-centred trilinear interpolation of phi (nz, ny, nx) on g at points
    (N, 3) given as (x, y, z).  Along each axis the point lies between centres
    i and i + 1 with weight w on i + 1 (u = (p - x0) / dx - 1/2, i = floor(u),
    w = u - i); every point must lie within the span of the centres."""
    pts = np.asarray(pts, dtype=np.float64)
    idx, wts = [], []
    for d, (lo, n) in enumerate(((g.x0, g.nx), (g.y0, g.ny), (g.z0, g.nz))):
        u = (pts[:, d] - lo) / g.dx - 0.5
        if np.any(u < -1e-12) or np.any(u > n - 1 + 1e-12):
            raise ValueError("point outside the span of the cell centres")
        i = np.clip(np.floor(u).astype(np.int64), 0, max(n - 2, 0))
        idx.append(i)
        wts.append(u - i)
    (ix, iy, iz), (wx, wy, wz) = idx, wts
    out = np.zeros(len(pts))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = (wz if dz else 1.0 - wz) * (wy if dy else 1.0 - wy) * (wx if dx else 1.0 - wx)
                out += w * phi[np.minimum(iz + dz, g.nz - 1), np.minimum(iy + dy, g.ny - 1),
                               np.minimum(ix + dx, g.nx - 1)]
    return out


def fine_ghosts(g: Grid, phi_c: np.ndarray, gc: Grid):
    """The six ghost faces of g (order x-, x+, y-, y+, z-, z+) interpolated
    from the coarse potential phi_c on gc."""
    shapes = ((g.nz, g.ny), (g.nz, g.ny), (g.nz, g.nx), (g.nz, g.nx), (g.ny, g.nx), (g.ny, g.nx))
    return [trilinear(phi_c, gc, p).reshape(s) for p, s in zip(ghost_points(g), shapes)]


class NestedOracle:
    """Fine grid g (bc "user") with its ghosts from coarser outer levels:
    level 1 has cell size 2 dx and extends ext of its cells beyond g, level 2
    the same around level 1, and so on up to ``levels - 1``; the outermost has
    the local boundary ``bc``, every inner level bc "user".  A hydro step of
    nsub substeps: the sources are restricted level by level, level l takes
    ceil(n_{l-1} / 2) substeps spanning nsub * dt (n_0 = nsub), and the levels
    are advanced from the outermost inwards, each inner one after its ghosts
    are interpolated from the level around it."""

    def __init__(self, g: Grid, ext: int, bc: str = "robin", G: float = 1.0, eta: float = 0.0,
                 origin=(0.0, 0.0, 0.0), storage: str = "f64", levels: int = 2):
        if ext < 1:
            raise ValueError("the coarse grid must extend at least one cell beyond the fine one")
        if levels < 2:
            raise ValueError("at least one coarse level")
        self.g, self.ext = g, ext
        self.grids = [g]
        for _ in range(levels - 1):
            self.grids.append(coarse_grid(self.grids[-1], ext))
        self.levels = [Oracle(q, G=G, eta=eta, bc=(bc if i == levels - 1 else "user"), origin=origin,
                              storage=storage) for i, q in enumerate(self.grids)]
        self.fine, self.coarse, self.gc = self.levels[0], self.levels[1], self.grids[1]

    def step(self, rho: np.ndarray, c: float, dt: float, nsub: int) -> None:
        srcs, counts = [np.asarray(rho, dtype=np.float64)], [nsub]
        for _ in range(1, len(self.levels)):
            srcs.append(coarse_source(srcs[-1], self.ext))
            counts.append((counts[-1] + 1) // 2)
        for lev in range(len(self.levels) - 1, -1, -1):
            if lev < len(self.levels) - 1:
                outer = self.levels[lev + 1]
                self.levels[lev].set_boundary(fine_ghosts(self.grids[lev], outer.potential()[0], self.grids[lev + 1]))
            self.levels[lev].step(srcs[lev], c, dt if lev == 0 else nsub * dt / counts[lev], counts[lev])

    def potential(self):
        return self.fine.potential()

    def accel(self):
        return self.fine.accel()
