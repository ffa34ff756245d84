"""The boundary study of Sec. 4 (Table I) as a pin of the oracle's outer
boundaries (no GPU).

The fixture ``golden/table1_models.txt`` holds the paper's Table I.  Its rows
are first checked against what the paper's text states about them: the wider
domains keep the cell size, and the smallest and largest Robin domains have
5.88e4 and 1.92e6 zones.  The domain ratios of the table (600/210 and
1200/210 at one cell size) then set three 3D domains around one hydro grid,
and the error of the Robin boundary in the hydro region must fall in the
paper's order: Robin at the hydro faces is the worst, the multipole Dirichlet
boundary on the same grid is several times better, and the widest Robin
domain is better still (Sec. 4 reports about 10%, 0.1% and 0.003%).  The
error is measured against the same discrete problem on the hydro grid with
the closed-form free-space potential as Dirichlet ghosts, so that only the
boundary's error is counted, not the discretisation's.
"""
import os

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import analytic, poisson
from oracle.core import Grid, boundary, moments, padded, set_faces
from test_oracle_bc import _robin_matrix

HERE = os.path.dirname(os.path.abspath(__file__))


def _table():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "table1_models.txt")):
        if line.startswith("#") or not line.strip():
            continue
        m, r, z, nr, nz, bc, kg = line.split()
        rows[m] = dict(r=float(r), z=float(z), nr=int(nr), nz=int(nz), bc=bc, kg=int(kg))
    return rows


def test_table1_agrees_with_the_text():
    t = _table()
    assert len(t) == 7
    for m in t.values():
        # one resolution for every model: 3e9 cm in r and z
        assert abs(m["r"] / m["nr"] - 3.0e9) < 1e-3 * 3.0e9
        assert abs(m["z"] / m["nz"] - 3.0e9) < 1e-3 * 3.0e9
    assert t["aR05"]["nr"] * t["aR05"]["nz"] == 58800
    assert t["cR05"]["nr"] * t["cR05"]["nz"] == 1920000
    assert [k for k, m in t.items() if m["bc"] == "Dirichlet"] == ["aD05"]
    for size in "abc":
        a, b = t[size + "R05"], t[size + "R20"]
        assert (a["r"], a["z"], a["nr"], a["nz"], a["kg"], b["kg"]) == (b["r"], b["z"], b["nr"], b["nz"], 5, 20)


def _robin_matrix_v(g: Grid):
    """-L_h with the Robin ghosts phi_g = (r_i / r_g) phi_i eliminated about
    the origin, built with array operations (the loop form is
    ``test_oracle_bc._robin_matrix``; the two are compared below)."""
    x, y, z = g.centres()
    Z, Y, X = np.meshgrid(z[1:-1], y[1:-1], x[1:-1], indexing="ij")
    R = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    h2 = 1.0 / g.dx ** 2
    idx = np.arange(g.nx * g.ny * g.nz).reshape(g.shape)
    diag = np.full(g.shape, -6.0 * h2)
    rows, cols = [], []
    for ax, n in ((2, g.nx), (1, g.ny), (0, g.nz)):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax], hi[ax] = slice(0, n - 1), slice(1, n)
        rows += [idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()]
        cols += [idx[tuple(hi)].ravel(), idx[tuple(lo)].ravel()]
    for ax, (c, n) in zip((2, 1, 0), ((x, g.nx), (y, g.ny), (z, g.nz))):
        for side, gi in ((0, 0), (n - 1, n + 1)):
            s = [slice(None)] * 3
            s[ax] = side
            s = tuple(s)
            p = [X[s], Y[s], Z[s]]
            p[2 - ax] = np.full_like(p[2 - ax], c[gi])
            diag[s] += h2 * R[s] / np.sqrt(p[0] ** 2 + p[1] ** 2 + p[2] ** 2)
    r = np.concatenate(rows + [idx.ravel()])
    cc = np.concatenate(cols + [idx.ravel()])
    v = np.concatenate([np.full(len(a), h2) for a in rows] + [diag.ravel()])
    N = g.nx * g.ny * g.nz
    return sp.csr_matrix((v, (r, cc)), shape=(N, N))


def test_array_built_robin_matrix_matches_the_loop_form():
    g = Grid(7, 5, 6, -0.7, -0.5, -0.6, 0.2)
    assert abs(_robin_matrix_v(g) - _robin_matrix(g, (0.0, 0.0, 0.0))).max() < 1e-12


BLOBS = (((0.35, 0.1, 0.0), 1.0, 0.25), ((-0.3, -0.2, 0.15), 0.6, 0.2))


def _density(g: Grid):
    x, y, z = g.centres()
    Z, Y, X = np.meshgrid(z[1:-1], y[1:-1], x[1:-1], indexing="ij")
    rho = np.zeros(g.shape)
    for (cx, cy, cz), a0, sg in BLOBS:
        rho += a0 * np.exp(-0.5 * ((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2) / sg ** 2)
    return rho


def _free_space(pts):
    v = np.zeros(len(pts))
    for (cx, cy, cz), a0, sg in BLOBS:
        r = np.sqrt((pts[:, 0] - cx) ** 2 + (pts[:, 1] - cy) ** 2 + (pts[:, 2] - cz) ** 2)
        v += analytic.gaussian_potential(r, a0, sg)
    return v


def test_table1_domains_order_the_boundary_errors():
    t = _table()
    n0 = 12
    g0 = Grid.cube(n0)
    rho0 = _density(g0)
    shapes = ((n0, n0),) * 6
    P = padded(g0)
    set_faces(P, [_free_space(p).reshape(s) for p, s in zip(analytic.ghost_points(g0), shapes)])
    ref = poisson.solve_dst(g0, rho0, 1.0, P)
    scale = np.max(np.abs(ref))

    def err(phi):
        return np.sqrt(np.mean((phi - ref) ** 2)) / scale

    errs = {}
    for size in "abc":
        ratio = t[size + "R05"]["nr"] / t["aR05"]["nr"]
        n = 2 * int(round(n0 * ratio / 2))
        g = Grid(n, n, n, -n * g0.dx / 2, -n * g0.dx / 2, -n * g0.dx / 2, g0.dx)
        A = _robin_matrix_v(g)
        phi, info = spla.cg(-A, -4.0 * np.pi * _density(g).ravel(), rtol=1e-12, maxiter=20000)
        assert info == 0
        o = (n - n0) // 2
        errs[size + "R"] = err(phi.reshape(g.shape)[o:o + n0, o:o + n0, o:o + n0])
    PD = padded(g0)
    boundary(g0, moments(g0, rho0, 4), 4, 1.0, PD)
    errs["aD"] = err(poisson.solve_dst(g0, rho0, 1.0, PD))
    assert errs["aR"] > 5 * errs["aD"], errs
    assert errs["aR"] > errs["bR"] > errs["cR"], errs
    assert errs["cR"] < errs["aD"], errs
