"""The boundary study of Sec. 4 (Table I) on the GPU: around a 12^3 hydro grid,
Robin domains in the table's ratios (1 : 600/210 : 1200/210 at one cell size)
and the multipole Dirichlet boundary on the hydro grid, each relaxed by the
damped FP64 wave iteration to its steady state.  Each steady state is
compared with an independent sparse solve of the same discrete problem, then
the boundary errors in the hydro region (against the closed-form free-space
ghosts) must come in the paper's order."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import analytic, poisson
from oracle.core import Grid, boundary, moments, padded, set_faces
from test_gpu_parity import host, rel, to_dev
from test_oracle_table1 import _density, _free_space, _robin_matrix_v, _table

pytestmark = pytest.mark.gpu


def _relax(s, rho, dt, tol=1e-12, chunk=1000, max_chunks=60):
    r = to_dev(rho)
    for _ in range(max_chunks):
        s.step(r, 1.0, dt, chunk)
        if s.residual(r)[0] < tol:
            return host(s.potential()[0])
    raise AssertionError("no steady state within %d substeps" % (chunk * max_chunks))


def test_table1_domains_on_the_gpu(gpu_lib):
    t = _table()
    n0 = 12
    g0 = Grid.cube(n0)
    rho0 = _density(g0)
    P = padded(g0)
    set_faces(P, [_free_space(p).reshape(n0, n0) for p in analytic.ghost_points(g0)])
    ref = poisson.solve_dst(g0, rho0, 1.0, P)
    scale = np.max(np.abs(ref))

    def err(phi):
        return np.sqrt(np.mean((phi - ref) ** 2)) / scale

    errs = {}
    for size in "abc":
        n = 2 * int(round(n0 * t[size + "R05"]["nr"] / t["aR05"]["nr"] / 2))
        h = n * g0.dx / 2
        g = Grid(n, n, n, -h, -h, -h, g0.dx)
        rho = _density(g)
        want, info = spla.cg(-_robin_matrix_v(g), -4.0 * np.pi * rho.ravel(), rtol=1e-13, maxiter=20000)
        assert info == 0
        want = want.reshape(g.shape)
        s = gpu_lib.Solver(n, x0=(-h, -h, -h), dx=g0.dx, bc="robin", storage="f64",
                           eta=2.0 * np.sqrt(poisson.lambda_min(g)))
        got = _relax(s, rho, 0.4 * g0.dx)
        s.close()
        assert rel(got, want) < 1e-8, size
        o = (n - n0) // 2
        errs[size + "R"] = err(got[o:o + n0, o:o + n0, o:o + n0])
    s = gpu_lib.Solver(n0, bc="multipole", lmax=4, storage="f64", eta=2.0 * np.sqrt(poisson.lambda_min(g0)))
    got = _relax(s, rho0, 0.4 * g0.dx)
    s.close()
    PD = padded(g0)
    boundary(g0, moments(g0, rho0, 4), 4, 1.0, PD)
    assert rel(got, poisson.solve_dst(g0, rho0, 1.0, PD)) < 1e-8
    errs["aD"] = err(got)
    assert errs["aR"] > 5 * errs["aD"], errs
    assert errs["aR"] > errs["bR"] > errs["cR"], errs
    assert errs["cR"] < errs["aD"], errs
