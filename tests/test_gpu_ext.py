"""The extended gravity-only grid (Sec. 4): the wave equation solved on a grid
wider than the hydrodynamics region, the extension taken as vacuum.  Parity
with the oracle run on the zero-padded density, and the paper's finding that
with a local (Robin) boundary the error falls as the region widens, roughly
inversely with the number of zones."""
import math

import numpy as np
import pytest

import workloads
from oracle import core, poisson
from oracle.core import Grid, Oracle, interior, padded
from test_gpu_parity import F32_TOL, F64_TOL, dens, grid_of, host, rel, rel_phidot, rel_vec, to_dev

pytestmark = pytest.mark.gpu


def _outer(g: Grid, e: int) -> Grid:
    return Grid(g.nx + 2 * e, g.ny + 2 * e, g.nz + 2 * e, g.x0 - e * g.dx, g.y0 - e * g.dx, g.z0 - e * g.dx, g.dx)


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("bc", ["outgoing", "robin", "multipole"])
def test_extended_grid_matches_oracle_on_padded_density(gpu_lib, storage, bc):
    shape = (12, 10, 14)
    e = 5
    g = grid_of(shape)
    rho = dens(shape, 40, storage)
    s = gpu_lib.ExtendedSolver(shape, e, x0=(g.x0, g.y0, g.z0), dx=g.dx, bc=bc, storage=storage, eta=1.5)
    o = Oracle(_outer(g, e), eta=1.5, bc=bc)
    rp = np.pad(rho.astype(np.float64), e)
    for nsub in (3, 17):
        s.step(to_dev(rho), 1.0, 0.4 * g.dx, nsub)
        o.step(rp, 1.0, 0.4 * g.dx, nsub)
    tol = F64_TOL if storage == "f64" else F32_TOL
    phi, pd = s.potential()
    ophi, opd = o.potential()
    sl = (slice(e, e + shape[0]), slice(e, e + shape[1]), slice(e, e + shape[2]))
    assert tuple(phi.shape) == shape
    assert rel(host(phi), ophi[sl]) < tol
    assert rel_phidot(host(pd), opd[sl], ophi[sl], 0.4 * g.dx) < tol
    assert rel_vec([host(a) for a in s.accel()], [b[sl] for b in o.accel()]) < tol
    # embed writes zeros around the hydrodynamics region
    import torch
    out = torch.full(s.solver.shape, 7.0, dtype=s.dtype, device="cuda")
    s.embed(to_dev(rho), out)
    assert np.array_equal(host(out), rp.astype(rho.dtype).astype(np.float64))


def test_robin_error_falls_with_extension(gpu_lib):
    """Robin boundary on the hydrodynamics box widened by e cells of vacuum,
    converged (damped); error against the Dirichlet-multipole Poisson solution
    of the box (the paper's aD05 reference).  It falls monotonically, and the
    product error x zones stays within a factor 1.6 (inverse proportionality,
    Sec. 4)."""
    n = 24
    g = Grid.cube(n)
    x, y, z = workloads.centred_axes((n, n, n), g.dx)
    rho = workloads.blob_density_axes(x, y, z, workloads.blob_params(3, 6), dtype=np.float64)
    P = padded(g)
    core.boundary(g, core.moments(g, rho, 4), 4, 1.0, P)
    ref = poisson.solve_dst(g, rho, 1.0, P)
    errs, zones = [], []
    for e in (0, 8, 16):
        half = 1.0 + e * g.dx
        eta = 2.0 * math.sqrt(0.66) * math.pi / (2.0 * half)  # slowest Robin mode of the box, critically damped
        s = gpu_lib.ExtendedSolver(n, e, dx=g.dx, bc="robin", storage="f64", eta=eta)
        steps = int(60.0 / eta / (0.4 * g.dx))
        s.step(to_dev(rho), 1.0, 0.4 * g.dx, steps)
        assert s.residual(to_dev(rho))[0] < 1e-9
        phi = host(s.potential(with_phidot=False)[0])
        errs.append(float(np.mean(np.abs(phi - ref)) / np.mean(np.abs(ref))))
        zones.append((n + 2 * e) ** 3)
    assert errs[0] > errs[1] > errs[2], errs
    prod = [a * b for a, b in zip(errs, zones)]
    assert max(prod) / min(prod) < 1.6, (errs, prod)


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("shape,e", [((3, 5, 7), 0), ((3, 5, 7), 1), ((9, 4, 70), 33), ((20, 18, 129), 2)])
def test_embed_extract_round_trip(gpu_lib, storage, shape, e):
    """hgs_embed writes every outer cell (zeros around the region), and
    hgs_extract returns the region bitwise, for rows shorter and longer than
    a wave and extensions wider than the region."""
    import torch

    nz, ny, nx = shape
    rng = np.random.default_rng(41)
    a = rng.normal(size=shape).astype(np.float64 if storage == "f64" else np.float32)
    g = grid_of(shape)
    s = gpu_lib.ExtendedSolver(shape, e, x0=(g.x0, g.y0, g.z0), dx=g.dx, storage=storage)
    outer = torch.full(tuple(v + 2 * e for v in shape), float("nan"), dtype=s.dtype, device="cuda")
    s.embed(to_dev(a), outer)
    assert np.array_equal(host(outer), np.pad(a.astype(np.float64), e))
    assert np.array_equal(host(s.extract(outer)), a)
