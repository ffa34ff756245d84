"""The nested coarse outer level on the GPU (Sec. 4 names nested grids as a way
to move the outer boundary out): the coarse source and the interpolated fine
ghosts against the oracle's, and the two-level step against the oracle's
NestedOracle over several hydro steps (odd and even substep counts), for the
Robin and outgoing rules at the coarse faces."""
import numpy as np
import pytest

from oracle.core import Grid
from oracle.nested import NestedOracle, coarse_grid, coarse_source, fine_ghosts
from test_gpu_parity import F32_TOL, F64_TOL, corner, dens, grid_of, host, npdt, rel, rel_vec, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("shape,ext", [((8, 6, 10), 0), ((8, 6, 10), 3), ((2, 130, 4), 1), ((64, 64, 64), 8)])
def test_nest_source_matches_oracle(gpu_lib, storage, shape, ext):
    import torch

    rho = np.random.default_rng(51).uniform(0.0, 2.0, shape).astype(npdt(storage))
    nz, ny, nx = shape
    out = torch.full((nz // 2 + 2 * ext, ny // 2 + 2 * ext, nx // 2 + 2 * ext), float("nan"),
                     dtype=torch.float64 if storage == "f64" else torch.float32, device="cuda")
    code = gpu_lib.HGS_F64 if storage == "f64" else gpu_lib.HGS_F32
    L = gpu_lib.library()
    r = to_dev(rho)
    assert L.hgs_nest_source(r.data_ptr(), nx, ny, nz, ext, out.data_ptr(), code, None) == gpu_lib.HGS_OK
    want = coarse_source(rho.astype(np.float64), ext)
    tol = 1e-15 if storage == "f64" else 1e-7
    assert rel(host(out), want) <= tol


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("shape,ext", [((12, 10, 14), 1), ((12, 10, 14), 3), ((6, 40, 300), 2)])
def test_nest_ghosts_match_oracle(gpu_lib, storage, shape, ext):
    g = grid_of(shape)
    gc = coarse_grid(g, ext)
    phi_c = np.random.default_rng(52).normal(size=gc.shape).astype(npdt(storage))
    s = gpu_lib.NestedSolver(shape, ext, x0=corner(shape), dx=g.dx, storage=storage)
    got = host(s.fine_ghosts(to_dev(phi_c)))
    want = gpu_lib.faces_to_flat(fine_ghosts(g, phi_c.astype(np.float64), gc))
    tol = 1e-14 if storage == "f64" else 1e-7
    assert rel(got, want) <= tol
    s.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("bc", ["robin", "outgoing"])
def test_nested_solver_matches_oracle(gpu_lib, storage, bc):
    shape, ext = (12, 10, 14), 3
    g = grid_of(shape)
    rho = dens(shape, 53, storage)
    s = gpu_lib.NestedSolver(shape, ext, x0=corner(shape), dx=g.dx, bc=bc, storage=storage, eta=1.5)
    o = NestedOracle(g, ext, bc=bc, eta=1.5)
    dt = 0.4 * g.dx
    for nsub in (4, 5, 4, 8):
        s.step(to_dev(rho), 1.0, dt, nsub)
        o.step(rho.astype(np.float64), 1.0, dt, nsub)
    tol = F64_TOL if storage == "f64" else F32_TOL
    phi, _ = s.potential()
    assert rel(host(phi), o.potential()[0]) < tol
    assert rel_vec([host(a) for a in s.accel()], o.accel()) < tol
    s.close()


def test_nested_full_size_256_f32(gpu_lib):
    """The benchmarked nested configuration: 256^3 FP32 fine grid, the 8-blob
    density, Robin 16 coarse cells beyond it (160^3 coarse), 4 substeps per
    hydro step at the default fused depth, from a smooth non-zero start on
    both levels, two hydro steps against the FP64 oracle over every cell."""
    import torch

    import workloads

    n, ext = 256, 16
    g = Grid.cube(n)
    rho = workloads.blob_density_torch(n, workloads.blob_params(0, 8), "cuda", torch.float32)
    s = gpu_lib.NestedSolver(n, ext, bc="robin", storage="f32", eta=0.0)
    o = NestedOracle(g, ext, bc="robin", eta=0.0)
    dt = 0.4 * g.dx

    def smooth(grid):
        x, y, z = (c[1:-1] for c in grid.centres())
        r2 = z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2
        return -1.0 / np.sqrt(r2 + 0.09)

    for lev, olev, h in ((s.fine, o.fine, dt), (s.coarse, o.coarse, 2.0 * dt)):  # the coarse step is 2 dt
        p0 = smooth(olev.g).astype(np.float32)
        lev.set_state(to_dev(p0), None, h)
        olev.set_state(p0.astype(np.float64), None, h)
    r64 = host(rho)
    for _ in range(2):
        s.step(rho, 1.0, dt, 4)
        o.step(r64, 1.0, dt, 4)
    assert rel(host(s.potential()[0]), o.potential()[0]) < F32_TOL
    assert rel_vec([host(a) for a in s.accel()], o.accel()) < F32_TOL
    s.close()


def test_nested_converges_to_composite_steady_state(gpu_lib):
    """Damped, the two-level GPU step settles on the composite steady state
    built from independent direct solves (a sparse Robin solve on the coarse
    grid, a DST-I solve on the fine grid with the interpolated ghosts)."""
    from test_oracle_nested import _composite_steady_state

    shape, ext = (12, 10, 14), 3
    g = grid_of(shape)
    origin = (0.05, -0.03, 0.02)
    rho = dens(shape, 54, "f64")
    phi_ref, gc, A = _composite_steady_state(g, ext, rho, origin)
    lam_min = float(np.linalg.eigvalsh(-A.toarray())[0])
    s = gpu_lib.NestedSolver(shape, ext, x0=corner(shape), dx=g.dx, bc="robin", storage="f64",
                             eta=2.0 * np.sqrt(lam_min), origin=origin)
    r = to_dev(rho)
    for _ in range(200):
        s.step(r, 1.0, 0.4 * g.dx, 8)
    assert rel(host(s.potential()[0]), phi_ref) < 1e-8
    s.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_three_levels_match_oracle(gpu_lib, storage):
    """Three levels (dx, 2 dx, 4 dx), the outgoing rule at the outermost
    faces, odd and even substep counts, against the oracle's three-level step."""
    shape, ext = (16, 12, 20), 2
    g = grid_of(shape)
    rho = dens(shape, 55, storage)
    s = gpu_lib.NestedSolver(shape, ext, x0=corner(shape), dx=g.dx, bc="outgoing", storage=storage, eta=1.0,
                             levels=3)
    o = NestedOracle(g, ext, bc="outgoing", eta=1.0, levels=3)
    assert [t.shape for t in s.solvers] == [q.shape for q in o.grids]
    dt = 0.4 * g.dx
    for nsub in (4, 5, 8, 3):
        s.step(to_dev(rho), 1.0, dt, nsub)
        o.step(rho.astype(np.float64), 1.0, dt, nsub)
    tol = F64_TOL if storage == "f64" else F32_TOL
    assert rel(host(s.potential()[0]), o.potential()[0]) < tol
    assert rel_vec([host(a) for a in s.accel()], o.accel()) < tol
    s.close()
