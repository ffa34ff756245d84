"""Pins of the oracle's nested coarse outer level (no GPU).

The interpolation is pinned by exactness on affine fields and at the coarse
centres, the coarse source by mass conservation, the damped nested iteration
by the composite steady state built from independent direct solves (a sparse
Robin solve on the coarse grid, then a DST-I Dirichlet solve on the fine grid
with the interpolated ghosts), and the scheme as a whole by the property it is
for (Sec. 4): a boundary moved further out gives a potential closer to the
free-space one.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import analytic, poisson
from oracle.core import Grid, padded, set_faces
from oracle.nested import NestedOracle, coarse_grid, coarse_source, fine_ghosts, trilinear
from test_oracle_bc import _robin_matrix


def test_trilinear_exact_on_affine_fields():
    gc = Grid(7, 6, 9, -1.3, -0.7, -1.1, 0.3)
    x, y, z = (c[1:-1] for c in gc.centres())
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    a, b, c, d = 0.7, -1.9, 0.4, 2.3
    phi = a + b * X + c * Y + d * Z
    rng = np.random.default_rng(5)
    pts = np.stack([rng.uniform(x[0], x[-1], 500), rng.uniform(y[0], y[-1], 500), rng.uniform(z[0], z[-1], 500)], 1)
    want = a + b * pts[:, 0] + c * pts[:, 1] + d * pts[:, 2]
    assert np.max(np.abs(trilinear(phi, gc, pts) - want)) < 1e-12
    # at the centres themselves (the last centre included) it returns the values
    cen = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    phi2 = rng.normal(size=gc.shape)
    assert np.max(np.abs(trilinear(phi2, gc, cen) - phi2.ravel())) < 1e-12
    with pytest.raises(ValueError):
        trilinear(phi, gc, np.array([[x[0] - 0.01, y[0], z[0]]]))


def test_coarse_source_conserves_mass():
    g = Grid(8, 6, 10, -1.0, -0.75, -1.25, 0.25)
    rho = np.random.default_rng(6).uniform(0.0, 2.0, g.shape)
    rc = coarse_source(rho, 3)
    gc = coarse_grid(g, 3)
    assert rc.shape == gc.shape
    assert abs(rc.sum() * gc.dx ** 3 - rho.sum() * g.dx ** 3) < 1e-12 * rho.sum() * g.dx ** 3
    assert np.all(rc[:3] == 0) and np.all(rc[:, :, -3:] == 0)
    # the coarse grid's cells line up with 2 x 2 x 2 blocks of fine cells
    assert gc.x0 + 3 * gc.dx == g.x0 and gc.z0 + 3 * gc.dx == g.z0


def _composite_steady_state(g, ext, rho, origin):
    """Coarse Robin steady state by a sparse solve, fine Dirichlet steady state
    by DST-I with the ghosts interpolated from it."""
    gc = coarse_grid(g, ext)
    A = _robin_matrix(gc, origin)
    phi_c = spla.spsolve(A.tocsc(), 4.0 * np.pi * coarse_source(rho, ext).ravel()).reshape(gc.shape)
    P = padded(g)
    set_faces(P, fine_ghosts(g, phi_c, gc))
    return poisson.solve_dst(g, rho, 1.0, P), gc, A


def test_damped_nested_iteration_reaches_the_composite_steady_state():
    g = Grid(12, 10, 14, -1.0, -10 / 12, -14 / 12, 2.0 / 12)
    origin = (0.05, -0.03, 0.02)
    x, y, z = (c[1:-1] for c in g.centres())
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    rho = np.exp(-0.5 * ((X - 0.1) ** 2 + (Y + 0.05) ** 2 + Z ** 2) / 0.2 ** 2)
    ext = 3
    phi_ref, gc, A = _composite_steady_state(g, ext, rho, origin)
    lam_min = float(np.linalg.eigvalsh(-A.toarray())[0])
    o = NestedOracle(g, ext, bc="robin", eta=2.0 * np.sqrt(lam_min), origin=origin)
    dt = 0.4 * g.dx
    for _ in range(200):
        o.step(rho, 1.0, dt, 8)
    phi = o.potential()[0]
    assert np.max(np.abs(phi - phi_ref)) < 1e-9 * np.max(np.abs(phi_ref))


def test_three_levels_reach_their_composite_steady_state():
    """Three levels (cell sizes dx, 2 dx, 4 dx): the damped iteration settles
    on a sparse Robin solve of the outermost level, then DST-I solves of the
    middle and fine levels, each with ghosts interpolated from the level
    around it."""
    g = Grid.cube(16)
    origin = (0.0, 0.0, 0.0)
    X, Y, Z = analytic.cell_centres(g)
    rho = np.exp(-0.5 * ((X - 0.2) ** 2 + (Y + 0.1) ** 2 + Z ** 2) / 0.25 ** 2)
    ext = 2
    g1 = coarse_grid(g, ext)
    g2 = coarse_grid(g1, ext)
    r1 = coarse_source(rho, ext)
    r2 = coarse_source(r1, ext)
    A = _robin_matrix(g2, origin)
    phi2 = spla.spsolve(A.tocsc(), 4.0 * np.pi * r2.ravel()).reshape(g2.shape)
    P1 = padded(g1)
    set_faces(P1, fine_ghosts(g1, phi2, g2))
    phi1 = poisson.solve_dst(g1, r1, 1.0, P1)
    P0 = padded(g)
    set_faces(P0, fine_ghosts(g, phi1, g1))
    phi_ref = poisson.solve_dst(g, rho, 1.0, P0)
    lam_min = float(np.linalg.eigvalsh(-A.toarray())[0])
    o = NestedOracle(g, ext, bc="robin", eta=2.0 * np.sqrt(lam_min), origin=origin, levels=3)
    assert [q.nx for q in o.grids] == [16, 12, 10]
    dt = 0.4 * g.dx
    for _ in range(150):
        o.step(rho, 1.0, dt, 8)
    phi = o.potential()[0]
    assert np.max(np.abs(phi - phi_ref)) < 1e-9 * np.max(np.abs(phi_ref))


def test_outer_boundary_further_out_is_closer_to_free_space():
    """Sec. 4: the error of a local boundary falls as it moves away from the
    matter.  Two Gaussians off the expansion centre (so that the monopole
    fall-off the Robin relation assumes is wrong at the faces) on a 24^3 fine
    grid: the composite steady state against the closed-form free-space
    potential, for coarse extensions of 2, 4 and 8 cells, against the fine
    grid with the Robin boundary at its own faces."""
    g = Grid.cube(24)
    X, Y, Z = analytic.cell_centres(g)
    blobs = (((0.35, 0.1, 0.0), 1.0, 0.2), ((-0.3, -0.2, 0.15), 0.6, 0.16))
    rho = np.zeros(g.shape)
    exact = np.zeros(g.shape)
    for (cx, cy, cz), a0, sg in blobs:
        r = np.sqrt((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2)
        rho += a0 * np.exp(-0.5 * r ** 2 / sg ** 2)
        exact += analytic.gaussian_potential(r, a0, sg)
    scale = np.max(np.abs(exact))
    B = _robin_matrix(g, (0.0, 0.0, 0.0))
    alone = spla.spsolve(B.tocsc(), 4.0 * np.pi * rho.ravel()).reshape(g.shape)
    errs = [np.sqrt(np.mean((alone - exact) ** 2)) / scale]
    for ext in (2, 4, 8):
        phi, _, _ = _composite_steady_state(g, ext, rho, (0.0, 0.0, 0.0))
        errs.append(np.sqrt(np.mean((phi - exact) ** 2)) / scale)
    assert errs[1] < errs[0] and errs[2] < errs[1] and errs[3] < errs[2], errs
