"""Pins of the FP64 oracle against what the mathematics fixes (no GPU).

Each check is chosen so that a plausible mistake in the oracle (a dropped
term, a wrong sign, index or power of dx, a transposed axis) fails at least one
of them.  The paper (arXiv:1602.05700) prints no worked example, so every pin is
a closed form, an invariant, a special case or a brute-force sum.
"""
import numpy as np
import pytest
import scipy.integrate
import scipy.special

import workloads
from oracle import analytic, core, poisson
from oracle.core import Grid, interior, padded


def _mode(g: Grid, k):
    i = np.arange(g.nx)
    j = np.arange(g.ny)
    kk = np.arange(g.nz)
    fx = np.sin(np.pi * k[0] * (i + 1) / (g.nx + 1))
    fy = np.sin(np.pi * k[1] * (j + 1) / (g.ny + 1))
    fz = np.sin(np.pi * k[2] * (kk + 1) / (g.nz + 1))
    return fz[:, None, None] * fy[None, :, None] * fx[None, None, :]


def _lam(g: Grid, k):
    return sum((4.0 / g.dx ** 2) * np.sin(np.pi * kd / (2.0 * (nd + 1))) ** 2
               for kd, nd in zip(k, (g.nx, g.ny, g.nz)))


def _run_mode(g, k, C, eta, nsteps):
    m = _mode(g, k)
    Pn, Pm = padded(g), padded(g)
    interior(Pn)[...] = m
    interior(Pm)[...] = m
    dt = C * g.dx
    core.substeps(g, Pn, Pm, np.zeros(g.shape), 1.0, dt, eta, 1.0, nsteps)
    return m, interior(Pn).copy(), interior(Pm).copy(), dt


# ---------------------------------------------------------------- time stepping (Eq. 2)

@pytest.mark.parametrize("nsteps", [1, 2, 7, 60])
def test_eigenmode_closed_form_undamped(nsteps):
    """A Dirichlet eigenmode with rho = 0 and zero ghosts evolves as
    a_n = cos((n + 1/2) theta) / cos(theta / 2), cos theta = 1 - c^2 dt^2 lambda / 2,
    when phi^{-1} = phi^0 (Chebyshev solution of the leapfrog recurrence)."""
    g = Grid(12, 10, 8, -0.6, -0.5, -0.4, 0.1)
    k = (2, 3, 1)
    m, pn, pm, dt = _run_mode(g, k, 0.4, 0.0, nsteps)
    th = np.arccos(1.0 - dt ** 2 * _lam(g, k) / 2.0)
    a = lambda n: np.cos((n + 0.5) * th) / np.cos(th / 2.0)
    assert np.max(np.abs(pn - a(nsteps) * m)) < 1e-12
    assert np.max(np.abs(pm - a(nsteps - 1) * m)) < 1e-12


@pytest.mark.parametrize("eta", [0.7, 3.0, 40.0])
def test_eigenmode_closed_form_damped(eta):
    """With damping eta the mode amplitude is A mu1^n + B mu2^n, mu the roots of
    (1+a) mu^2 - (2 - c^2 dt^2 lambda) mu + (1-a) = 0, a = eta dt / 2."""
    g = Grid(9, 11, 10, 0.0, 0.0, 0.0, 0.05)
    k = (1, 4, 2)
    n = 45
    m, pn, pm, dt = _run_mode(g, k, 0.35, eta, n)
    a = 0.5 * eta * dt
    mu = np.roots([1.0 + a, -(2.0 - dt ** 2 * _lam(g, k)), 1.0 - a]).astype(complex)
    # a_0 = a_{-1} = 1
    M = np.array([[1.0, 1.0], [1.0 / mu[0], 1.0 / mu[1]]])
    AB = np.linalg.solve(M, np.array([1.0, 1.0], dtype=complex))
    amp = lambda s: (AB[0] * mu[0] ** s + AB[1] * mu[1] ** s).real
    assert np.max(np.abs(pn - amp(n) * m)) < 1e-12
    assert np.max(np.abs(pm - amp(n - 1) * m)) < 1e-12


def test_stability_limit():
    """Leapfrog with the 7-point Laplacian is stable iff c^2 dt^2 lambda_max <= 4;
    for the highest grid mode that is just above c dt/dx = 1/sqrt(3)."""
    g = Grid(16, 16, 16, 0, 0, 0, 1.0 / 16)
    k = (16, 16, 16)
    s2 = np.sin(np.pi * 16 / 34.0) ** 2
    c_lim = 1.0 / np.sqrt(3.0 * s2)
    assert 0.577 < 1 / np.sqrt(3) < c_lim < 0.59
    _, stable, _, _ = _run_mode(g, k, 1 / np.sqrt(3), 0.0, 600)
    _, unstable, _, _ = _run_mode(g, k, 0.59, 0.0, 600)
    assert np.max(np.abs(stable)) < 20.0
    assert np.max(np.abs(unstable)) > 1e6


def test_energy_conserved_undamped():
    """For eta = 0, rho = 0 and zero ghosts the discrete energy
    ||phi^{n+1}-phi^n||^2 - c^2 dt^2 <phi^{n+1}, L_h phi^n> is exactly conserved."""
    g = Grid(10, 9, 8, 0, 0, 0, 0.1)
    rng = np.random.default_rng(5)
    Pn, Pm = padded(g), padded(g)
    interior(Pn)[...] = rng.standard_normal(g.shape)
    interior(Pm)[...] = rng.standard_normal(g.shape) * 0.3 + interior(Pn)
    dt = 0.5 * g.dx

    def energy(P1, P0):
        return np.sum((interior(P1) - interior(P0)) ** 2) - dt ** 2 * np.sum(interior(P1) * core.laplacian(g, P0))

    Pn2, Pm2 = Pn.copy(), Pm.copy()
    core.substeps(g, Pn2, Pm2, np.zeros(g.shape), 1.0, dt, 0.0, 1.0, 1)
    e0 = energy(Pn2, Pm2)
    core.substeps(g, Pn2, Pm2, np.zeros(g.shape), 1.0, dt, 0.0, 1.0, 300)
    e1 = energy(Pn2, Pm2)
    assert abs(e1 - e0) < 1e-11 * abs(e0)
    # damping removes energy
    Pn3, Pm3 = Pn.copy(), Pm.copy()
    core.substeps(g, Pn3, Pm3, np.zeros(g.shape), 1.0, dt, 1.0, 1.0, 301)
    assert energy(Pn3, Pm3) < 0.9 * e0


def test_source_sign_and_scale():
    """One substep from phi = 0 everywhere, rho uniform: phi^1 = -c^2 dt^2 4 pi G rho / (1+a)."""
    g = Grid(6, 5, 4, 0, 0, 0, 0.2)
    Pn, Pm = padded(g), padded(g)
    rho = np.full(g.shape, 0.7)
    dt, G, c, eta = 0.05, 2.0, 1.5, 3.0
    core.substeps(g, Pn, Pm, rho, c, dt, eta, G, 1)
    expect = -(c * dt) ** 2 * 4 * np.pi * G * 0.7 / (1 + 0.5 * eta * dt)
    assert np.allclose(interior(Pn), expect, rtol=1e-14, atol=0)
    assert np.all(interior(Pm) == 0.0)


# ---------------------------------------------------------------- steady state (Eq. 1)

def _random_problem(g, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.0, 1.0, g.shape)
    P = padded(g)
    core.set_faces(P, [rng.uniform(-2, -1, f.shape) for f in core.faces(P)])
    return rho, P


def test_dst_equals_dense_lu():
    g = Grid(9, 7, 6, -0.3, 0.1, 0.2, 0.13)
    rho, P = _random_problem(g, 1)
    a = poisson.solve_dst(g, rho, 1.3, P)
    b = poisson.solve_dense(g, rho, 1.3, P)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


def test_poisson_solution_is_fixed_point():
    g = Grid(11, 9, 10, -1, -1, -1, 0.2)
    rho, P = _random_problem(g, 2)
    phi = poisson.solve_dst(g, rho, 1.0, P)
    for eta in (0.0, 2.5):
        Pn = poisson.with_solution(g, P, phi)
        Pm = Pn.copy()
        core.substeps(g, Pn, Pm, rho, 1.0, 0.5 * g.dx, eta, 1.0, 25)
        assert np.max(np.abs(interior(Pn) - phi)) < 1e-12 * np.max(np.abs(phi))


def test_residual_definitions():
    g = Grid(8, 9, 7, 0, 0, 0, 0.1)
    rho, P = _random_problem(g, 3)
    r0 = core.residual(g, P, rho, 1.0)
    assert r0[0] == pytest.approx(1.0, abs=1e-15)  # R_b = 1 at phi = 0
    b = poisson.rhs(g, rho, 1.0, P)
    assert r0[1] == pytest.approx(np.linalg.norm(b) / np.linalg.norm(4 * np.pi * rho), rel=1e-13)
    phi = poisson.solve_dst(g, rho, 1.0, P)
    r1 = core.residual(g, poisson.with_solution(g, P, phi), rho, 1.0)
    assert r1[0] < 1e-13 and r1[1] < 1e-12
    assert r1[2] == pytest.approx(np.linalg.norm(phi), rel=1e-14)
    assert r1[3] == 0.0
    bad = rho.copy()
    bad[3, 4, 5] = np.nan
    assert core.residual(g, P, bad, 1.0)[3] == 1.0


def test_gauss_law_telescoping():
    """sum over interior of L_h phi dx^3 equals the face flux sum (phi_ghost - phi_adj) dx."""
    g = Grid(7, 8, 9, 0, 0, 0, 0.3)
    rng = np.random.default_rng(4)
    P = rng.standard_normal(g.pshape)
    lhs = np.sum(core.laplacian(g, P)) * g.dx ** 3
    flux = (np.sum(P[1:-1, 1:-1, 0] - P[1:-1, 1:-1, 1]) + np.sum(P[1:-1, 1:-1, -1] - P[1:-1, 1:-1, -2])
            + np.sum(P[1:-1, 0, 1:-1] - P[1:-1, 1, 1:-1]) + np.sum(P[1:-1, -1, 1:-1] - P[1:-1, -2, 1:-1])
            + np.sum(P[0, 1:-1, 1:-1] - P[1, 1:-1, 1:-1]) + np.sum(P[-1, 1:-1, 1:-1] - P[-2, 1:-1, 1:-1]))
    assert lhs == pytest.approx(flux * g.dx, rel=1e-12, abs=1e-12)


def _quadratic(g):
    """phi = al x^2 + be y^2 + ga z^2 + de x y + ep y z + ze x + et, with
    2 (al + be + ga) = 4 pi G rho0 (G = 1, rho0 = 0.8)."""
    x, y, z = g.centres()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    al, be = 0.9, -0.4
    ga = 2 * np.pi * 0.8 - al - be
    de, ep, ze = 0.3, -0.7, 0.25
    phi = al * X ** 2 + be * Y ** 2 + ga * Z ** 2 + de * X * Y + ep * Y * Z + ze * X + 0.1
    grad = (2 * al * X + de * Y + ze, 2 * be * Y + de * X + ep * Z, 2 * ga * Z + ep * Y)
    return phi, grad


def test_quadratic_potential_exact():
    """L_h and central differences are exact on quadratics: the quadratic with
    Laplacian 4 pi G rho0 is a fixed point, and g = -grad phi exactly."""
    g = Grid(9, 8, 7, -0.45, -0.1, -0.3, 0.11)
    P, grad = _quadratic(g)
    rho = np.full(g.shape, 0.8)
    assert np.max(np.abs(core.laplacian(g, P) - 4 * np.pi * 0.8)) < 1e-10
    Pn, Pm = P.copy(), P.copy()
    core.substeps(g, Pn, Pm, rho, 1.0, 0.4 * g.dx, 1.0, 1.0, 30)
    assert np.max(np.abs(Pn - P)) < 1e-12
    gx, gy, gz = core.gradient(g, P)
    for got, want in zip((gx, gy, gz), grad):
        assert np.max(np.abs(got + want[1:-1, 1:-1, 1:-1])) < 1e-12


def test_linearity_in_rho():
    g = Grid(10, 10, 10, -1, -1, -1, 0.2)
    r1 = workloads.gaussian_density(10, 0.2, 1.0, (0.2, -0.1, 0.0))
    r2 = workloads.gaussian_density(10, 0.3, 2.0, (-0.3, 0.2, 0.1))
    outs = []
    for rho in (r1, r2, r1 + r2):
        o = core.Oracle(g, lmax=4, eta=1.0)
        o.step(rho, 1.0, 0.4 * g.dx, 40)
        outs.append(o.potential()[0])
    assert np.max(np.abs(outs[2] - outs[0] - outs[1])) < 1e-12 * np.max(np.abs(outs[2]))


def test_damped_relaxation_reaches_poisson_solution():
    """With critical damping of the slowest mode the scheme relaxes from zero to
    the discrete Poisson solution (same ghosts)."""
    n = 16
    g = Grid.cube(n)
    rho = workloads.blob_density(n, workloads.blob_params(7, 4))
    lam = poisson.lambda_min(g)
    o = core.Oracle(g, lmax=4, eta=2.0 * np.sqrt(lam))
    o.step(rho, 1.0, 0.4 * g.dx, 700)
    phi = o.potential()[0]
    want = poisson.solve_dst(g, rho, 1.0, o.Pn)
    assert np.max(np.abs(phi - want)) < 1e-10 * np.max(np.abs(want))
    assert o.residual(rho)[0] < 1e-10


def test_sphere_symmetry():
    """A centred sphere on a cube grid keeps the octahedral symmetry of the grid."""
    n = 16
    g = Grid.cube(n)
    rho = workloads.sphere_density(n, 0.5)
    o = core.Oracle(g, lmax=4, eta=0.0)
    o.step(rho, 1.0, 0.4 * g.dx, 50)
    phi = o.potential()[0]
    scale = np.max(np.abs(phi))
    for t in [(0, 2, 1), (1, 0, 2), (2, 1, 0)]:
        assert np.max(np.abs(phi - phi.transpose(t))) < 1e-13 * scale
    for ax in range(3):
        assert np.max(np.abs(phi - np.flip(phi, ax))) < 1e-13 * scale


# ---------------------------------------------------------------- multipole boundary

def test_ylm_matches_scipy():
    """Moments of a single off-axis point-like cell equal m r^l conj(Y_lm) with
    scipy's spherical harmonics."""
    g = Grid(3, 3, 3, -0.3, 0.2, -0.1, 0.2)
    rho = np.zeros(g.shape)
    rho[1, 2, 0] = 5.0
    q = core.moments(g, rho, 4, (0.05, -0.02, 0.1))
    x = -0.3 + 0.5 * 0.2 - 0.05
    y = 0.2 + 2.5 * 0.2 + 0.02
    z = -0.1 + 1.5 * 0.2 - 0.1
    r = np.sqrt(x * x + y * y + z * z)
    th, ph = np.arccos(z / r), np.arctan2(y, x) % (2 * np.pi)
    m = 5.0 * 0.2 ** 3
    for l in range(5):
        for mm in range(-l, l + 1):
            want = m * r ** l * np.conj(scipy.special.sph_harm_y(l, mm, th, ph))
            assert q[l * l + l + mm] == pytest.approx(want, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("lmax", [0, 1, 2, 3, 4])
def test_boundary_equals_legendre_addition(lmax):
    """sum_m 4 pi/(2l+1) Q_lm Y_lm / r^{l+1} equals the brute-force Legendre sum
    -G sum_j m_j r_j^l P_l(cos gamma_j) / r^{l+1} (addition theorem)."""
    g = Grid(7, 6, 5, -0.7, -0.6, -0.5, 0.2)
    rng = np.random.default_rng(lmax + 10)
    rho = rng.uniform(0, 1, g.shape)
    origin = (0.03, -0.05, 0.02)
    q = core.moments(g, rho, lmax, origin)
    P = padded(g)
    core.boundary(g, q, lmax, 1.7, P, origin)
    pts = analytic.ghost_points(g)
    for f, pt in zip(core.faces(P), pts):
        want = analytic.legendre_multipole(g, rho, pt, lmax, 1.7, origin)
        assert np.max(np.abs(f.ravel() - want)) < 1e-13 * np.max(np.abs(want))


def test_monopole_boundary_is_minus_gm_over_r():
    g = Grid(8, 8, 8, -1, -1, -1, 0.25)
    rho = workloads.random_field(g.shape, 3, 0.0, 1.0)
    q = core.moments(g, rho, 0)
    P = padded(g)
    core.boundary(g, q, 0, 2.0, P)
    M = rho.sum() * g.dx ** 3
    for f, pt in zip(core.faces(P), analytic.ghost_points(g)):
        assert np.allclose(f.ravel(), -2.0 * M / np.linalg.norm(pt, axis=1), rtol=1e-13, atol=0)


def test_boundary_converges_to_direct_sum_with_lmax():
    """For a compact off-centre source the multipole boundary approaches the
    free-space potential as lmax grows (error ~ (r_src / r)^(lmax+1))."""
    n = 16
    g = Grid.cube(n)
    rho = workloads.gaussian_density(n, 0.06, 1.0, (0.31, -0.22, 0.17))
    pts = np.concatenate(analytic.ghost_points(g))
    want = analytic.direct_sum_points(g, rho, pts)
    errs = []
    for lmax in range(5):
        q = core.moments(g, rho, lmax)
        P = padded(g)
        core.boundary(g, q, lmax, 1.0, P)
        got = np.concatenate([f.ravel() for f in core.faces(P)])
        errs.append(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    assert all(errs[i + 1] < 0.6 * errs[i] for i in range(4)), errs
    assert errs[4] < 5e-3, errs


# ---------------------------------------------------------------- closed forms

def test_cube_self_potential_constant():
    """int over [-1/2,1/2]^3 of 1/|x| = 6 * (1/8) * int_{[-1,1]^2} du dv / sqrt(1+u^2+v^2)
    (six pyramids with apex at the centre)."""
    i2, _ = scipy.integrate.dblquad(lambda v, u: 1.0 / np.sqrt(1 + u * u + v * v), -1, 1, -1, 1,
                                    epsabs=1e-13, epsrel=1e-13)
    assert analytic.CUBE_SELF == pytest.approx(6.0 * i2 / 8.0, rel=1e-11)
    assert analytic.CUBE_SELF == pytest.approx(2.3800773640, abs=1e-9)


def _gaussian_error(n):
    g = Grid.cube(n)
    rho = workloads.gaussian_density(n, 0.1, 1.0)
    q = core.moments(g, rho, 0)
    P = padded(g)
    core.boundary(g, q, 0, 1.0, P)
    phi = poisson.solve_dst(g, rho, 1.0, P)
    X, Y, Z = analytic.cell_centres(g)
    exact = analytic.gaussian_potential(np.sqrt(X * X + Y * Y + Z * Z), 1.0, 0.1)
    M_h = rho.sum() * g.dx ** 3
    return np.linalg.norm(phi - exact) / np.linalg.norm(exact), M_h, phi, g, P


def test_gaussian_second_order_convergence():
    """Discrete Poisson solution of a centred Gaussian against the closed form
    -G M erf(r/(sqrt2 sigma))/r: error falls ~4x per halving of dx; the
    monopole boundary is exact to round-off because the mass is all inside."""
    e32, m32, *_ = _gaussian_error(32)
    e64, m64, *_ = _gaussian_error(64)
    M = analytic.gaussian_mass(1.0, 0.1)
    assert m64 == pytest.approx(M, rel=1e-12)
    assert 3.7 < e32 / e64 < 4.3, (e32, e64)
    assert e64 < 1.5e-3


def test_gradient_second_order_convergence():
    errs = []
    for n in (32, 64):
        _, _, phi, g, P = _gaussian_error(n)
        X, Y, Z = analytic.cell_centres(g)
        r = np.sqrt(X * X + Y * Y + Z * Z)
        M = analytic.gaussian_mass(1.0, 0.1)
        s = 0.1
        # d/dr of -G M erf(r/(sqrt2 s))/r; g = -grad phi = -(dphi/dr) x/r
        dphidr = M * (scipy.special.erf(r / (np.sqrt(2) * s)) / r ** 2
                      - np.sqrt(2 / np.pi) / s * np.exp(-r * r / (2 * s * s)) / r)
        want = [-dphidr * X / r, -dphidr * Y / r, -dphidr * Z / r]
        got = core.gradient(g, poisson.with_solution(g, P, phi))
        errs.append(max(np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(got, want)))
    assert 3.5 < errs[0] / errs[1] < 4.5, errs


def test_sphere_against_closed_form():
    """Uniform sphere (R = 0.25): converged discrete potential within a few
    percent of -GM/r, -GM(3R^2-r^2)/(2R^3); the gap is the staircase mass."""
    n = 32
    g = Grid.cube(n)
    rho = workloads.sphere_density(n, 0.25)
    q = core.moments(g, rho, 0)
    P = padded(g)
    core.boundary(g, q, 0, 1.0, P)
    phi = poisson.solve_dst(g, rho, 1.0, P)
    M = 4 * np.pi * 0.25 ** 3 / 3
    X, Y, Z = analytic.cell_centres(g)
    exact = analytic.sphere_potential(np.sqrt(X * X + Y * Y + Z * Z), M, 0.25)
    err = np.linalg.norm(phi - exact) / np.linalg.norm(exact)
    mh = rho.sum() * g.dx ** 3
    assert abs(mh / M - 1) < 0.1
    assert err < 0.1
    # the discrete problem with the exact staircase mass in the boundary is consistent:
    # Gauss law flux equals 4 pi G M_h
    flux = np.sum(core.laplacian(g, poisson.with_solution(g, P, phi))) * g.dx ** 3
    assert flux == pytest.approx(4 * np.pi * mh, rel=1e-10)


def test_direct_sum_convergence_tiny_grids():
    """Relaxed with ghosts from the free-space direct sum, the interior converges
    toward the brute-force direct-sum potential as the grid is refined."""
    errs = []
    for n in (8, 16):
        g = Grid.cube(n)
        rho = workloads.gaussian_density(n, 0.2, 1.0, (0.1, -0.05, 0.0))
        pts = analytic.ghost_points(g)
        o = core.Oracle(g, eta=2.0 * np.sqrt(poisson.lambda_min(g)), bc="user")
        o.set_boundary([analytic.direct_sum_points(g, rho, p).reshape(f.shape)
                        for p, f in zip(pts, core.faces(o.Pn))])
        o.step(rho, 1.0, 0.4 * g.dx, 40 * n)
        phi = o.potential()[0]
        ds = analytic.direct_sum_cells(g, rho)
        errs.append(np.linalg.norm(phi - ds) / np.linalg.norm(ds))
    assert errs[1] < errs[0] / 2.5, errs


# ---------------------------------------------------------------- solver bookkeeping

def test_set_state_and_dt_change_keep_phidot():
    g = Grid(6, 6, 6, -1, -1, -1, 1 / 3)
    rng = np.random.default_rng(9)
    o = core.Oracle(g, bc="user")
    o.set_boundary([np.zeros(f.shape) for f in core.faces(o.Pn)])
    phi = rng.standard_normal(g.shape)
    pd = rng.standard_normal(g.shape)
    o.set_state(phi, pd, 0.05)
    p, d = o.potential()
    assert np.allclose(p, phi, rtol=0, atol=0)
    assert np.allclose(d, pd, rtol=1e-12, atol=1e-12)
    # rescale on a dt change keeps (phi^n - phi^{n-1})/dt, then zero substeps is impossible,
    # so check via one step at the new dt against the leapfrog with a consistent start
    o2 = core.Oracle(g, bc="user")
    o2.set_boundary([np.zeros(f.shape) for f in core.faces(o.Pn)])
    o2.set_state(phi, pd, 0.02)
    o.step(np.zeros(g.shape), 1.0, 0.02, 3)
    o2.step(np.zeros(g.shape), 1.0, 0.02, 3)
    assert np.max(np.abs(o.potential()[0] - o2.potential()[0])) < 1e-12


def test_f32_storage_emulation_close_to_f64():
    n = 16
    g = Grid.cube(n)
    rho = workloads.blob_density(n, workloads.blob_params(1, 4), dtype=np.float32).astype(np.float64)
    a = core.Oracle(g, lmax=4, eta=0.0)
    b = core.Oracle(g, lmax=4, eta=0.0, storage="f32")
    for _ in range(5):
        a.step(rho, 1.0, 0.4 * g.dx, 8)
        b.step(rho, 1.0, 0.4 * g.dx, 8)
    pa, pb = a.potential()[0], b.potential()[0]
    assert np.all(pb == pb.astype(np.float32).astype(np.float64))
    err = np.max(np.abs(pa - pb)) / np.max(np.abs(pa))
    assert 0 < err < 1e-5


def test_energy_of_uniform_sphere_converges_to_closed_form():
    """W = 1/2 sum rho phi dV of the discrete Poisson solution of a uniform
    sphere tends to -3 G M^2 / (5 R) at second order (M, R of the voxelised
    sphere)."""
    from oracle import core, poisson

    errs = []
    for n in (24, 48):
        g = Grid.cube(n)
        x, y, z = (c[1:-1] for c in g.centres())
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        rho = (X ** 2 + Y ** 2 + Z ** 2 < 0.25).astype(float)
        dv = g.dx ** 3
        M = rho.sum() * dv
        R = (3.0 * M / (4.0 * np.pi)) ** (1.0 / 3.0)
        P = core.padded(g)
        core.boundary(g, core.moments(g, rho, 0), 0, 1.0, P)
        W = core.energy(g, rho, poisson.solve_dst(g, rho, 1.0, P))
        errs.append(abs(W / (-0.6 * M * M / R) - 1.0))
    assert errs[1] < 2e-3 and errs[0] / errs[1] > 3.0, errs


def test_mean_relative_error_eq6():
    """Eq. 6 closed forms: a uniform relative offset eps gives |eps|; a field
    whose relative offset is +eps on half the cells and -eps on the other half
    gives eps; offsets 0 and 2 eps on halves give sqrt(2) eps (an RMS, not a
    mean of magnitudes); identical fields give 0."""
    rng = np.random.default_rng(12)
    p = -rng.uniform(0.5, 2.0, (6, 7, 8))
    eps = 3e-3
    assert poisson.mean_relative_error(p * (1 + eps), p) == pytest.approx(eps, rel=1e-12)
    sign = np.where(np.arange(p.size).reshape(p.shape) % 2 == 0, 1.0, -1.0)
    assert poisson.mean_relative_error(p * (1 + eps * sign), p) == pytest.approx(eps, rel=1e-12)
    two = np.where(sign > 0, 2 * eps, 0.0)
    assert poisson.mean_relative_error(p * (1 + two), p) == pytest.approx(np.sqrt(2) * eps, rel=1e-12)
    assert poisson.mean_relative_error(p, p) == 0.0
