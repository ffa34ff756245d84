"""Pins of the oracle's local outer boundaries (no GPU).

Robin (monopole fall-off r_g phi_g = r_i phi_i), outgoing (the radiative form
d(r phi)/dt + c d(r phi)/dr = 0) and periodic (wrap, mean-subtracted source),
Sec. 2 and Sec. 4 of the paper.  Each is pinned against something other than
itself: exactness on -G M / r, a sparse direct solve of the Robin linear
system, an FFT solve with the 7-point symbol, and radiation of a free pulse
through the outgoing boundary against total reflection by a zero Dirichlet one.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import core
from oracle.core import Grid, Oracle, interior, padded


def _blob(g: Grid, centre=(0.15, -0.1, 0.05), sigma=0.18):
    x, y, z = (c[1:-1] for c in g.centres())
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    r2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2
    return np.exp(-0.5 * r2 / sigma ** 2)


def _robin_matrix(g: Grid, origin):
    """-L_h with every face ghost eliminated by phi_g = (r_i / r_g) phi_i:
    each ghost neighbour adds (r_i / r_g) / dx^2 to its cell's diagonal."""
    nx, ny, nz = g.nx, g.ny, g.nz
    x, y, z = g.centres()
    o = np.asarray(origin)
    N = nx * ny * nz
    idx = lambda i, j, k: (k * ny + j) * nx + i
    rows, cols, vals = [], [], []
    h2 = 1.0 / g.dx ** 2
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                p = idx(i, j, k)
                diag = -6.0 * h2
                ri = np.linalg.norm([x[i + 1] - o[0], y[j + 1] - o[1], z[k + 1] - o[2]])
                for di, dj, dk in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
                    a, b, c = i + di, j + dj, k + dk
                    if 0 <= a < nx and 0 <= b < ny and 0 <= c < nz:
                        rows.append(p)
                        cols.append(idx(a, b, c))
                        vals.append(h2)
                    else:
                        rg = np.linalg.norm([x[a + 1] - o[0], y[b + 1] - o[1], z[c + 1] - o[2]])
                        diag += h2 * ri / rg
                rows.append(p)
                cols.append(p)
                vals.append(diag)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def _run_to_convergence(g, bc, rho, eta, steps, origin=(0.0, 0.0, 0.0), G=1.0):
    o = Oracle(g, G=G, origin=origin, eta=eta, bc=bc)
    dt = 0.4 * g.dx
    o.step(rho, 1.0, dt, steps)
    return o


def test_robin_ghosts_exact_for_monopole():
    g = Grid(9, 10, 11, -1.0, -0.9, -1.1, 0.2)
    origin = (0.1, 0.05, -0.12)
    x, y, z = g.centres()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    R = np.sqrt((X - origin[0]) ** 2 + (Y - origin[1]) ** 2 + (Z - origin[2]) ** 2)
    exact = -2.5 / R  # -G M / r on the whole padded grid, ghosts included
    P = padded(g)
    interior(P)[...] = interior(exact)
    core.local_ghosts(g, "robin", P, origin)
    for got, want in zip(core.faces(P), core.faces(exact)):
        assert np.allclose(got, want, rtol=1e-14, atol=0)
    # the outgoing rule's steady form is the same relation
    Q = padded(g)
    interior(Q)[...] = interior(exact)
    core.local_ghosts(g, "outgoing", Q, origin)
    for got, want in zip(core.faces(Q), core.faces(exact)):
        assert np.allclose(got, want, rtol=1e-14, atol=0)


def test_periodic_ghosts_wrap():
    g = Grid(5, 6, 7, 0.0, 0.0, 0.0, 1.0)
    P = padded(g)
    interior(P)[...] = np.random.default_rng(0).standard_normal(g.shape)
    core.local_ghosts(g, "periodic", P)
    I = interior(P)
    f = core.faces(P)
    assert np.array_equal(f[0], I[:, :, -1]) and np.array_equal(f[1], I[:, :, 0])
    assert np.array_equal(f[2], I[:, -1, :]) and np.array_equal(f[3], I[:, 0, :])
    assert np.array_equal(f[4], I[-1, :, :]) and np.array_equal(f[5], I[0, :, :])


@pytest.mark.parametrize("bc", ["robin", "outgoing"])
def test_local_bc_steady_state_is_sparse_robin_solve(bc):
    """The damped evolution with either rule settles on the solution of the
    Robin linear system (outgoing's steady state is the Robin relation)."""
    g = Grid.cube(12)
    origin = (0.05, -0.03, 0.02)
    rho = _blob(g)
    A = _robin_matrix(g, origin)
    s = 4.0 * np.pi * rho.ravel()
    phi_ref = spla.spsolve(A.tocsc(), s).reshape(g.shape)
    lam_min = float(np.linalg.eigvalsh(-A.toarray())[0])
    o = _run_to_convergence(g, bc, rho, eta=2.0 * np.sqrt(lam_min), steps=2500, origin=origin)
    phi = interior(o.Pn)
    err = np.max(np.abs(phi - phi_ref)) / np.max(np.abs(phi_ref))
    assert err < 1e-10, err
    assert o.residual(rho)[0] < 1e-10


def test_periodic_steady_state_is_fft_solve():
    """Periodic with the mean-subtracted source converges to the FFT solution
    of L_h phi = 4 pi G (rho - mean rho) with the 7-point symbol, mean zero."""
    g = Grid(12, 10, 14, -1.0, -1.0, -1.0, 2.0 / 12)
    rho = _blob(g, centre=(0.3, 0.2, -0.4), sigma=0.25)
    k = [2.0 * np.pi * np.fft.fftfreq(n) for n in (g.nz, g.ny, g.nx)]
    KZ, KY, KX = np.meshgrid(*k, indexing="ij")
    sym = (2.0 * np.cos(KX) + 2.0 * np.cos(KY) + 2.0 * np.cos(KZ) - 6.0) / g.dx ** 2
    sh = np.fft.fftn(4.0 * np.pi * (rho - rho.mean()))
    sym[0, 0, 0] = 1.0
    ph = sh / sym
    ph[0, 0, 0] = 0.0
    phi_ref = np.real(np.fft.ifftn(ph))
    lam_min = (2.0 - 2.0 * np.cos(2.0 * np.pi / max(g.nx, g.ny, g.nz))) / g.dx ** 2
    o = _run_to_convergence(g, "periodic", rho, eta=2.0 * np.sqrt(lam_min), steps=3000)
    phi = interior(o.Pn)
    assert abs(phi.mean()) < 1e-12
    err = np.max(np.abs(phi - phi_ref)) / np.max(np.abs(phi_ref))
    assert err < 1e-10, err
    assert o.residual(rho)[0] < 1e-10
    # the source really is mean-subtracted: without it there is no steady state
    assert abs(o.rbar(rho) - rho.mean()) < 1e-15


def test_outgoing_lets_a_free_pulse_leave():
    """rho = 0, a Gaussian bump of phi at rest: through the outgoing boundary
    it leaves the box (Sec. 4: errors propagate out through the boundary);
    a zero Dirichlet boundary reflects it and keeps the energy."""
    g = Grid.cube(32)
    x, y, z = (c[1:-1] for c in g.centres())
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    bump = np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / (2 * 0.15 ** 2))
    rho = np.zeros(g.shape)
    dt = 0.4 * g.dx
    steps = int(round(4.0 / dt))  # four half-widths at c = 1

    out = Oracle(g, bc="outgoing")
    out.set_state(bump, None, dt)
    out.step(rho, 1.0, dt, steps)
    ref = Oracle(g, bc="user")
    ref.set_boundary([np.zeros_like(f) for f in core.faces(padded(g))])
    ref.set_state(bump, None, dt)
    ref.step(rho, 1.0, dt, steps)

    rob = Oracle(g, bc="robin")
    rob.set_state(bump, None, dt)
    rob.step(rho, 1.0, dt, steps)

    n0 = np.linalg.norm(bump)
    left = np.linalg.norm(interior(out.Pn)) / n0
    kept = np.linalg.norm(interior(ref.Pn)) / n0
    kept_robin = np.linalg.norm(interior(rob.Pn)) / n0
    assert left < 5e-3, left
    assert kept > 0.1, kept
    # the static Robin relation is not radiative: it reflects too
    assert kept_robin > 0.3, kept_robin


def test_outgoing_relaxes_a_zero_start_without_damping():
    """eta = 0: with the outgoing boundary the zero-start transient radiates
    away and the static solution emerges; with the multipole Dirichlet
    boundary the same start keeps oscillating (no dissipation)."""
    g = Grid.cube(24)
    rho = _blob(g, centre=(0.1, 0.0, -0.05), sigma=0.15)
    dt = 0.4 * g.dx
    steps = int(round(8.0 / dt))
    out = _run_to_convergence(g, "outgoing", rho, eta=0.0, steps=steps)
    dir_ = _run_to_convergence(g, "multipole", rho, eta=0.0, steps=steps)
    r_out = out.residual(rho)[1]
    r_dir = dir_.residual(rho)[1]
    assert r_out < 1e-3, r_out
    assert r_dir > 0.3, r_dir
