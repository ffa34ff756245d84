"""GPU parity of the local outer boundaries (Robin, outgoing, periodic) against
the FP64 oracle, through the C ABI, plus the properties that hold at any size:
relaxation of a zero start through the outgoing boundary without damping,
the FFT solution on a periodic box, and a bitwise checkpoint of the outgoing
boundary's ghost state."""
import numpy as np
import pytest

from oracle import core
from oracle.core import Oracle
from test_gpu_parity import F32_EMU_TOL, F32_TOL, F64_TOL, compare_state, dens, grid_of, host, npdt, rel, solver, \
    to_dev

pytestmark = pytest.mark.gpu

LOCAL = ["robin", "outgoing", "periodic"]
# single cell, ragged (scalar kernel), vector path with several tiles and z chunks
SHAPES = [(1, 1, 1), (7, 9, 5), (23, 29, 37), (40, 33, 132), (64, 64, 64)]


def pair(hgs, shape, bc, storage="f64", eta=0.0, origin=(0.03, -0.02, 0.01)):
    s = solver(hgs, shape, storage=storage, eta=eta, origin=origin, bc=bc)
    o = Oracle(grid_of(shape), eta=eta, origin=origin, bc=bc)
    return s, o


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", LOCAL)
def test_local_bc_f64(gpu_lib, shape, bc):
    rho = dens(shape, 21, "f64")
    g = grid_of(shape)
    s, o = pair(gpu_lib, shape, bc, eta=1.5)
    for dt, nsub in ((0.4, 1), (0.4, 9), (0.3, 14)):  # the last step rescales phi^{n-1}
        s.step(to_dev(rho), 1.0, dt * g.dx, nsub)
        o.step(rho, 1.0, dt * g.dx, nsub)
    compare_state(s, o, "f64", F64_TOL)
    got = host(s.get_boundary())
    want = gpu_lib.faces_to_flat(core.faces(o.Pn))
    assert rel(got, want) < F64_TOL
    r = s.residual(to_dev(rho))
    ro = o.residual(rho)
    assert abs(r[0] - ro[0]) <= 1e-9 * ro[0] and r[0] == pytest.approx(r[1], rel=1e-12)


@pytest.mark.parametrize("shape", [(7, 9, 5), (40, 33, 132)])
@pytest.mark.parametrize("bc", LOCAL)
def test_local_bc_f32(gpu_lib, shape, bc):
    rho = dens(shape, 22, "f32")
    r64 = rho.astype(np.float64)
    g = grid_of(shape)
    origin = (0.03, -0.02, 0.01)
    s, o = pair(gpu_lib, shape, bc, storage="f32", eta=1.0, origin=origin)
    emu = Oracle(g, eta=1.0, origin=origin, bc=bc, storage="f32")
    for nsub in (4, 4, 11):
        s.step(to_dev(rho), 1.0, 0.4 * g.dx, nsub)
        o.step(r64, 1.0, 0.4 * g.dx, nsub)
        emu.step(r64, 1.0, 0.4 * g.dx, nsub)
    compare_state(s, o, "f32", F32_TOL)
    assert rel(host(s.potential()[0]), emu.potential()[0]) < F32_EMU_TOL


@pytest.mark.parametrize("bc", LOCAL)
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_local_bc_set_state(gpu_lib, bc, storage):
    """set_state builds the ghosts by the steady rule; later substeps match."""
    shape = (20, 18, 24)
    g = grid_of(shape)
    rng = np.random.default_rng(4)
    phi0 = rng.uniform(-2, -1, shape).astype(npdt(storage))
    pd0 = rng.uniform(-0.1, 0.1, shape).astype(npdt(storage))
    rho = dens(shape, 23, storage)
    origin = (0.03, -0.02, 0.01)
    s = solver(gpu_lib, shape, storage=storage, eta=0.5, origin=origin, bc=bc)
    o = Oracle(g, eta=0.5, origin=origin, bc=bc, storage=storage)
    s.set_state(to_dev(phi0), to_dev(pd0), 0.35 * g.dx)
    o.set_state(phi0.astype(np.float64), pd0.astype(np.float64), 0.35 * g.dx)
    tol = F64_TOL if storage == "f64" else F32_EMU_TOL
    assert rel(host(s.get_boundary()), gpu_lib.faces_to_flat(core.faces(o.Pn))) < tol
    s.step(to_dev(rho), 1.0, 0.4 * g.dx, 6)
    o.step(rho.astype(np.float64), 1.0, 0.4 * g.dx, 6)
    assert rel(host(s.potential()[0]), o.potential()[0]) < tol


def test_outgoing_relaxes_without_damping(gpu_lib):
    """eta = 0, zero start: through the outgoing boundary the transient leaves
    and the residual falls below 1e-3 after eight light-crossing half-widths,
    while the multipole Dirichlet boundary keeps the transient (R_f ~ 1)."""
    shape = (64, 64, 64)
    g = grid_of(shape)
    rho = dens(shape, 24, "f64", k=5)
    steps = int(round(8.0 / (0.4 * g.dx)))
    out = solver(gpu_lib, shape, storage="f64", bc="outgoing")
    dirichlet = solver(gpu_lib, shape, storage="f64", bc="multipole")
    for s in (out, dirichlet):
        s.step(to_dev(rho), 1.0, 0.4 * g.dx, steps)
    r_out = out.residual(to_dev(rho))[1]
    r_dir = dirichlet.residual(to_dev(rho))[1]
    assert r_out < 1e-3 and r_dir > 0.1, (r_out, r_dir)


def test_periodic_converges_to_fft_solution(gpu_lib):
    """Periodic box, damped: the GPU solution reaches the FFT solution of
    L_h phi = 4 pi G (rho - mean rho) (7-point symbol, mean zero)."""
    shape = (32, 24, 40)
    g = grid_of(shape)
    rho = dens(shape, 25, "f64", k=4)
    k = [2.0 * np.pi * np.fft.fftfreq(n) for n in shape]
    KZ, KY, KX = np.meshgrid(*k, indexing="ij")
    sym = (2.0 * np.cos(KX) + 2.0 * np.cos(KY) + 2.0 * np.cos(KZ) - 6.0) / g.dx ** 2
    sym[0, 0, 0] = 1.0
    ph = np.fft.fftn(4.0 * np.pi * (rho - rho.mean())) / sym
    ph[0, 0, 0] = 0.0
    want = np.real(np.fft.ifftn(ph))
    lam = (2.0 - 2.0 * np.cos(2.0 * np.pi / max(shape))) / g.dx ** 2
    s = solver(gpu_lib, shape, storage="f64", bc="periodic", eta=2.0 * np.sqrt(lam))
    s.step(to_dev(rho), 1.0, 0.4 * g.dx, 6000)
    phi = host(s.potential()[0])
    assert abs(phi.mean()) < 1e-10 * np.max(np.abs(want))
    assert rel(phi, want) < 1e-9
    assert s.residual(to_dev(rho))[0] < 1e-9


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_outgoing_checkpoint_bitwise(gpu_lib, storage):
    """The outgoing ghosts carry state: raw state + ghost faces restore a run
    bitwise (hgs_load_raw then hgs_set_boundary)."""
    shape = (24, 20, 28)
    g = grid_of(shape)
    rho = to_dev(dens(shape, 26, storage))
    a = solver(gpu_lib, shape, storage=storage, bc="outgoing")
    a.step(rho, 1.0, 0.4 * g.dx, 10)
    raw = a.save_raw()
    gh = a.get_boundary()
    a.step(rho, 1.0, 0.4 * g.dx, 10)
    b = solver(gpu_lib, shape, storage=storage, bc="outgoing")
    b.load_raw(*raw)
    b.set_boundary(gh)
    b.step(rho, 1.0, 0.4 * g.dx, 10)
    assert np.array_equal(host(a.potential()[0]), host(b.potential()[0]))
    assert np.array_equal(host(a.get_boundary()), host(b.get_boundary()))


def test_local_bc_rejected_in_batch_and_tuned(gpu_lib):
    """Local boundaries are refused in batches; the autotuner times every
    depth and tile for each of them (all three fuse substeps)."""
    hgs = gpu_lib
    with pytest.raises(hgs.HGSError):
        hgs.Batch([16, 32], bc="robin", storage="f32", device="cuda")
    rho = to_dev(dens((16, 16, 16), 27, "f32"))
    for bc in LOCAL:
        best, tile, times = hgs.autotune((16, 16, 16), rho, 1.0, 0.4 * 2.0 / 16, 4, storage="f32", bc=bc,
                                         device="cuda")
        assert 1 <= best <= 4 and 0 <= tile < max(1, hgs.tile_count(best)) and all(t > 0 for t in times)


@pytest.mark.parametrize("bc", LOCAL)
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(2, 2, 2), (3, 2, 4), (7, 9, 5), (23, 29, 37), (40, 33, 130), (70, 61, 66),
                                   (9, 150, 67)])
@pytest.mark.parametrize("T,tile", [(4, 0), (4, 1), (4, 2), (3, 0), (3, 1), (2, 0), (2, 1)])
def test_fused_local_bc_bitwise_equals_streaming(gpu_lib, bc, storage, shape, T, tile):
    """Robin, outgoing and periodic substeps fused T per launch give the
    streaming results bit for bit: the potential, phi^{n-1}, the ghost faces
    and g, over hydro steps whose substep counts are and are not multiples of
    T, with a dt change (phi^{n-1} rescaled), on grids smaller than one tile,
    with ragged tiles in every direction, and more tiles in y than in x.  The
    outgoing ghosts carry their own state from launch to launch, so a wrong
    ghost level anywhere inside a fused launch shows in the faces."""
    import torch

    g = grid_of(shape)
    rho = to_dev(dens(shape, 28, storage))
    origin = (0.03, -0.02, 0.01)
    a = solver(gpu_lib, shape, storage=storage, eta=0.7, origin=origin, bc=bc, tblock=1)
    b = solver(gpu_lib, shape, storage=storage, eta=0.7, origin=origin, bc=bc, tblock=T, tile=tile)
    assert a.tblock == 1 and b.tblock == T
    for dt, nsub in [(0.4, T), (0.4, 2 * T + 1), (0.3, 5), (0.45, 3 * T)]:
        a.step(rho, 1.0, dt * g.dx, nsub)
        b.step(rho, 1.0, dt * g.dx, nsub)
    ra, rb = a.save_raw(), b.save_raw()
    torch.cuda.synchronize()
    assert torch.equal(ra[0], rb[0]) and torch.equal(ra[1], rb[1])
    assert torch.equal(a.get_boundary(), b.get_boundary())
    assert all(torch.equal(u, v) for u, v in zip(a.accel(), b.accel()))


@pytest.mark.parametrize("tblock", [1, 4])
@pytest.mark.parametrize("bc", LOCAL)
def test_fused_local_bc_against_oracle_256(gpu_lib, bc, tblock):
    """At 256^3 FP32, fused depth 4 and one substep per launch (the two forms
    the bench times for these boundaries, the latter with its ghosts
    evaluated or advanced inside the substep), two hydro steps against the
    FP64 oracle at the FP32 bar."""
    import torch

    import workloads
    from oracle.core import Grid

    n = 256
    g = Grid.cube(n)
    rho = workloads.blob_density_torch(n, workloads.blob_params(0, 8), "cuda", torch.float32)
    r64 = rho.double().cpu().numpy()
    origin = (0.03, -0.02, 0.01)
    s = gpu_lib.Solver(n, storage="f32", eta=0.5, bc=bc, origin=origin, tblock=tblock)
    o = Oracle(g, eta=0.5, bc=bc, origin=origin)
    for _ in range(2):
        s.step(rho, 1.0, 0.4 * g.dx, 4)
        o.step(r64, 1.0, 0.4 * g.dx, 4)
    compare_state(s, o, "f32", F32_TOL)


def test_periodic_and_energy_256_against_oracle(gpu_lib):
    """At 256^3 (FP32, the size of the bench's next-row runs) the reductions
    take their 16-byte, unrolled paths: the periodic mean of rho inside one
    hydro step, and the energy sum W = 1/2 sum rho phi dx^3 of the result,
    against the FP64 oracle."""
    import torch

    import workloads
    from oracle.core import Grid

    n = 256
    g = Grid.cube(n)
    rho = workloads.blob_density_torch(n, workloads.blob_params(0, 8), "cuda", torch.float32)
    r64 = rho.double().cpu().numpy()
    ax = -1.0 + (np.arange(n) + 0.5) * g.dx
    p0 = (np.cos(np.pi * ax)[:, None, None] * np.sin(np.pi * ax)[None, :, None] * np.cos(np.pi * ax)[None, None, :])
    s = gpu_lib.Solver(n, storage="f32", eta=0.5, bc="periodic")
    o = Oracle(g, eta=0.5, bc="periodic")
    dt = 0.4 * g.dx
    s.set_state(torch.from_numpy(p0.astype(np.float32)).cuda(), None, dt)
    o.set_state(p0.astype(np.float32).astype(np.float64), None, dt)
    s.step(rho, 1.0, dt, 4)
    o.step(r64, 1.0, dt, 4)
    phi = s.potential(with_phidot=False)[0].double().cpu().numpy()
    ref = o.potential()[0]
    assert np.max(np.abs(phi - ref)) / np.max(np.abs(ref)) < 1e-4
    # the energy of the GPU's own potential, on the scale of its terms
    w = s.energy(rho)
    terms = 0.5 * r64 * phi * g.dx ** 3
    assert abs(w - terms.sum()) <= 1e-12 * np.abs(terms).sum()
