"""ctypes binding of the FP64 oracle core (hgs_oracle.c) plus a small solver
object with the same call sequence as the product API -- TEST INFRASTRUCTURE.

Fields are numpy float64 arrays.  Padded arrays have shape (nz+2, ny+2, nx+2)
(one ghost layer on each face, x fastest); compact arrays have shape
(nz, ny, nx).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hgs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile the oracle core with the host C compiler (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            i, d = ctypes.c_int, ctypes.c_double
            L.orc_moments.argtypes = [i, i, i, d, d, d, d, _dp, i, _dp, _dp, _dp]
            L.orc_boundary.argtypes = [i, i, i, d, d, d, d, _dp, i, d, _dp, _dp, _dp]
            L.orc_laplacian.argtypes = [i, i, i, d, _dp, _dp]
            L.orc_substeps.argtypes = [i, i, i, d, _dp, _dp, _dp, d, d, d, d, i, i]
            L.orc_gradient.argtypes = [i, i, i, d, _dp, _dp, _dp, _dp]
            L.orc_residual.argtypes = [i, i, i, d, _dp, _dp, d, _dp]
            L.orc_substeps_local.argtypes = [i, i, i, d, d, d, d, _dp, i, _dp, _dp, _dp, d, d, d, d, d, i, i]
            L.orc_local_ghosts.argtypes = [i, i, i, d, d, d, d, _dp, i, _dp, i]
            L.orc_residual_local.argtypes = [i, i, i, d, _dp, _dp, d, d, _dp]
            L.orc_max_threads.restype = ctypes.c_int
            L.orc_max_threads.argtypes = []
            L.orc_set_threads.restype = None
            L.orc_set_threads.argtypes = [i]
            for f in ("orc_moments", "orc_boundary", "orc_laplacian", "orc_substeps",
                      "orc_gradient", "orc_residual", "orc_substeps_local", "orc_local_ghosts",
                      "orc_residual_local"):
                getattr(L, f).restype = None
            _lib = L
    return _lib


def max_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().orc_max_threads())


def set_threads(n: int) -> None:
    """Threads for the oracle's later parallel loops (n >= 1)."""
    lib().orc_set_threads(int(n))


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


@dataclass(frozen=True)
class Grid:
    """Cell-centred uniform grid; cell (i,j,k) centre = origin corner + (idx+1/2) dx."""

    nx: int
    ny: int
    nz: int
    x0: float = -1.0
    y0: float = -1.0
    z0: float = -1.0
    dx: float = 2.0 / 64

    @staticmethod
    def cube(n: int, lo: float = -1.0, hi: float = 1.0) -> "Grid":
        return Grid(n, n, n, lo, lo, lo, (hi - lo) / n)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def pshape(self):
        return (self.nz + 2, self.ny + 2, self.nx + 2)

    def centres(self):
        """1D arrays of cell-centre coordinates including the ghost layers
        (index 0 and -1 are the ghost centres)."""
        x = self.x0 + (np.arange(-1, self.nx + 1) + 0.5) * self.dx
        y = self.y0 + (np.arange(-1, self.ny + 1) + 0.5) * self.dx
        z = self.z0 + (np.arange(-1, self.nz + 1) + 0.5) * self.dx
        return x, y, z


def padded(g: Grid) -> np.ndarray:
    return np.zeros(g.pshape)


def interior(P: np.ndarray) -> np.ndarray:
    return P[1:-1, 1:-1, 1:-1]


FACE_NAMES = ("x-", "x+", "y-", "y+", "z-", "z+")


def faces(P: np.ndarray):
    """The six ghost faces of a padded array, in the order x-, x+, y-, y+, z-, z+.
    x faces have shape (nz, ny), y faces (nz, nx), z faces (ny, nx)."""
    return (P[1:-1, 1:-1, 0].copy(), P[1:-1, 1:-1, -1].copy(),
            P[1:-1, 0, 1:-1].copy(), P[1:-1, -1, 1:-1].copy(),
            P[0, 1:-1, 1:-1].copy(), P[-1, 1:-1, 1:-1].copy())


def set_faces(P: np.ndarray, f) -> None:
    P[1:-1, 1:-1, 0] = f[0]
    P[1:-1, 1:-1, -1] = f[1]
    P[1:-1, 0, 1:-1] = f[2]
    P[1:-1, -1, 1:-1] = f[3]
    P[0, 1:-1, 1:-1] = f[4]
    P[-1, 1:-1, 1:-1] = f[5]


def moments(g: Grid, rho: np.ndarray, lmax: int, origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Complex Q_lm, index l*l + l + m (m = -l..l)."""
    assert 0 <= lmax <= 4
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    assert rho.shape == g.shape
    nq = (lmax + 1) ** 2
    qr = np.zeros(nq)
    qi = np.zeros(nq)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    lib().orc_moments(g.nx, g.ny, g.nz, g.x0, g.y0, g.z0, g.dx, _p(o), lmax, _p(rho), _p(qr), _p(qi))
    return qr + 1j * qi


def boundary(g: Grid, q: np.ndarray, lmax: int, G: float, P: np.ndarray, origin=(0.0, 0.0, 0.0)) -> None:
    """Write multipole ghost values into the padded array P (in place)."""
    qr = np.ascontiguousarray(q.real, dtype=np.float64)
    qi = np.ascontiguousarray(q.imag, dtype=np.float64)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    lib().orc_boundary(g.nx, g.ny, g.nz, g.x0, g.y0, g.z0, g.dx, _p(o), lmax, G, _p(qr), _p(qi), _p(P))


def laplacian(g: Grid, P: np.ndarray) -> np.ndarray:
    out = np.zeros(g.shape)
    lib().orc_laplacian(g.nx, g.ny, g.nz, g.dx, _p(P), _p(out))
    return out


def substeps(g: Grid, Pn: np.ndarray, Pnm1: np.ndarray, rho: np.ndarray, c: float, dt: float,
             eta: float, G: float, nsub: int, f32: bool = False) -> None:
    """Advance (Pn, Pnm1) by nsub leapfrog substeps, in place."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    lib().orc_substeps(g.nx, g.ny, g.nz, g.dx, _p(Pn), _p(Pnm1), _p(rho), c, dt, eta, G, nsub, int(f32))


# local outer boundaries: the ghost layer follows the interior every substep
LOCAL_BC = {"robin": 2, "outgoing": 3, "periodic": 4}


def substeps_local(g: Grid, bc: str, Pn: np.ndarray, Pnm1: np.ndarray, rho: np.ndarray, c: float, dt: float,
                   eta: float, G: float, nsub: int, origin=(0.0, 0.0, 0.0), rbar: float = 0.0,
                   f32: bool = False) -> None:
    """Advance (Pn, Pnm1) by nsub substeps with a local boundary, in place.
    rbar is subtracted from rho in the source (the domain mean for periodic)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    lib().orc_substeps_local(g.nx, g.ny, g.nz, g.x0, g.y0, g.z0, g.dx, _p(o), LOCAL_BC[bc], _p(Pn), _p(Pnm1),
                             _p(rho), rbar, c, dt, eta, G, nsub, int(f32))


def local_ghosts(g: Grid, bc: str, P: np.ndarray, origin=(0.0, 0.0, 0.0), f32: bool = False) -> None:
    """Steady form of a local rule on the ghosts of P (Robin for robin and
    outgoing, the wrap for periodic), in place."""
    o = np.ascontiguousarray(origin, dtype=np.float64)
    lib().orc_local_ghosts(g.nx, g.ny, g.nz, g.x0, g.y0, g.z0, g.dx, _p(o), LOCAL_BC[bc], _p(P), int(f32))


def residual_local(g: Grid, P: np.ndarray, rho: np.ndarray, G: float, rbar: float = 0.0) -> np.ndarray:
    """[R_b (= R_f), R_f, ||phi||, nonfinite] with b = s = 4 pi G (rho - rbar)."""
    out = np.zeros(4)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    lib().orc_residual_local(g.nx, g.ny, g.nz, g.dx, _p(P), _p(rho), G, rbar, _p(out))
    return out


def energy(g: Grid, rho: np.ndarray, phi: np.ndarray) -> float:
    """Gravitational energy W = 1/2 sum_cells rho phi dx^3 (phi compact)."""
    return float(0.5 * np.sum(np.asarray(rho, dtype=np.float64) * np.asarray(phi, dtype=np.float64)) * g.dx ** 3)


def gradient(g: Grid, P: np.ndarray):
    gx, gy, gz = np.zeros(g.shape), np.zeros(g.shape), np.zeros(g.shape)
    lib().orc_gradient(g.nx, g.ny, g.nz, g.dx, _p(P), _p(gx), _p(gy), _p(gz))
    return gx, gy, gz


def residual(g: Grid, P: np.ndarray, rho: np.ndarray, G: float) -> np.ndarray:
    """[R_b, R_f, ||phi||, nonfinite]."""
    out = np.zeros(4)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    lib().orc_residual(g.nx, g.ny, g.nz, g.dx, _p(P), _p(rho), G, _p(out))
    return out


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


class Oracle:
    """Same call sequence as the product solver (init / step / potential /
    accel / set_state / residual), written with the plain routines above.

    storage="f64" is the FP64 oracle proper.  storage="f32" additionally rounds
    every stored field (ghosts, each new time level, set_state inputs) to
    binary32 while keeping FP64 arithmetic -- an emulation of FP32 storage used
    for tighter checks than the FP64-oracle tolerance.
    """

    def __init__(self, g: Grid, G: float = 1.0, lmax: int = 4, origin=(0.0, 0.0, 0.0), eta: float = 0.0,
                 bc: str = "multipole", storage: str = "f64"):
        assert bc in ("multipole", "user") or bc in LOCAL_BC
        assert storage in ("f64", "f32")
        self.g, self.G, self.lmax, self.origin, self.eta, self.bc = g, G, lmax, origin, eta, bc
        self.f32 = storage == "f32"
        self.Pn = padded(g)
        self.Pnm1 = padded(g)
        self.dt_prev = 0.0
        self.q = None

    def _store(self, a):
        return _f32(a) if self.f32 else np.asarray(a, dtype=np.float64)

    def set_boundary(self, face_list) -> None:
        f = [self._store(x) for x in face_list]
        set_faces(self.Pn, f)
        set_faces(self.Pnm1, f)

    def step(self, rho: np.ndarray, c: float, dt: float, nsub: int) -> None:
        rho = np.asarray(rho, dtype=np.float64)
        if self.bc == "multipole":
            self.q = moments(self.g, rho, self.lmax, self.origin)
            tmp = padded(self.g)
            boundary(self.g, self.q, self.lmax, self.G, tmp, self.origin)
            self.set_boundary(faces(tmp))
        if self.dt_prev > 0.0 and dt != self.dt_prev:
            # keep the time derivative (phi^n - phi^{n-1}) / dt when the step changes
            In, Inm1 = interior(self.Pn), interior(self.Pnm1)
            Inm1[...] = self._store(In - (dt / self.dt_prev) * (In - Inm1))
        if self.bc in LOCAL_BC:
            substeps_local(self.g, self.bc, self.Pn, self.Pnm1, rho, c, dt, self.eta, self.G, nsub, self.origin,
                           self.rbar(rho), self.f32)
        else:
            substeps(self.g, self.Pn, self.Pnm1, rho, c, dt, self.eta, self.G, nsub, self.f32)
        self.dt_prev = dt

    def rbar(self, rho) -> float:
        """Density subtracted from the source: the domain mean when periodic."""
        return float(np.mean(np.asarray(rho, dtype=np.float64))) if self.bc == "periodic" else 0.0

    def potential(self):
        phi = interior(self.Pn).copy()
        phidot = None
        if self.dt_prev > 0.0:
            phidot = (interior(self.Pn) - interior(self.Pnm1)) / self.dt_prev
        return phi, phidot

    def accel(self):
        return gradient(self.g, self.Pn)

    def set_state(self, phi, phidot, dt: float) -> None:
        phi = self._store(phi)
        interior(self.Pn)[...] = phi
        pd = np.zeros(self.g.shape) if phidot is None else self._store(phidot)
        interior(self.Pnm1)[...] = self._store(phi - dt * pd)
        if self.bc in LOCAL_BC:
            local_ghosts(self.g, self.bc, self.Pn, self.origin, self.f32)
        self.dt_prev = dt

    def residual(self, rho) -> np.ndarray:
        rho = np.asarray(rho, dtype=np.float64)
        if self.bc in LOCAL_BC:
            return residual_local(self.g, self.Pn, rho, self.G, self.rbar(rho))
        return residual(self.g, self.Pn, rho, self.G)
