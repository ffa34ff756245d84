"""Python binding of the C ABI in include/hgs.h (ctypes; argument marshalling only).

Every step of the method runs in the HIP library libhgs.so.  PyTorch supplies
device memory (the workspace and I/O tensors) and the stream.  If the library
has not been built, importing this module raises ImportError: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HGS_LIBRARY") or os.path.join(_HERE, "libhgs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first (python -c 'import __graft_entry__ as g; g.build()')")

# One HIP runtime per process: torch ships its own libamdhip64 (soname
# libamdhip64.so.7) and loads it by an unversioned name from its own directory.
# Loading torch first lets libhgs.so's dependency on libamdhip64.so.7 bind to
# that already-loaded runtime instead of starting a second one, which would
# find no device once torch's runtime holds it.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

HGS_OK, HGS_ERR_ARG, HGS_ERR_CFL, HGS_ERR_WORKSPACE, HGS_ERR_DEVICE, HGS_ERR_NONFINITE, HGS_ERR_STATE = range(7)
HGS_F64, HGS_F32 = 0, 1
HGS_BC_MULTIPOLE, HGS_BC_USER, HGS_BC_ROBIN, HGS_BC_OUTGOING, HGS_BC_PERIODIC = 0, 1, 2, 3, 4
BC_NAMES = {"multipole": HGS_BC_MULTIPOLE, "user": HGS_BC_USER, "robin": HGS_BC_ROBIN,
            "outgoing": HGS_BC_OUTGOING, "periodic": HGS_BC_PERIODIC}
TMAX = 4
LMAX = 4


class Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double),
        ("dx", ctypes.c_double), ("G", ctypes.c_double), ("origin", ctypes.c_double * 3),
        ("lmax", ctypes.c_int32), ("bc", ctypes.c_int32), ("storage", ctypes.c_int32),
        ("tblock", ctypes.c_int32), ("eta", ctypes.c_double), ("stream", ctypes.c_void_p),
    ]


_vp, _cp, _dp = ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double)
_i32, _dbl, _sz = ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
_CFG = ctypes.POINTER(Config)

_SIGS = {
    "hgs_config_cube": (_i32, [_CFG, _i32, _dbl, _dbl]),
    "hgs_workspace_bytes": (_i32, [_CFG, ctypes.POINTER(_sz)]),
    "hgs_init": (_i32, [_CFG, _vp, _sz, ctypes.POINTER(_vp)]),
    "hgs_step": (_i32, [_vp, _vp, _dbl, _dbl, _i32]),
    "hgs_validate_step": (_i32, [_CFG, _vp, _dbl, _dbl, _i32]),
    "hgs_potential": (_i32, [_vp, _vp, _vp]),
    "hgs_accel": (_i32, [_vp, _vp, _vp, _vp]),
    "hgs_accel_box": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp]),
    "hgs_set_state": (_i32, [_vp, _vp, _vp, _dbl]),
    "hgs_set_boundary": (_i32, [_vp, _vp]),
    "hgs_get_boundary": (_i32, [_vp, _vp]),
    "hgs_moments": (_i32, [_vp, _dp]),
    "hgs_residual": (_i32, [_vp, _vp, _dp]),
    "hgs_max_signal_speed": (_i32, [_vp, _vp, _vp, _vp, _vp, _dp]),
    "hgs_hydro_step": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _dbl, _dbl, _dbl, _dp, ctypes.POINTER(_i32), _dp]),
    "hgs_energy": (_i32, [_vp, _vp, _dp]),
    "hgs_embed": (_i32, [_vp, _i32, _i32, _i32, _i32, _vp, _i32, _vp]),
    "hgs_extract": (_i32, [_vp, _i32, _i32, _i32, _i32, _vp, _i32, _vp]),
    "hgs_nest_source": (_i32, [_vp, _i32, _i32, _i32, _i32, _vp, _i32, _vp]),
    "hgs_nest_ghosts": (_i32, [_vp, _i32, _i32, _i32, _dp, _dbl, _i32, _i32, _i32, _dp, _dbl, _vp, _i32, _vp]),
    "hgs_save_raw": (_i32, [_vp, _vp, _vp, _dp]),
    "hgs_load_raw": (_i32, [_vp, _vp, _vp, _dbl]),
    "hgs_poisson_direct": (_i32, [_vp, _vp, _vp, _sz]),
    "hgs_multipole_boundary": (_i32, [_vp, _vp]),
    "hgs_keep_start_if_better": (_i32, [_vp, _vp, _vp]),
    "hgs_set_tblock": (_i32, [_vp, _i32]),
    "hgs_get_tblock": (_i32, [_vp]),
    "hgs_tile_count": (_i32, [_i32]),
    "hgs_tile_shape": (_i32, [_i32, _i32, _i32, ctypes.POINTER(_i32)]),
    "hgs_set_tile": (_i32, [_vp, _i32]),
    "hgs_get_tile": (_i32, [_vp]),
    "hgs_timing_enable": (_i32, [_vp, _i32]),
    "hgs_timing_read": (_i32, [_vp, _i32, _dp]),
    "hgs_workspace_bytes_batch": (_i32, [_CFG, _i32, ctypes.POINTER(_sz)]),
    "hgs_init_batch": (_i32, [_CFG, _i32, _vp, _sz, ctypes.POINTER(_vp)]),
    "hgs_batch_grid": (_i32, [_vp, _i32, ctypes.POINTER(_vp)]),
    "hgs_step_batch": (_i32, [_vp, ctypes.POINTER(_vp), _dp, _dp, _i32]),
    "hgs_batch_used_graph": (_i32, [_vp]),
    "hgs_batch_set_launch": (_i32, [_vp, _i32]),
    "hgs_batch_get_launch": (_i32, [_vp]),
    "hgs_batch_last_error": (_cp, [_vp]),
    "hgs_destroy_batch": (_i32, [_vp]),
    "hgs_nn_conv3d": (_i32, [_vp, _vp, _vp, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp]),
    "hgs_nn_flip_weights": (_i32, [_vp, _vp, _vp]),
    "hgs_nn_wgrad_workspace_bytes": (_i32, [_i32, _i32, _i32, _i32, ctypes.POINTER(_sz)]),
    "hgs_nn_wgrad": (_i32, [_vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _sz, _vp]),
    "hgs_nn_pack": (_i32, [_vp, _i32, _i32, ctypes.c_int64, _vp, _vp]),
    "hgs_nn_unpack": (_i32, [_vp, _i32, _i32, ctypes.c_int64, _vp, _vp]),
    "hgs_nn_mse": (_i32, [_vp, _vp, _i32, _i32, ctypes.c_int64, _vp, _vp, _vp, _vp]),
    "hgs_nn_maxabs": (_i32, [_vp, _i32, ctypes.c_int64, _vp, _vp, _vp]),
    "hgs_nn_maxabs_noalloc": (_i32, [_vp, _i32, ctypes.c_int64, _vp, _vp]),
    "hgs_nn_features": (_i32, [_vp, _vp, _vp, _i32, _i32, _i32, _i32, _dbl, _vp, _vp]),
    "hgs_nn_compose": (_i32, [_vp, _vp, _vp, _i32, ctypes.c_int64, _dbl, _vp, _vp, _vp]),
    "hgs_nn_lapmse": (_i32, [_vp, _vp, _i32, _i32, _i32, _i32, _i32, _i32, ctypes.c_float, _vp, _vp, _vp, _vp,
                             _vp]),
    "hgs_nn_adam": (_i32, [_vp, _vp, _vp, _vp, _vp, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, _i32, _vp]),
    "hgs_nn_restrict2": (_i32, [_vp, _vp, _i32, _i32, _i32, _i32, _i32, _vp]),
    "hgs_nn_prolong2": (_i32, [_vp, _vp, _i32, _i32, _i32, _i32, _i32, _vp]),
    "hgs_nn_last_error": (_cp, []),
    "hgs_autotune": (_i32, [_CFG, _vp, _dbl, _dbl, _i32, _vp, _sz, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                            _dp]),
    "hgs_destroy": (_i32, [_vp]),
    "hgs_status_str": (_cp, [_i32]),
    "hgs_last_error": (_cp, [_vp]),
    "hgs_abi_version": (_i32, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class HGSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_lib.hgs_status_str(status).decode()}: {msg}")
        self.status = status


def _check(status: int, ctx=None):
    if status != HGS_OK:
        raise HGSError(status, _lib.hgs_last_error(ctx).decode())


def library():
    """The loaded ctypes library (for tests of the raw ABI)."""
    return _lib


def make_config(shape, x0=(-1.0, -1.0, -1.0), dx: Optional[float] = None, G: float = 1.0,
                origin=(0.0, 0.0, 0.0), lmax: int = 4, bc: str = "multipole", storage: str = "f32",
                tblock: int = 0, eta: float = 0.0, stream: int = 0) -> Config:
    """shape = (nz, ny, nx) or n; default dx spans [-1, 1] along x."""
    nz, ny, nx = (shape, shape, shape) if np.isscalar(shape) else shape
    c = Config()
    c.nx, c.ny, c.nz = int(nx), int(ny), int(nz)
    c.x0, c.y0, c.z0 = (float(v) for v in x0)
    c.dx = float(dx) if dx is not None else 2.0 / nx
    c.G = float(G)
    c.origin = (ctypes.c_double * 3)(*[float(v) for v in origin])
    c.lmax = int(lmax)
    c.bc = BC_NAMES[bc]
    c.storage = {"f64": HGS_F64, "f32": HGS_F32}[storage]
    c.tblock = int(tblock)
    c.eta = float(eta)
    c.stream = int(stream) or None
    return c


def workspace_bytes(cfg: Config) -> int:
    n = _sz(0)
    _check(_lib.hgs_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n)))
    return n.value


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Solver:
    """One grid; all tensors live on the CUDA (HIP) device in the storage dtype."""

    def __init__(self, shape, x0=(-1.0, -1.0, -1.0), dx: Optional[float] = None, G: float = 1.0,
                 origin=(0.0, 0.0, 0.0), lmax: int = 4, bc: str = "multipole", storage: str = "f32",
                 tblock: int = 0, eta: float = 0.0, device="cuda", stream=None, tile: int = 0):
        import torch

        self.torch = torch
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.dtype = torch.float32 if storage == "f32" else torch.float64
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.cfg = make_config(shape, x0, dx, G, origin, lmax, bc, storage, tblock, eta, self.stream.cuda_stream)
        self.shape = (self.cfg.nz, self.cfg.ny, self.cfg.nx)
        nbytes = workspace_bytes(self.cfg)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = _vp()
        _check(_lib.hgs_init(ctypes.byref(self.cfg), self.workspace.data_ptr(), nbytes, ctypes.byref(h)))
        self._h = h
        self._owned = True
        if tile:
            self.set_tile(tile)

    @classmethod
    def _view(cls, handle, cfg, device, dtype, stream, owner):
        """A Solver over a context owned by a Batch (not destroyed by close())."""
        import torch

        obj = cls.__new__(cls)
        obj.torch = torch
        obj.device = device
        obj.dtype = dtype
        obj.stream = stream
        obj.cfg = cfg
        obj.shape = (cfg.nz, cfg.ny, cfg.nx)
        obj.workspace = None
        obj._h = handle
        obj._owned = False
        obj._owner = owner  # keeps the batch (and its workspace) alive
        return obj

    # -- helpers
    def _need(self, t, shape=None):
        shape = self.shape if shape is None else shape
        if t is None:
            return None
        if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected a contiguous {self.dtype} tensor of shape {shape} on {self.device}")
        return t

    def _new(self, shape=None):
        return self.torch.empty(self.shape if shape is None else shape, dtype=self.dtype, device=self.device)

    @property
    def face_count(self) -> int:
        nz, ny, nx = self.shape
        return 2 * (nz * ny + nz * nx + ny * nx)

    @property
    def dx(self) -> float:
        return self.cfg.dx

    # -- API
    def step(self, rho, c_g: float, dt: float, nsub: int) -> None:
        self._need(rho)
        _check(_lib.hgs_step(self._h, rho.data_ptr(), float(c_g), float(dt), int(nsub)), self._h)

    def potential(self, with_phidot: bool = True, out=None):
        """(phi, phidot or None); out: an existing tensor for phi."""
        phi = self._new() if out is None else self._need(out)
        pd = self._new() if with_phidot else None
        _check(_lib.hgs_potential(self._h, phi.data_ptr(), _ptr(pd)), self._h)
        return phi, pd

    def multipole_boundary(self, rho) -> None:
        """Ghost shell from the moments of rho into the current state (bc = multipole)."""
        self._need(rho)
        _check(_lib.hgs_multipole_boundary(self._h, rho.data_ptr()), self._h)

    def keep_start_if_better(self, rho, kept=None):
        """Reset the state to zero unless its R_b for rho is below the zero
        start's (decided on the device, no synchronisation); kept: device
        int32 tensor of one element receiving 1 (kept) or 0 (reset)."""
        self._need(rho)
        _check(_lib.hgs_keep_start_if_better(self._h, rho.data_ptr(), _ptr(kept)), self._h)
        return kept

    def poisson_direct(self, rho, scratch=None):
        """Set the state to the discrete Dirichlet Poisson solution for rho
        (phidot = 0); scratch: float64 device tensor of 2 nx ny nz elements
        (allocated if None)."""
        self._need(rho)
        nz, ny, nx = self.shape
        if scratch is None:
            scratch = self.torch.empty(2 * nx * ny * nz, dtype=self.torch.float64, device=self.device)
        _check(_lib.hgs_poisson_direct(self._h, rho.data_ptr(), scratch.data_ptr(),
                                       scratch.numel() * scratch.element_size()), self._h)

    def accel(self, out=None):
        g = [self._new() for _ in range(3)] if out is None else [self._need(t) for t in out]
        _check(_lib.hgs_accel(self._h, *(t.data_ptr() for t in g)), self._h)
        return tuple(g)

    def accel_box(self, start, shape, out=None):
        """g on the box of the interior that starts at cell start = (k0, j0, i0)
        and has shape (bz, by, bx), as three compact arrays of that shape."""
        (k0, j0, i0), shape = start, tuple(int(v) for v in shape)
        g = [self._new(shape) for _ in range(3)] if out is None else [self._need(t, shape) for t in out]
        _check(_lib.hgs_accel_box(self._h, int(i0), int(j0), int(k0), shape[2], shape[1], shape[0],
                                  *(t.data_ptr() for t in g)), self._h)
        return tuple(g)

    def set_state(self, phi, phidot, dt: float) -> None:
        self._need(phi)
        self._need(phidot)
        _check(_lib.hgs_set_state(self._h, phi.data_ptr(), _ptr(phidot), float(dt)), self._h)

    def set_boundary(self, ghosts) -> None:
        self._need(ghosts, (self.face_count,))
        _check(_lib.hgs_set_boundary(self._h, ghosts.data_ptr()), self._h)

    def get_boundary(self):
        out = self._new((self.face_count,))
        _check(_lib.hgs_get_boundary(self._h, out.data_ptr()), self._h)
        return out

    def moments(self) -> np.ndarray:
        n = (self.cfg.lmax + 1) ** 2
        buf = (ctypes.c_double * (2 * n))()
        _check(_lib.hgs_moments(self._h, buf), self._h)
        a = np.frombuffer(buf, dtype=np.float64).copy()
        return a[0::2] + 1j * a[1::2]

    def residual(self, rho) -> np.ndarray:
        """[R_b, R_f, ||phi||, nonfinite]; raises HGSError(HGS_ERR_NONFINITE) on NaN/Inf."""
        self._need(rho)
        out = (ctypes.c_double * 4)()
        st = _lib.hgs_residual(self._h, rho.data_ptr(), out)
        res = np.frombuffer(out, dtype=np.float64).copy()
        if st == HGS_ERR_NONFINITE:
            err = HGSError(st, _lib.hgs_last_error(self._h).decode())
            err.values = res
            raise err
        _check(st, self._h)
        return res

    def max_signal_speed(self, cs, v=None) -> float:
        """max over cells of c_s + |v|; v = (vx, vy, vz) or None."""
        self._need(cs)
        vs = [None, None, None] if v is None else list(v)
        for a in vs:
            self._need(a)
        out = ctypes.c_double(0.0)
        _check(_lib.hgs_max_signal_speed(self._h, cs.data_ptr(), *(_ptr(a) for a in vs), ctypes.byref(out)), self._h)
        return out.value

    def hydro_step(self, rho, cs, v=None, k_g: float = 5.0, courant_hydro: float = 0.3,
                   courant_grav: float = 0.3):
        """One coupled hydrodynamical step (c_g = k_g max(c_s + |v|), nsub
        substeps); returns (dt_hydro, nsub, c_g)."""
        self._need(rho)
        self._need(cs)
        vs = [None, None, None] if v is None else list(v)
        for a in vs:
            self._need(a)
        dth, cg = ctypes.c_double(0.0), ctypes.c_double(0.0)
        n = _i32(0)
        _check(_lib.hgs_hydro_step(self._h, rho.data_ptr(), cs.data_ptr(), *(_ptr(a) for a in vs), float(k_g),
                                   float(courant_hydro), float(courant_grav), ctypes.byref(dth), ctypes.byref(n),
                                   ctypes.byref(cg)), self._h)
        return dth.value, int(n.value), cg.value

    def energy(self, rho) -> float:
        """W = 1/2 sum rho phi dx^3 of the current potential."""
        self._need(rho)
        out = ctypes.c_double(0.0)
        _check(_lib.hgs_energy(self._h, rho.data_ptr(), ctypes.byref(out)), self._h)
        return out.value

    def save_raw(self):
        a, b = self._new(), self._new()
        dtp = ctypes.c_double(0.0)
        _check(_lib.hgs_save_raw(self._h, a.data_ptr(), b.data_ptr(), ctypes.byref(dtp)), self._h)
        return a, b, dtp.value

    def load_raw(self, phi_n, phi_nm1, dt_prev: float) -> None:
        self._need(phi_n)
        self._need(phi_nm1)
        _check(_lib.hgs_load_raw(self._h, phi_n.data_ptr(), phi_nm1.data_ptr(), float(dt_prev)), self._h)

    KERNEL_KINDS = {"stencil": 0, "multipole": 1, "gradient": 2}

    def timing(self, enable: bool) -> None:
        _check(_lib.hgs_timing_enable(self._h, int(bool(enable))), self._h)

    def timing_read(self, kind: str = "stencil") -> dict:
        out = (ctypes.c_double * 4)()
        _check(_lib.hgs_timing_read(self._h, self.KERNEL_KINDS[kind], out), self._h)
        n, ms, nbytes, upd = list(out)
        return {"launches": int(n), "ms": ms, "bytes": nbytes, "updates": upd}

    def set_tblock(self, t: int) -> None:
        _check(_lib.hgs_set_tblock(self._h, int(t)), self._h)

    @property
    def tblock(self) -> int:
        return int(_lib.hgs_get_tblock(self._h))

    def set_tile(self, tile: int) -> None:
        _check(_lib.hgs_set_tile(self._h, int(tile)), self._h)

    @property
    def tile(self) -> int:
        return int(_lib.hgs_get_tile(self._h))

    def close(self) -> None:
        if getattr(self, "_h", None) and getattr(self, "_owned", True):
            _lib.hgs_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ExtendedSolver:
    """A solver on a grid wider than the hydrodynamics region by `ext` cells on
    every side, the extension treated as vacuum (Sec. 4: a cheap way to move a
    local boundary away from the matter).  rho, phi and g are exchanged on the
    hydrodynamics region (nz, ny, nx) only; hgs_embed / hgs_extract move rho
    and phi, and g comes from hgs_accel_box on that region."""

    def __init__(self, shape, ext: int, x0=(-1.0, -1.0, -1.0), dx: Optional[float] = None, bc: str = "outgoing",
                 **kw):
        import torch

        nz, ny, nx = (shape, shape, shape) if np.isscalar(shape) else shape
        dx = float(dx) if dx is not None else 2.0 / nx
        self.inner = (nz, ny, nx)
        self.ext = int(ext)
        e = self.ext
        self.solver = Solver((nz + 2 * e, ny + 2 * e, nx + 2 * e),
                             x0=tuple(float(v) - e * dx for v in x0), dx=dx, bc=bc, **kw)
        s = self.solver
        self.dtype, self.device, self.stream = s.dtype, s.device, s.stream
        self._code = HGS_F32 if s.dtype == torch.float32 else HGS_F64
        self._rho = torch.empty(s.shape, dtype=s.dtype, device=s.device)

    def _in(self, t):
        if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() or tuple(t.shape) != self.inner:
            raise ValueError(f"expected a contiguous {self.dtype} tensor of shape {self.inner} on {self.device}")
        return t

    def embed(self, inner, outer) -> None:
        nz, ny, nx = self.inner
        _check(_lib.hgs_embed(self._in(inner).data_ptr(), nx, ny, nz, self.ext, outer.data_ptr(), self._code,
                              self.stream.cuda_stream))

    def extract(self, outer, inner=None):
        nz, ny, nx = self.inner
        out = self.solver.torch.empty(self.inner, dtype=self.dtype, device=self.device) if inner is None else inner
        _check(_lib.hgs_extract(outer.data_ptr(), nx, ny, nz, self.ext, self._in(out).data_ptr(), self._code,
                                self.stream.cuda_stream))
        return out

    def step(self, rho, c_g: float, dt: float, nsub: int) -> None:
        self.embed(rho, self._rho)
        self.solver.step(self._rho, c_g, dt, nsub)

    def potential(self, with_phidot: bool = True):
        phi, pd = self.solver.potential(with_phidot)
        return self.extract(phi), (self.extract(pd) if pd is not None else None)

    def accel(self, out=None):
        """g on the hydrodynamics region only (the gradient of the extension
        is never computed)."""
        e = self.ext
        return self.solver.accel_box((e, e, e), self.inner, out)

    def residual(self, rho) -> np.ndarray:
        """Residual over the whole wider grid (rho embedded)."""
        self.embed(rho, self._rho)
        return self.solver.residual(self._rho)

    def close(self) -> None:
        self.solver.close()


class NestedSolver:
    """A fine grid whose outer boundary comes from coarse outer levels (Sec. 4
    names nested grids as a way to move the boundary out cheaply).  Level 1
    has cell size 2 dx, covers the fine grid and `ext` of its cells more on
    every side; each further level (up to `levels - 1`) does the same around
    the one inside it.  The outermost level has a local boundary (Robin or
    outgoing), every inner level frozen Dirichlet ghosts.  Per hydrodynamical
    step: the densities restricted level by level (hgs_nest_source), then from
    the outermost level inwards: level l takes ceil(n_{l-1} / 2) substeps
    spanning nsub * dt (n_0 = nsub), and the level inside it gets its ghosts
    interpolated from it (hgs_nest_ghosts) before its own substeps.  rho, phi
    and g live on the fine grid (nz, ny, nx); every level but the outermost
    needs even sizes."""

    def __init__(self, shape, ext: int, x0=(-1.0, -1.0, -1.0), dx: Optional[float] = None, bc: str = "robin",
                 storage: str = "f32", eta: float = 0.0, G: float = 1.0, origin=(0.0, 0.0, 0.0), tblock: int = 0,
                 device="cuda", stream=None, levels: int = 2):
        import torch

        nz, ny, nx = (shape, shape, shape) if np.isscalar(shape) else shape
        if bc not in ("robin", "outgoing"):
            raise ValueError("the coarse level needs a local boundary: 'robin' or 'outgoing'")
        if int(ext) < 1:
            raise ValueError("ext must be at least 1")
        if int(levels) < 2:
            raise ValueError("levels must be at least 2 (the fine grid and one coarse level)")
        self.ext = e = int(ext)
        dx = float(dx) if dx is not None else 2.0 / nx
        sizes, corners, cells = [(nz, ny, nx)], [tuple(float(v) for v in x0)], [dx]
        for _ in range(int(levels) - 1):
            if any(v % 2 for v in sizes[-1]):
                raise ValueError(f"a level of shape {sizes[-1]} is not even: 2 x 2 x 2 cells per coarser cell")
            h = 2.0 * cells[-1]
            sizes.append(tuple(v // 2 + 2 * e for v in sizes[-1]))
            corners.append(tuple(v - e * h for v in corners[-1]))
            cells.append(h)
        L = len(sizes)
        self.solvers = []
        for i in range(L):
            outer = i == L - 1
            kw = dict(x0=corners[i], dx=cells[i], G=G, origin=origin, bc=bc if outer else "user", storage=storage,
                      eta=eta)
            if i == 0:
                s = Solver(sizes[0], tblock=tblock, device=device, stream=stream, **kw)
            else:
                s = Solver(sizes[i], device=self.solvers[0].device, stream=self.solvers[0].stream, **kw)
            self.solvers.append(s)
        self.fine, self.coarse = self.solvers[0], self.solvers[1]
        f = self.fine
        self.shape, self.dtype, self.device, self.stream = f.shape, f.dtype, f.device, f.stream
        self._code = HGS_F32 if f.dtype == torch.float32 else HGS_F64
        self._rho = [None] + [torch.empty(s.shape, dtype=f.dtype, device=f.device) for s in self.solvers[1:]]
        self._faces = [torch.empty(s.face_count, dtype=f.dtype, device=f.device) for s in self.solvers[:-1]]
        self._x0 = [(ctypes.c_double * 3)(s.cfg.x0, s.cfg.y0, s.cfg.z0) for s in self.solvers]

    def coarse_source(self, rho, level: int = 1):
        """Density of `level` (>= 1) from the density of the level inside it."""
        nz, ny, nx = self.solvers[level - 1].shape
        self.solvers[level - 1]._need(rho)
        _check(_lib.hgs_nest_source(rho.data_ptr(), nx, ny, nz, self.ext, self._rho[level].data_ptr(), self._code,
                                    self.stream.cuda_stream))
        return self._rho[level]

    def fine_ghosts(self, phi_c, level: int = 0):
        """Ghost faces of `level` interpolated from the potential of level + 1."""
        inner, outer = self.solvers[level], self.solvers[level + 1]
        mz, my, mx = outer.shape
        nz, ny, nx = inner.shape
        outer._need(phi_c)
        _check(_lib.hgs_nest_ghosts(phi_c.data_ptr(), mx, my, mz, self._x0[level + 1], outer.cfg.dx, nx, ny, nz,
                                    self._x0[level], inner.cfg.dx, self._faces[level].data_ptr(), self._code,
                                    self.stream.cuda_stream))
        return self._faces[level]

    def step(self, rho, c_g: float, dt: float, nsub: int) -> None:
        nsub = int(nsub)
        srcs, counts = [rho], [nsub]
        for lev in range(1, len(self.solvers)):
            srcs.append(self.coarse_source(srcs[-1], lev))
            counts.append((counts[-1] + 1) // 2)
        for lev in range(len(self.solvers) - 1, -1, -1):
            s = self.solvers[lev]
            if lev < len(self.solvers) - 1:
                s.set_boundary(self.fine_ghosts(self.solvers[lev + 1].potential(with_phidot=False)[0], lev))
            s.step(srcs[lev], c_g, dt if lev == 0 else nsub * float(dt) / counts[lev], counts[lev])

    def potential(self, with_phidot: bool = True):
        return self.fine.potential(with_phidot)

    def accel(self, out=None):
        return self.fine.accel(out)

    def close(self) -> None:
        for s in self.solvers:
            s.close()


def tile_count(tblock: int) -> int:
    """Tile shapes compiled for fused depth tblock."""
    return int(_lib.hgs_tile_count(int(tblock)))


def tile_shape(storage: str, tblock: int, tile: int):
    """(rows per thread, waves per workgroup, input planes in flight) of a tile."""
    sh = (_i32 * 3)()
    _check(_lib.hgs_tile_shape(HGS_F64 if storage == "f64" else HGS_F32, int(tblock), int(tile), sh))
    return tuple(int(v) for v in sh)


def autotune(shape, rho, c_g: float, dt: float, nsub: int, storage: str = "f32", lmax: int = 4,
             x0=(-1.0, -1.0, -1.0), dx=None, eta: float = 0.0, bc: str = "multipole", device="cuda", stream=None):
    """Fastest fused depth and tile shape for hydro steps of nsub substeps on
    this grid (the library times every depth and every tile compiled for it
    on a temporary workspace).  Returns (best_tblock, best_tile, [best ms per
    substep for depth 1..TMAX] or None when cached)."""
    import torch

    dev = torch.device(device)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    cfg = make_config(shape, x0, dx, 1.0, (0.0, 0.0, 0.0), lmax, bc, storage, 0, eta, st.cuda_stream)
    nb = workspace_bytes(cfg)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    best = _i32(0)
    tile = _i32(0)
    ms = (ctypes.c_double * TMAX)()
    _check(_lib.hgs_autotune(ctypes.byref(cfg), rho.data_ptr(), float(c_g), float(dt), int(nsub), ws.data_ptr(), nb,
                             ctypes.byref(best), ctypes.byref(tile), ms))
    times = list(ms)
    return int(best.value), int(tile.value), (None if times[0] < 0 else times)


class Batch:
    """Independent cube or box grids stepped together (one launch per fused
    substep group covering all grids, replayed from a captured hipGraph)."""

    def __init__(self, shapes, dxs=None, x0s=None, G: float = 1.0, lmax: int = 4, storage: str = "f32",
                 tblock: int = 0, eta=0.0, bc: str = "multipole", device="cuda", stream=None):
        import torch

        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.dtype = torch.float32 if storage == "f32" else torch.float64
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        n = len(shapes)
        self.n = n
        etas = list(eta) if not np.isscalar(eta) else [eta] * n
        self.cfgs = (Config * n)()
        for i, sh in enumerate(shapes):
            nz, ny, nx = (sh, sh, sh) if np.isscalar(sh) else sh
            dx = dxs[i] if dxs is not None else 2.0 / nx
            x0 = x0s[i] if x0s is not None else (-0.5 * nx * dx, -0.5 * ny * dx, -0.5 * nz * dx)
            self.cfgs[i] = make_config((nz, ny, nx), x0, dx, G, (0.0, 0.0, 0.0), lmax, bc, storage,
                                       tblock, etas[i], self.stream.cuda_stream)
        nb = _sz(0)
        _check(_lib.hgs_workspace_bytes_batch(self.cfgs, n, ctypes.byref(nb)))
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        h = _vp()
        _check(_lib.hgs_init_batch(self.cfgs, n, self.workspace.data_ptr(), nb.value, ctypes.byref(h)))
        self._h = h
        self.grids = []
        for i in range(n):
            c = _vp()
            _check(_lib.hgs_batch_grid(self._h, i, ctypes.byref(c)))
            self.grids.append(Solver._view(c, self.cfgs[i], dev, self.dtype, self.stream, self))

    def step(self, rhos, c_g, dt, nsub: int) -> None:
        n = self.n
        for g, r in zip(self.grids, rhos):
            g._need(r)
        ptrs = (_vp * n)(*[r.data_ptr() for r in rhos])
        cg = (ctypes.c_double * n)(*([float(c_g)] * n if np.isscalar(c_g) else [float(v) for v in c_g]))
        dts = (ctypes.c_double * n)(*([float(dt)] * n if np.isscalar(dt) else [float(v) for v in dt]))
        st = _lib.hgs_step_batch(self._h, ptrs, cg, dts, int(nsub))
        if st != HGS_OK:
            raise HGSError(st, _lib.hgs_batch_last_error(self._h).decode())

    @property
    def used_graph(self) -> bool:
        return bool(_lib.hgs_batch_used_graph(self._h))

    LAUNCHES = {"per_item": 0, "persistent": 1}

    def set_launch(self, launch: str) -> None:
        """Fused launches with one workgroup per work item ("per_item", the
        default) or one persistent workgroup per CU ("persistent")."""
        st = _lib.hgs_batch_set_launch(self._h, self.LAUNCHES[launch])
        if st != HGS_OK:
            raise HGSError(st, _lib.hgs_batch_last_error(self._h).decode())

    @property
    def launch(self) -> str:
        v = int(_lib.hgs_batch_get_launch(self._h))
        return {0: "per_item", 1: "persistent"}.get(v, "?")

    def close(self) -> None:
        if getattr(self, "_h", None):
            for g in self.grids:
                g._h = None
            _lib.hgs_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def faces_to_flat(face_list: Sequence) -> np.ndarray:
    """Concatenate six face arrays (x-, x+, y-, y+, z-, z+) into the flat ghost layout."""
    return np.concatenate([np.asarray(f).ravel() for f in face_list])


def flat_to_faces(flat, shape):
    nz, ny, nx = shape
    sizes = [nz * ny, nz * ny, nz * nx, nz * nx, ny * nx, ny * nx]
    shapes = [(nz, ny), (nz, ny), (nz, nx), (nz, nx), (ny, nx), (ny, nx)]
    out, o = [], 0
    for s, sh in zip(sizes, shapes):
        out.append(np.asarray(flat[o:o + s]).reshape(sh))
        o += s
    return out


# ---------------------------------------------------------------------------
# Network kernels of the learned warm start (channels-last, 16 channels,
# torch.bfloat16 tensors carry the bfloat16 bit patterns)
NN_F32, NN_TANH_BF16, NN_DTANH_BF16, NN_BF16 = 0, 1, 2, 3
NN_CHANNELS = 16
NN_MSE_PARTIALS = 1024


def _nn_check(st):
    if st != HGS_OK:
        raise HGSError(st, _lib.hgs_nn_last_error().decode())


def _stream_of(t):
    import torch

    return torch.cuda.current_stream(t.device).cuda_stream


def nn_conv3d(inp, w, bias, out, mode: int, aux=None):
    """inp: (B,Z,Y,X,16) bf16; w: (27,16,16) bf16; bias: (16,) fp32 or None;
    out: (B,Z,Y,X,16) fp32 (mode 0) or bf16."""
    B, Z, Y, X, C = inp.shape
    assert C == NN_CHANNELS and inp.is_contiguous() and out.is_contiguous() and w.is_contiguous()
    _nn_check(_lib.hgs_nn_conv3d(inp.data_ptr(), w.data_ptr(), _ptr(bias), B, Z, Y, X, int(mode), _ptr(aux),
                                 out.data_ptr(), _stream_of(inp)))
    return out


def nn_flip_weights(w, wt):
    _nn_check(_lib.hgs_nn_flip_weights(w.data_ptr(), wt.data_ptr(), _stream_of(w)))
    return wt


def nn_wgrad(a, g, dw, db, workspace=None):
    import torch

    B, Z, Y, X, C = a.shape
    nb = _sz(0)
    _nn_check(_lib.hgs_nn_wgrad_workspace_bytes(B, Z, Y, X, ctypes.byref(nb)))
    if workspace is None or workspace.numel() < nb.value:
        workspace = torch.empty(nb.value, dtype=torch.uint8, device=a.device)
    _nn_check(_lib.hgs_nn_wgrad(a.data_ptr(), g.data_ptr(), B, Z, Y, X, dw.data_ptr(), db.data_ptr(),
                                workspace.data_ptr(), workspace.numel(), _stream_of(a)))
    return workspace


def nn_pack(fields, out):
    """fields: (B, C, *spatial) fp32 -> out (B, *spatial, 16) bf16."""
    B, C = fields.shape[:2]
    nvox = fields[0, 0].numel()
    _nn_check(_lib.hgs_nn_pack(fields.data_ptr(), B, C, nvox, out.data_ptr(), _stream_of(fields)))
    return out


def nn_unpack(inp, C, fields):
    B = inp.shape[0]
    nvox = inp[0].numel() // NN_CHANNELS
    _nn_check(_lib.hgs_nn_unpack(inp.data_ptr(), B, C, nvox, fields.data_ptr(), _stream_of(inp)))
    return fields


def nn_mse(out, target, grad, loss_dev, partials):
    B, C = target.shape[:2]
    nvox = target[0, 0].numel()
    _nn_check(_lib.hgs_nn_mse(out.data_ptr(), target.data_ptr(), B, C, nvox, grad.data_ptr(), loss_dev.data_ptr(),
                              partials.data_ptr(), _stream_of(out)))


def nn_lapmse(out, target, grad, loss_dev, partials, scratch, ch: int = 0, w: float = 1.0):
    """target: planar (B, C, Z, Y, X) fp32; out: channels-last (B, Z, Y, X, 16)
    fp32; scratch: fp32 with B*Z*Y*X elements."""
    B, C, Z, Y, X = target.shape
    assert scratch.numel() >= B * Z * Y * X
    _nn_check(_lib.hgs_nn_lapmse(out.data_ptr(), target.data_ptr(), B, C, Z, Y, X, int(ch), float(w),
                                 scratch.data_ptr(), grad.data_ptr(), loss_dev.data_ptr(), partials.data_ptr(),
                                 _stream_of(out)))


NN_MAXABS_CHUNKS = 64


def nn_maxabs(x, out, scratch=None):
    """x: (B, ...) fp32; out: (B,) fp32 receives the per-sample max |x|;
    scratch: fp32 with B * NN_MAXABS_CHUNKS elements (allocated if None)."""
    import torch

    B = x.shape[0]
    assert out.numel() == B and x.is_contiguous()
    if scratch is None:
        scratch = torch.empty(B * NN_MAXABS_CHUNKS, dtype=torch.float32, device=x.device)
    assert scratch.numel() >= B * NN_MAXABS_CHUNKS
    _nn_check(_lib.hgs_nn_maxabs(x.data_ptr(), B, x[0].numel(), out.data_ptr(), scratch.data_ptr(),
                                 _stream_of(x)))


NN_MAXABS_NOALLOC_MAX_B = 4096


def nn_maxabs_noalloc(x, out):
    """nn_maxabs without a scratch buffer: the library's static per-device
    partials (B <= NN_MAXABS_NOALLOC_MAX_B); allocates nothing."""
    B = x.shape[0]
    assert out.numel() == B and x.is_contiguous()
    _nn_check(_lib.hgs_nn_maxabs_noalloc(x.data_ptr(), B, x[0].numel(), out.data_ptr(), _stream_of(x)))


def nn_features(rho, phi, scale, c: float, out):
    """rho, phi: (B, Z, Y, X) fp32; scale: (B,) fp32; out: (B, 3, Z, Y, X) fp32."""
    B, Z, Y, X = rho.shape
    assert tuple(phi.shape) == tuple(rho.shape) and tuple(out.shape) == (B, 3, Z, Y, X) and scale.numel() == B
    _nn_check(_lib.hgs_nn_features(rho.data_ptr(), phi.data_ptr(), scale.data_ptr(), B, Z, Y, X, float(c),
                                   out.data_ptr(), _stream_of(rho)))


def nn_compose(phi_c, y, scale, out_scale: float, phi, phidot=None):
    """phi_c, phi, phidot: (B, Z, Y, X) fp32; y: (B, Z, Y, X, 16) fp32."""
    B = phi_c.shape[0]
    nvox = phi_c[0].numel()
    assert y.numel() == B * nvox * NN_CHANNELS and phi.shape == phi_c.shape and scale.numel() == B
    _nn_check(_lib.hgs_nn_compose(phi_c.data_ptr(), y.data_ptr(), scale.data_ptr(), B, nvox,
                                  float(1.0 / out_scale), phi.data_ptr(), _ptr(phidot), _stream_of(phi_c)))


def nn_adam(p, m, v, g, p16, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    _nn_check(_lib.hgs_nn_adam(p.data_ptr(), m.data_ptr(), v.data_ptr(), g.data_ptr(), _ptr(p16), p.numel(),
                               float(lr), float(b1), float(b2), float(eps), int(t), _stream_of(p)))


def nn_restrict2(fine, coarse):
    """fine (B, 2cz, 2cy, 2cx) -> coarse (B, cz, cy, cx); fp32 or fp64."""
    import torch

    B, cz, cy, cx = coarse.shape
    dt = HGS_F32 if coarse.dtype == torch.float32 else HGS_F64
    _nn_check(_lib.hgs_nn_restrict2(fine.data_ptr(), coarse.data_ptr(), B, cz, cy, cx, dt, _stream_of(fine)))
    return coarse


def nn_prolong2(coarse, fine):
    import torch

    B, cz, cy, cx = coarse.shape
    dt = HGS_F32 if coarse.dtype == torch.float32 else HGS_F64
    _nn_check(_lib.hgs_nn_prolong2(coarse.data_ptr(), fine.data_ptr(), B, cz, cy, cx, dt, _stream_of(coarse)))
    return fine
