"""The C-ABI library loads, exports every declared symbol, and validates on the
host (no GPU needed: every case here returns before any device work)."""
import ctypes
import os
import re

import pytest

from paper_1602_05700_amd import hgs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "hgs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hgs_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(hgs.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    assert set(declared_functions()) <= set(hgs._SIGS)


def test_abi_version_and_status_strings():
    L = hgs.library()
    assert L.hgs_abi_version() == 2
    assert L.hgs_status_str(hgs.HGS_ERR_CFL) == b"HGS_ERR_CFL"
    assert L.hgs_status_str(99) == b"HGS_ERR_UNKNOWN"


def test_config_cube_defaults():
    L = hgs.library()
    c = hgs.Config()
    assert L.hgs_config_cube(ctypes.byref(c), 64, -1.0, 1.0) == hgs.HGS_OK
    assert (c.nx, c.ny, c.nz, c.lmax, c.storage, c.bc) == (64, 64, 64, 4, hgs.HGS_F32, hgs.HGS_BC_MULTIPOLE)
    assert c.dx == pytest.approx(2.0 / 64)
    assert L.hgs_config_cube(ctypes.byref(c), 0, -1.0, 1.0) == hgs.HGS_ERR_ARG
    assert L.hgs_config_cube(ctypes.byref(c), 8, 1.0, 1.0) == hgs.HGS_ERR_ARG


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("ny", -3), ("nz", 9000), ("dx", 0.0), ("dx", float("nan")), ("lmax", 5), ("lmax", -1),
    ("bc", 5), ("bc", -1), ("storage", 7), ("tblock", 5), ("tblock", -1), ("eta", -0.5), ("eta", float("inf")),
    ("G", float("nan")),
])
def test_bad_config_rejected(field, value):
    c = hgs.make_config(16)
    setattr(c, field, value)
    n = ctypes.c_size_t(0)
    L = hgs.library()
    assert L.hgs_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == hgs.HGS_ERR_ARG
    assert L.hgs_last_error(None) != b""
    h = ctypes.c_void_p()
    assert L.hgs_init(ctypes.byref(c), 256, 1 << 30, ctypes.byref(h)) == hgs.HGS_ERR_ARG
    assert h.value is None


def test_too_large_grid_rejected():
    c = hgs.make_config((4096, 4096, 4096))
    with pytest.raises(hgs.HGSError):
        hgs.workspace_bytes(c)


def test_workspace_size_and_checks():
    L = hgs.library()
    c = hgs.make_config((23, 29, 37), storage="f64")
    nb = hgs.workspace_bytes(c)
    # four padded state buffers at least
    assert nb >= 4 * (37 + 2) * (29 + 2) * (23 + 2) * 8
    h = ctypes.c_void_p()
    assert L.hgs_init(ctypes.byref(c), None, nb, ctypes.byref(h)) == hgs.HGS_ERR_WORKSPACE
    assert L.hgs_init(ctypes.byref(c), 4096, nb - 1, ctypes.byref(h)) == hgs.HGS_ERR_WORKSPACE
    assert L.hgs_init(ctypes.byref(c), 4096 + 8, nb, ctypes.byref(h)) == hgs.HGS_ERR_WORKSPACE
    assert b"aligned" in L.hgs_last_error(None)
    assert L.hgs_init(ctypes.byref(c), 4096, nb, None) == hgs.HGS_ERR_ARG
    f32 = hgs.workspace_bytes(hgs.make_config((23, 29, 37), storage="f32"))
    assert f32 < nb


def test_step_validation_host_only():
    L = hgs.library()
    c = hgs.make_config(32)
    dx = c.dx
    v = lambda rho, cg, dt, n: L.hgs_validate_step(ctypes.byref(c), rho, cg, dt, n)
    assert v(1, 1.0, 0.4 * dx, 4) == hgs.HGS_OK
    assert v(1, 1.0, dx / 3 ** 0.5, 4) == hgs.HGS_OK  # exactly at the limit
    assert v(1, 1.0, 0.58 * dx, 4) == hgs.HGS_ERR_CFL
    assert b"1/sqrt(3)" in L.hgs_last_error(None)
    assert v(1, 2.0, 0.3 * dx, 4) == hgs.HGS_ERR_CFL  # c_g enters the Courant number
    assert v(None, 1.0, 0.4 * dx, 4) == hgs.HGS_ERR_ARG
    assert v(1, 1.0, 0.4 * dx, 0) == hgs.HGS_ERR_ARG
    assert v(1, 1.0, -0.1, 4) == hgs.HGS_ERR_ARG
    assert v(1, 1.0, float("nan"), 4) == hgs.HGS_ERR_ARG
    assert v(1, 0.0, 0.1, 4) == hgs.HGS_ERR_ARG
    assert v(1, float("inf"), 0.1, 4) == hgs.HGS_ERR_ARG


def test_null_context_calls():
    L = hgs.library()
    assert L.hgs_destroy(None) == hgs.HGS_OK
    for f, args in [("hgs_step", (None, 1, 1.0, 0.01, 1)), ("hgs_potential", (None, 1, None)),
                    ("hgs_accel", (None, 1, 1, 1)), ("hgs_set_state", (None, 1, None, 0.1)),
                    ("hgs_set_boundary", (None, 1)), ("hgs_get_boundary", (None, 1)),
                    ("hgs_residual", (None, 1, (ctypes.c_double * 4)())),
                    ("hgs_moments", (None, (ctypes.c_double * 50)())),
                    ("hgs_set_tblock", (None, 2))]:
        assert getattr(L, f)(*args) == hgs.HGS_ERR_ARG, f
    assert L.hgs_get_tblock(None) == 0


def test_face_helpers_roundtrip():
    import numpy as np

    shape = (3, 4, 5)
    flat = np.arange(2 * (3 * 4 + 3 * 5 + 4 * 5), dtype=float)
    faces = hgs.flat_to_faces(flat, shape)
    assert [f.shape for f in faces] == [(3, 4), (3, 4), (3, 5), (3, 5), (4, 5), (4, 5)]
    assert np.array_equal(hgs.faces_to_flat(faces), flat)


def test_multipole_centre_must_be_inside():
    L = hgs.library()
    n = ctypes.c_size_t(0)
    c = hgs.make_config((3, 2, 5))  # y spans [-1, -0.2]: the centre (0,0,0) is outside
    assert L.hgs_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == hgs.HGS_ERR_ARG
    assert b"centre" in L.hgs_last_error(None)
    c = hgs.make_config((3, 2, 5), bc="user")  # no expansion: any placement
    assert L.hgs_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == hgs.HGS_OK
    c = hgs.make_config(8, origin=(0.9, 0.0, 0.0))
    assert L.hgs_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == hgs.HGS_OK
    c = hgs.make_config(8, origin=(1.0, 0.0, 0.0))  # on the face: a ghost could sit at r = 0
    assert L.hgs_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == hgs.HGS_ERR_ARG


def test_local_boundaries_host_checks():
    L = hgs.library()
    n = ctypes.c_size_t(0)
    for bc in ("robin", "outgoing"):  # r-weighted rules need the centre inside
        c = hgs.make_config((3, 2, 5), bc=bc)
        assert L.hgs_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == hgs.HGS_ERR_ARG
        c = hgs.make_config(8, bc=bc)
        assert L.hgs_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == hgs.HGS_OK
    c = hgs.make_config((3, 2, 5), bc="periodic")  # no centre involved
    assert L.hgs_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == hgs.HGS_OK
    # batches need a boundary frozen over the step
    cfgs = (hgs.Config * 2)(hgs.make_config(16), hgs.make_config(16, bc="robin"))
    assert L.hgs_workspace_bytes_batch(cfgs, 2, ctypes.byref(n)) == hgs.HGS_ERR_ARG
    assert b"frozen" in L.hgs_last_error(None)


def test_embed_extract_host_checks():
    L = hgs.library()
    a = ctypes.c_void_p(16)  # never dereferenced: every case below fails validation first
    assert L.hgs_embed(None, 4, 4, 4, 2, a, hgs.HGS_F32, None) == hgs.HGS_ERR_ARG
    assert L.hgs_embed(a, 4, 4, 4, -1, a, hgs.HGS_F32, None) == hgs.HGS_ERR_ARG
    assert L.hgs_embed(a, 4, 0, 4, 1, a, hgs.HGS_F32, None) == hgs.HGS_ERR_ARG
    assert L.hgs_embed(a, 4, 4, 4, 1, a, 9, None) == hgs.HGS_ERR_ARG
    assert L.hgs_extract(a, 8000, 4, 4, 200, a, hgs.HGS_F64, None) == hgs.HGS_ERR_ARG
    assert L.hgs_extract(a, 4, 4, 4, 1, None, hgs.HGS_F64, None) == hgs.HGS_ERR_ARG
    assert L.hgs_accel_box(None, 0, 0, 0, 1, 1, 1, a, a, a) == hgs.HGS_ERR_ARG


def test_nest_host_checks():
    L = hgs.library()
    a = ctypes.c_void_p(16)  # never dereferenced: every case below fails validation first
    assert L.hgs_nest_source(None, 8, 8, 8, 2, a, hgs.HGS_F32, None) == hgs.HGS_ERR_ARG
    assert L.hgs_nest_source(a, 8, 7, 8, 2, a, hgs.HGS_F32, None) == hgs.HGS_ERR_ARG  # odd size
    assert L.hgs_nest_source(a, 8, 8, 8, -1, a, hgs.HGS_F32, None) == hgs.HGS_ERR_ARG
    assert L.hgs_nest_source(a, 8, 8, 8, 2, a, 5, None) == hgs.HGS_ERR_ARG
    c0 = (ctypes.c_double * 3)(-1.5, -1.5, -1.5)  # coarse 6^3 at 0.5 around a fine 4^3 at 0.25
    f0 = (ctypes.c_double * 3)(-0.5, -0.5, -0.5)
    assert L.hgs_nest_ghosts(None, 6, 6, 6, c0, 0.5, 4, 4, 4, f0, 0.25, a, hgs.HGS_F64, None) == hgs.HGS_ERR_ARG
    assert L.hgs_nest_ghosts(a, 1, 6, 6, c0, 0.5, 4, 4, 4, f0, 0.25, a, hgs.HGS_F64, None) == hgs.HGS_ERR_ARG
    assert L.hgs_nest_ghosts(a, 6, 6, 6, c0, 0.0, 4, 4, 4, f0, 0.25, a, hgs.HGS_F64, None) == hgs.HGS_ERR_ARG
    far = (ctypes.c_double * 3)(-0.5, -0.5, 0.6)  # ghost centres beyond the last coarse centre along z
    assert L.hgs_nest_ghosts(a, 6, 6, 6, c0, 0.5, 4, 4, 4, far, 0.25, a, hgs.HGS_F64, None) == hgs.HGS_ERR_ARG
    assert b"span" in L.hgs_last_error(None)


def test_warmstart_criterion_checks():
    """Convergence criteria are checked before any solver is built."""
    from paper_1602_05700_amd import warmstart as ws

    with pytest.raises(ValueError):
        ws.steps_to_tolerance(None, 16, 1e-4, metric="R_x")
    with pytest.raises(ValueError):
        ws.steps_to_tolerance(None, 16, 1e-4, metric="E")  # E needs the converged reference


def test_no_fallback_without_the_library(tmp_path):
    """Without libhgs.so the binding refuses to import: there is no CPU path."""
    import subprocess
    import sys

    env = dict(os.environ, HGS_LIBRARY=str(tmp_path / "absent" / "libhgs.so"))
    r = subprocess.run([sys.executable, "-c", "import paper_1602_05700_amd.hgs"], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "libhgs.so" in r.stderr


def test_noalloc_maxabs_validates_on_the_host():
    """The allocation-free maxabs refuses NULL pointers and sample counts
    beyond its static scratch before touching a device."""
    L = hgs.library()
    dummy = ctypes.c_void_p(1 << 20)
    assert L.hgs_nn_maxabs_noalloc(None, 1, 4, dummy, None) == hgs.HGS_ERR_ARG
    assert L.hgs_nn_maxabs_noalloc(dummy, hgs.NN_MAXABS_NOALLOC_MAX_B + 1, 4, dummy, None) == hgs.HGS_ERR_ARG
    assert b"static scratch" in L.hgs_nn_last_error()
    assert L.hgs_nn_maxabs_noalloc(dummy, 0, 4, dummy, None) == hgs.HGS_ERR_ARG
    assert L.hgs_nn_maxabs_noalloc(dummy, 1, 0, dummy, None) == hgs.HGS_ERR_ARG
