"""CPU checks of the C ABI: the library loads, exports every declared symbol and
rejects invalid arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_2203_00879_amd import nopcs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "nopcs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = nopcs.lib()
    names = declared_symbols()
    assert "nopcs_derivative" in names and "rk_step" in names and "nse_rhs" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_error_string():
    lib = nopcs.lib()
    assert lib.nopcs_version() >= 100
    assert isinstance(nopcs.last_error(), str)


@pytest.mark.parametrize("n,nseg", [((7, 16, 16), 1), ((16, 16, 2000), 1), ((16, 16, 16), 5), ((16, 16, 16), 0)])
def test_invalid_grid_rejected(n, nseg):
    g = nopcs.make_grid(n, nseg)
    assert nopcs.workspace_bytes(g) == 0
    rc = nopcs.lib().nopcs_derivative(ctypes.byref(g), 0, 0, ctypes.c_void_p(8), ctypes.c_void_p(8), None, None)
    assert rc == nopcs.NOPCS_EINVAL
    assert nopcs.last_error()


def test_invalid_arguments_rejected():
    lib = nopcs.lib()
    g = nopcs.make_grid(16)
    assert lib.nopcs_derivative(ctypes.byref(g), 3, 0, ctypes.c_void_p(8), ctypes.c_void_p(8), None, None) == -1
    assert lib.nopcs_derivative(ctypes.byref(g), 0, 0, None, ctypes.c_void_p(8), None, None) == -1
    assert lib.nopcs_derivative(ctypes.byref(g), 0, 0, ctypes.c_void_p(8), None, None, None) == -1
    assert lib.nopcs_derivative(ctypes.byref(g), 0, 7, ctypes.c_void_p(8), ctypes.c_void_p(8), None, None) == -1
    from paper_2203_00879_amd import inputs
    p = nopcs.make_params(inputs.AIR)
    ws = nopcs.workspace_bytes(g)
    assert ws == 3 * 5 * 16 ** 3 * 8
    # dt <= 0, too small workspace, NULL state
    assert lib.rk_step(ctypes.byref(p), ctypes.byref(g), 0, ctypes.c_void_p(256), 0.0, 1, ctypes.c_void_p(256), ws,
                       None) == -1
    assert lib.rk_step(ctypes.byref(p), ctypes.byref(g), 0, ctypes.c_void_p(256), 1e-5, 1, ctypes.c_void_p(256),
                       ws - 8, None) == -1
    assert lib.rk_step(ctypes.byref(p), ctypes.byref(g), 0, None, 1e-5, 1, ctypes.c_void_p(256), ws, None) == -1
    # misaligned state (the RK register update moves 16 bytes at a time)
    assert lib.rk_step(ctypes.byref(p), ctypes.byref(g), 0, ctypes.c_void_p(264), 1e-5, 1, ctypes.c_void_p(256), ws,
                       None) == -1
    assert b"aligned" in lib.nopcs_last_error()
    bad = dict(inputs.AIR, gamma=0.9)
    pb = nopcs.make_params(bad)
    assert lib.nse_rhs(ctypes.byref(pb), ctypes.byref(g), 0, ctypes.c_void_p(8), ctypes.c_void_p(16), None, 0,
                       None) == -1
    # the right-hand side needs the workspace too (closure array of the line-march sweeps)
    assert lib.nse_rhs(ctypes.byref(p), ctypes.byref(g), 0, ctypes.c_void_p(256), ctypes.c_void_p(512), None, 0,
                       None) == -1
    assert b"workspace" in lib.nopcs_last_error()


def test_workspace_includes_closure_array():
    """Three 5-field states plus, for y and z, 5 components x closure rows x lines
    (the larger of the two), 256-byte aligned; mixed precision adds a second FP64
    stage register (the z sweep that carries the RK4 update writes the next stage
    state there)."""
    g = nopcs.make_grid((16, 16, 16), nseg=(1, 2, 3))
    # y: 2 segments -> closure rows 7, 8; z: 3 segments of 6, 5, 5 -> rows 5, 6, 10, 11
    clo = max(5 * 2 * 16 * 16, 5 * 4 * 16 * 16) * 8
    assert nopcs.workspace_bytes(g) == 3 * 5 * 16 ** 3 * 8 + (clo + 255) // 256 * 256
    assert nopcs.workspace_bytes(g, nopcs.MIXED) == 4 * 5 * 16 ** 3 * 8 + (clo + 255) // 256 * 256


def test_vorticity_workspace_and_argument_checks():
    """19 fields padded to 32 doubles; NULL arrays, a short or misaligned
    workspace and bad parameters are rejected before any device work."""
    from paper_2203_00879_amd import inputs
    lib = nopcs.lib()
    g = nopcs.make_grid((9, 10, 11))
    S = (9 * 10 * 11 + 31) // 32 * 32
    ws = nopcs.vorticity_workspace_bytes(g)
    assert ws == 19 * S * 8
    assert nopcs.vorticity_workspace_bytes(nopcs.make_grid(4)) == 0
    p = nopcs.make_params(inputs.AIR)
    V = ctypes.c_void_p
    call = lib.nopcs_vorticity_budget
    assert call(ctypes.byref(p), ctypes.byref(g), None, V(256), V(4096), ws, None) == -1
    assert call(ctypes.byref(p), ctypes.byref(g), V(256), None, V(4096), ws, None) == -1
    assert call(ctypes.byref(p), ctypes.byref(g), V(256), V(512), V(4096), ws - 8, None) == -1
    assert b"workspace" in lib.nopcs_last_error()
    assert call(ctypes.byref(p), ctypes.byref(g), V(256), V(512), V(4104), ws, None) == -1
    assert b"aligned" in lib.nopcs_last_error()
    pb = nopcs.make_params(dict(inputs.AIR, gamma=1.0))
    assert call(ctypes.byref(pb), ctypes.byref(g), V(256), V(512), V(4096), ws, None) == -1


def test_disturbance_pressure_and_spectrum_argument_checks():
    from paper_2203_00879_amd import inputs
    lib = nopcs.lib()
    g = nopcs.make_grid(16)
    p = nopcs.make_params(inputs.AIR)
    V = ctypes.c_void_p
    assert lib.nopcs_disturbance_pressure(ctypes.byref(p), ctypes.byref(g), V(256), None, V(512), None) == -1
    assert lib.nopcs_disturbance_pressure(ctypes.byref(p), ctypes.byref(nopcs.make_grid(4)), V(256), V(512), V(768),
                                          None) == -1
    assert lib.nopcs_line_spectrum(V(256), 1, 1, V(512), None) == -1
    assert lib.nopcs_line_spectrum(V(256), 16385, 1, V(512), None) == -1
    assert lib.nopcs_line_spectrum(V(256), 64, 0, V(512), None) == -1
    assert lib.nopcs_line_spectrum(None, 64, 1, V(512), None) == -1
    assert b"NULL" in lib.nopcs_last_error()


def test_compact_viscous_workspace_and_argument_checks():
    from paper_2203_00879_amd import inputs
    lib = nopcs.lib()
    g = nopcs.make_grid((9, 10, 11))
    S = (9 * 10 * 11 + 31) // 32 * 32
    ws = nopcs.compact_viscous_workspace_bytes(g)
    assert ws == nopcs.workspace_bytes(g) + 28 * S * 8
    assert nopcs.compact_viscous_workspace_bytes(nopcs.make_grid(4)) == 0
    p = nopcs.make_params(inputs.AIR)
    V = ctypes.c_void_p
    call = lib.nse_rhs_compact_viscous
    assert call(ctypes.byref(p), ctypes.byref(g), None, V(512), V(4096), ws, None) == -1
    assert call(ctypes.byref(p), ctypes.byref(g), V(256), V(512), V(4096), ws - 8, None) == -1
    assert b"workspace" in lib.nopcs_last_error()
    assert call(ctypes.byref(p), ctypes.byref(g), V(256), V(512), V(4104), ws, None) == -1
    assert b"aligned" in lib.nopcs_last_error()


def test_batch_argument_checks():
    """rk_step_batch rejects a bad batch before any device work."""
    from paper_2203_00879_amd import inputs
    lib = nopcs.lib()
    p = nopcs.make_params(inputs.AIR)
    g = nopcs.make_grid(16)
    ws = nopcs.workspace_bytes(g)
    arr = (nopcs.Box * 2)()
    for i in range(2):
        arr[i].grid = g
        arr[i].Q = 256 * (i + 1)
        arr[i].ws = 4096 * (i + 1)
        arr[i].ws_bytes = ws
    call = lib.rk_step_batch
    assert call(ctypes.byref(p), 0, arr, 0, 1e-5, 1, None) == -1
    assert call(ctypes.byref(p), nopcs.MAX_BATCH + 1, arr, 0, 1e-5, 1, None) == -1
    assert call(ctypes.byref(p), 2, None, 0, 1e-5, 1, None) == -1
    assert call(ctypes.byref(p), 2, arr, 7, 1e-5, 1, None) == -1
    assert call(ctypes.byref(p), 2, arr, 0, -1.0, 1, None) == -1
    arr[1].Q = 256                                   # same state twice
    assert call(ctypes.byref(p), 2, arr, 0, 1e-5, 1, None) == -1
    assert b"share" in lib.nopcs_last_error()
    arr[1].Q = 520                                   # misaligned state
    assert call(ctypes.byref(p), 2, arr, 0, 1e-5, 1, None) == -1
    arr[1].Q = 512
    arr[1].ws_bytes = ws - 8                         # short workspace
    assert call(ctypes.byref(p), 2, arr, 0, 1e-5, 1, None) == -1
    assert b"workspace" in lib.nopcs_last_error()


def test_visc_chunk_setting():
    """The viscous kernel's z chunk: 0 (default: 64 planes, halved down to 16
    while the box has fewer than 1024 blocks) or 8..1024 planes, capped at nz;
    other values rejected (host only)."""
    lib = nopcs.lib()
    try:
        assert nopcs.visc_chunk(nopcs.make_grid(48)) == 16
        assert nopcs.visc_chunk(nopcs.make_grid(192, 3)) == 16    # 112 tiles: 64 planes would give 336 blocks
        assert nopcs.visc_chunk(nopcs.make_grid(256, 4)) == 32    # 220 tiles
        assert nopcs.visc_chunk(nopcs.make_grid(512, 4)) == 64
        for bad in (-1, 1, 7, 1025):
            assert lib.nopcs_set_visc_chunk(bad) == nopcs.NOPCS_EINVAL
        nopcs.set_visc_chunk(32)
        assert nopcs.visc_chunk(nopcs.make_grid(512, 4)) == 32
        assert nopcs.visc_chunk(nopcs.make_grid((16, 16, 20))) == 20
    finally:
        nopcs.set_visc_chunk(0)


def test_deriv_form_setting():
    """The form of the first derivative alone along y and z: 0 (by size), 1
    (pencil) or 2 (line march); other values rejected (host only)."""
    lib = nopcs.lib()
    try:
        for bad in (-1, 3):
            assert lib.nopcs_set_deriv_form(bad) == nopcs.NOPCS_EINVAL
        for form in (nopcs.DERIV_PENCIL, nopcs.DERIV_MARCH, nopcs.DERIV_BY_SIZE):
            nopcs.set_deriv_form(form)
    finally:
        nopcs.set_deriv_form(nopcs.DERIV_BY_SIZE)
