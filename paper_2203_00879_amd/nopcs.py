"""Thin ctypes binding of libnopcs.so (declared in include/nopcs.h).

Argument marshalling only: every step of the path runs in the HIP library.
PyTorch provides device memory (tensor.data_ptr()) and streams
(torch.cuda.current_stream().cuda_stream).  There is no CPU fallback: if the
library cannot be loaded the import of the first call raises.
"""
import ctypes
import os

from . import build as _build

NOPCS_OK = 0
NOPCS_EINVAL = -1
NOPCS_ENOMEM = -2
NOPCS_EDEVICE = -3
NOPCS_EAGAIN = -4
NOPCS_ENOTFOUND = -5
NOPCS_ENONFINITE = -6
NOPCS_EBUSY = -7
FP64 = 0
MIXED = 1

_ERRNAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EAGAIN", -5: "ENOTFOUND",
             -6: "ENONFINITE", -7: "EBUSY"}


class NopcsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "?"), code, msg))
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("len", ctypes.c_double * 3), ("nseg", ctypes.c_int32 * 3)]


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("gamma", "R_gas", "g", "L", "T_s", "rho_s", "Pr", "mu_ref", "T_ref", "S_suth", "mub_a", "mub_b")] + \
               [("viscous", ctypes.c_int32), ("gravity", ctypes.c_int32)]


class Box(ctypes.Structure):
    _fields_ = [("grid", Grid), ("Q", ctypes.c_void_p), ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t),
                ("dt", ctypes.c_double)]


MAX_BATCH = 64


class SolverConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("max_queue", ctypes.c_int32), ("device", ctypes.c_int32), ("batched", ctypes.c_int32)]


class SolveRequest(ctypes.Structure):
    _fields_ = [("params", Params), ("grid", Grid), ("nsteps", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("dt", ctypes.c_double), ("Q0_host", ctypes.c_void_p)]


class SolveResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("steps_done", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


_lib = None
_V = ctypes.c_void_p
_I = ctypes.c_int


def library_path():
    return _build.LIB


def lib():
    """Load libnopcs.so (built in-tree; built once if missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.nopcs_last_error.restype = ctypes.c_char_p
        L.nopcs_version.restype = _I
        L.nopcs_release_plans.restype = _I
        L.nopcs_workspace_bytes.restype = ctypes.c_size_t
        L.nopcs_workspace_bytes.argtypes = [ctypes.POINTER(Grid), _I]
        L.nopcs_derivative.argtypes = [ctypes.POINTER(Grid), _I, _I, _V, _V, _V, _V]
        L.nse_rhs.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Grid), _I, _V, _V, _V, ctypes.c_size_t, _V]
        L.nse_rhs_noalloc.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Grid), _I, _V, _V, _V]
        L.nopcs_filter.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Grid), ctypes.c_double, _V, _V]
        L.rk_step_filtered.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Grid), _I, _V, ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_double, _V, ctypes.c_size_t, _V]
        L.rk_step.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Grid), _I, _V, ctypes.c_double, ctypes.c_int32,
                              _V, ctypes.c_size_t, _V]
        L.nopcs_set_graphs.argtypes = [ctypes.c_int32]
        L.nopcs_set_deriv_form.argtypes = [ctypes.c_int32]
        L.nopcs_set_graph_cache_limit.argtypes = [ctypes.c_int32]
        L.nopcs_autotune.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Grid), _I, _V, _V, ctypes.c_size_t, _V,
                                     ctypes.POINTER(ctypes.c_int32 * 3)]
        L.nopcs_set_piece_length.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.nopcs_set_visc_chunk.argtypes = [ctypes.c_int32]
        L.nopcs_visc_chunk.argtypes = [ctypes.POINTER(Grid)]
        L.nopcs_visc_chunk.restype = ctypes.c_int32
        L.nopcs_disturbance_pressure.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Grid), _V, _V, _V, _V]
        L.nopcs_line_spectrum.argtypes = [_V, ctypes.c_int32, ctypes.c_int64, _V, _V]
        L.nopcs_compact_viscous_workspace_bytes.restype = ctypes.c_size_t
        L.nopcs_compact_viscous_workspace_bytes.argtypes = [ctypes.POINTER(Grid)]
        L.nse_rhs_compact_viscous.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Grid), _V, _V, _V,
                                              ctypes.c_size_t, _V]
        L.rk_step_batch.argtypes = [ctypes.POINTER(Params), ctypes.c_int32, ctypes.POINTER(Box), _I, ctypes.c_double,
                                    ctypes.c_int32, _V]
        L.nopcs_set_batch_mode.argtypes = [ctypes.c_int32]
        L.rk_step_compact_viscous.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Grid), _V, ctypes.c_double,
                                              ctypes.c_int32, _V, ctypes.c_size_t, _V]
        L.nopcs_vorticity_workspace_bytes.restype = ctypes.c_size_t
        L.nopcs_vorticity_workspace_bytes.argtypes = [ctypes.POINTER(Grid)]
        L.nopcs_vorticity_budget.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Grid), _V, _V, _V, ctypes.c_size_t,
                                             _V]
        if hasattr(L, "solver_create"):
            L.solver_create.argtypes = [ctypes.POINTER(SolverConfig), ctypes.POINTER(_V)]
            L.solver_submit.argtypes = [_V, ctypes.POINTER(SolveRequest), ctypes.POINTER(ctypes.c_uint64)]
            L.solver_poll.argtypes = [_V, ctypes.c_uint64, _V, ctypes.POINTER(SolveResult)]
            L.solver_create.restype = _I
            L.solver_submit.restype = _I
            L.solver_poll.restype = _I
            L.solver_destroy.restype = _I
            L.solver_destroy.argtypes = [_V]
            L.solver_now.argtypes = [_V]
            L.solver_now.restype = ctypes.c_double
        _lib = L
    return _lib


def last_error():
    return lib().nopcs_last_error().decode()


def _check(rc):
    if rc != NOPCS_OK:
        raise NopcsError(rc, last_error())
    return rc


def make_grid(n, nseg=1, length=1.0):
    n3 = (n, n, n) if isinstance(n, int) else tuple(n)
    s3 = (nseg, nseg, nseg) if isinstance(nseg, int) else tuple(nseg)
    l3 = (length,) * 3 if isinstance(length, (int, float)) else tuple(length)
    g = Grid()
    for d in range(3):
        g.n[d] = int(n3[d])
        g.nseg[d] = int(s3[d])
        g.len[d] = float(l3[d])
    return g


def make_params(d):
    return Params(**{k: d[k] for k, _ in Params._fields_})


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def workspace_bytes(grid, precision=FP64):
    return lib().nopcs_workspace_bytes(ctypes.byref(grid), precision)


def nopcs_derivative(grid, direction, f, d1=None, d2=None, precision=FP64, stream=None):
    """D1 and/or D2 of a device field f (float64 tensor of n0*n1*n2 elements)."""
    _check(lib().nopcs_derivative(ctypes.byref(grid), int(direction), int(precision), _ptr(f), _ptr(d1), _ptr(d2),
                                  _stream(stream)))


DERIV_BY_SIZE, DERIV_PENCIL, DERIV_MARCH = 0, 1, 2


def set_deriv_form(form):
    """How the first derivative alone along y or z is computed: DERIV_BY_SIZE
    (default: the line march from 2^17 lines), DERIV_PENCIL or DERIV_MARCH."""
    _check(lib().nopcs_set_deriv_form(int(form)))


def vorticity_workspace_bytes(grid):
    return lib().nopcs_vorticity_workspace_bytes(ctypes.byref(grid))


def vorticity_budget(params, grid, Q, out, ws=None, stream=None):
    """out (12 fields) = omega, stretching, dilatation and baroclinic terms of
    Eq. eqn12_1 at Q.  ws: device workspace of vorticity_workspace_bytes(grid)
    bytes; allocated here when not given."""
    if ws is None:
        import torch
        nb = vorticity_workspace_bytes(grid)
        if nb == 0:
            raise NopcsError(NOPCS_EINVAL, last_error())
        ws = torch.empty(nb, dtype=torch.uint8, device=Q.device)
    _check(lib().nopcs_vorticity_budget(ctypes.byref(params), ctypes.byref(grid), _ptr(Q), _ptr(out), _ptr(ws),
                                        ws.numel() * ws.element_size(), _stream(stream)))


def disturbance_pressure(params, grid, Q, Q0, out, stream=None):
    """out = p(Q) - p(Q0) (Section 4's disturbance pressure for Q0 the initial box)."""
    _check(lib().nopcs_disturbance_pressure(ctypes.byref(params), ctypes.byref(grid), _ptr(Q), _ptr(Q0), _ptr(out),
                                            _stream(stream)))


def line_spectrum(f, n, stride, amp, stream=None):
    """amp[k] = |DFT_k of f[j*stride], j < n| / n for k <= n // 2 (device tensors;
    f may be a view whose data_ptr() is the line's first sample)."""
    _check(lib().nopcs_line_spectrum(_ptr(f), int(n), int(stride), _ptr(amp), _stream(stream)))


def nse_rhs(params, grid, Q, R, precision=FP64, ws=None, stream=None):
    """R = right-hand side of ge17 at Q.  ws: device workspace of
    workspace_bytes(grid, precision) bytes; allocated here when not given."""
    if ws is None:
        ws = alloc_workspace(grid, precision, device=Q.device)
    nbytes = ws.numel() * ws.element_size()
    _check(lib().nse_rhs(ctypes.byref(params), ctypes.byref(grid), int(precision), _ptr(Q), _ptr(R), _ptr(ws),
                         nbytes, _stream(stream)))


FILTER_ALPHA = 0.135   # filtering coefficient of Section 4


def nopcs_filter(params, grid, Q, alpha_f=FILTER_ALPHA, stream=None):
    """The implicit 3D filter of a device state Q, in place."""
    _check(lib().nopcs_filter(ctypes.byref(params), ctypes.byref(grid), float(alpha_f), _ptr(Q), _stream(stream)))


def rk_step_filtered(params, grid, Q, dt, nsteps, ws, filter_every=50, alpha_f=FILTER_ALPHA, precision=FP64,
                     stream=None):
    """rk_step with the implicit filter after every filter_every-th step."""
    nbytes = ws.numel() * ws.element_size()
    _check(lib().rk_step_filtered(ctypes.byref(params), ctypes.byref(grid), int(precision), _ptr(Q), float(dt),
                                  int(nsteps), int(filter_every), float(alpha_f), _ptr(ws), nbytes, _stream(stream)))


NOALLOC_SCRATCH_BYTES = 64 << 20   # NOPCS_NOALLOC_SCRATCH_BYTES


def nse_rhs_noalloc(params, grid, Q, R, precision=FP64, stream=None):
    """R = right-hand side of ge17 at Q with no allocation: the library's static
    scratch array replaces the workspace; the grid's plans must be cached."""
    _check(lib().nse_rhs_noalloc(ctypes.byref(params), ctypes.byref(grid), int(precision), _ptr(Q), _ptr(R),
                                 _stream(stream)))


def compact_viscous_workspace_bytes(grid):
    return lib().nopcs_compact_viscous_workspace_bytes(ctypes.byref(grid))


def nse_rhs_compact_viscous(params, grid, Q, R, ws=None, stream=None):
    """R = right-hand side of ge17 with the viscous terms by the compact first
    derivative.  ws: device workspace of compact_viscous_workspace_bytes(grid)
    bytes; allocated here when not given."""
    if ws is None:
        import torch
        nb = compact_viscous_workspace_bytes(grid)
        if nb == 0:
            raise NopcsError(NOPCS_EINVAL, last_error())
        ws = torch.empty(nb, dtype=torch.uint8, device=Q.device)
    _check(lib().nse_rhs_compact_viscous(ctypes.byref(params), ctypes.byref(grid), _ptr(Q), _ptr(R), _ptr(ws),
                                         ws.numel() * ws.element_size(), _stream(stream)))


def rk_step_batch(params, boxes, dt, nsteps, precision=FP64, stream=None):
    """rk_step for a batch of boxes [(grid, Q, ws) or (grid, Q, ws, dt_box), ...]
    (small boxes share one launch per stage kernel, large ones run their own;
    one graph replay per step)."""
    arr = (Box * len(boxes))()
    for i, box in enumerate(boxes):
        grid, Q, ws = box[:3]
        arr[i].grid = grid
        arr[i].Q = Q.data_ptr()
        arr[i].ws = ws.data_ptr()
        arr[i].ws_bytes = ws.numel() * ws.element_size()
        arr[i].dt = float(box[3]) if len(box) > 3 else 0.0
    _check(lib().rk_step_batch(ctypes.byref(params), len(boxes), arr, int(precision), float(dt), int(nsteps),
                               _stream(stream)))


def set_graph_cache_limit(n):
    """Steps the library keeps cached (graphs, batched launches): 1..4096, default 64."""
    _check(lib().nopcs_set_graph_cache_limit(int(n)))


def set_batch_mode(mode):
    """0: every box in shared launches, as a graph; 1: one graph branch per box;
    2: shared launches issued directly (no graph); 3 (default): shared launches
    for boxes under 2^21 points and a branch for each larger one."""
    _check(lib().nopcs_set_batch_mode(int(mode)))


def rk_step_compact_viscous(params, grid, Q, dt, nsteps, ws, stream=None):
    """rk_step (FP64) with the D1-based viscous variant; ws of
    compact_viscous_workspace_bytes(grid) bytes."""
    _check(lib().rk_step_compact_viscous(ctypes.byref(params), ctypes.byref(grid), _ptr(Q), float(dt), int(nsteps),
                                         _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def rk_step(params, grid, Q, dt, nsteps, ws, precision=FP64, stream=None):
    nbytes = ws.numel() * ws.element_size()
    _check(lib().rk_step(ctypes.byref(params), ctypes.byref(grid), int(precision), _ptr(Q), float(dt), int(nsteps),
                         _ptr(ws), nbytes, _stream(stream)))


def autotune(params, grid, Q, ws, precision=FP64, stream=None):
    """Time rk_step for the candidate piece lengths, then the viscous z chunk,
    on a copy of Q; returns the chosen (x, y, z) lengths; lengths and chunk
    stay in force (process-wide; the chunk: visc_chunk(grid))."""
    out = (ctypes.c_int32 * 3)()
    _check(lib().nopcs_autotune(ctypes.byref(params), ctypes.byref(grid), int(precision), _ptr(Q), _ptr(ws),
                                ws.numel() * ws.element_size(), _stream(stream), ctypes.byref(out)))
    return tuple(out)


def set_piece_length(direction, length):
    _check(lib().nopcs_set_piece_length(int(direction), int(length)))


def set_visc_chunk(planes):
    """Planes per z chunk of the viscous kernel (0: the default)."""
    _check(lib().nopcs_set_visc_chunk(int(planes)))


def visc_chunk(grid):
    """The viscous z chunk in force for this grid."""
    v = lib().nopcs_visc_chunk(ctypes.byref(grid))
    if v < 0:
        raise NopcsError(v, last_error())
    return v


def alloc_workspace(grid, precision=FP64, device="cuda"):
    import torch
    nb = workspace_bytes(grid, precision)
    if nb == 0:
        raise NopcsError(NOPCS_EINVAL, last_error())
    return torch.empty(nb, dtype=torch.uint8, device=device)


class Solver:
    """Serving runtime (solver_create / submit / poll / destroy of include/nopcs.h).

    submit() copies the host initial state; poll() returns (status, result, Q)
    where status is NOPCS_EAGAIN while the request is pending.  Q is a new
    numpy array holding the final state once done."""

    def __init__(self, hbm_budget_bytes, max_slots=4, max_queue=1024, device=0, batched=False):
        cfg = SolverConfig(int(hbm_budget_bytes), int(max_slots), int(max_queue), int(device), int(bool(batched)))
        h = ctypes.c_void_p()
        _check(lib().solver_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._shapes = {}

    def submit(self, params, grid, Q0, nsteps, dt, precision=FP64):
        import numpy as np
        q = np.ascontiguousarray(Q0, dtype=np.float64)
        n = grid.n[0] * grid.n[1] * grid.n[2]
        if q.size != 5 * n:
            raise ValueError("Q0 must hold 5*n0*n1*n2 doubles")
        req = SolveRequest(params, grid, int(nsteps), int(precision), float(dt), q.ctypes.data_as(ctypes.c_void_p))
        rid = ctypes.c_uint64()
        _check(lib().solver_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        self._shapes[rid.value] = q.shape
        return rid.value

    def poll(self, rid):
        import numpy as np
        res = SolveResult()
        shape = self._shapes.get(rid)
        out = np.empty(shape, dtype=np.float64) if shape is not None else None
        ptr = out.ctypes.data_as(ctypes.c_void_p) if out is not None else None
        rc = lib().solver_poll(self._h, ctypes.c_uint64(rid), ptr, ctypes.byref(res))
        if rc == NOPCS_EAGAIN:
            return rc, res, None
        if rc == NOPCS_ENOTFOUND:
            raise NopcsError(rc, last_error())
        self._shapes.pop(rid, None)
        return rc, res, out

    def now(self):
        return lib().solver_now(self._h)

    def close(self):
        if self._h is not None:
            _check(lib().solver_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
