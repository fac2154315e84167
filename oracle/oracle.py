"""ctypes binding of the FP64 CPU oracle (``nopcs_oracle.c``).

Test infrastructure only.  The library is compiled from source by ``build()``
(gcc, ``-O2 -ffp-contract=off -fno-fast-math -fopenmp``) when it is missing.
All arrays are C-contiguous float64 numpy arrays; 3D fields are indexed
``[k][j][i]`` (x fastest) and a state is ``Q[5, nz, ny, nx]`` holding
``[rho, rho u, rho v, rho w, E']`` with ``E' = rho e_t - Rh/(gamma-1)``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nopcs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libnopcs_oracle.so")
_lib = None

__all__ = [
    "build", "lib", "OraParams", "alpha", "b1", "b2", "nb", "thomas", "d1_line", "equiv_row",
    "d1_line_seg", "d1", "d1_seg", "d2", "rhs", "rhs_points", "apply_bc", "rk4", "rk4_linear",
    "scales", "segment_starts", "num_threads", "vorticity_budget", "disturbance_pressure", "line_spectrum", "rhs_compact_viscous", "rk4_compact_viscous",
    "filter_line", "filter_line_seg", "filter_equiv_row", "filter_dir", "filter_dir_seg", "filter_state",
    "rk4_filtered", "FILTER_ALPHA",
]

FILTER_ALPHA = 0.135   # filtering coefficient of Section 4


def build(force=False):
    """Compile the oracle shared library with gcc."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OraParams(ctypes.Structure):
    """SI parameters (Section 2); the oracle non-dimensionalizes them itself."""
    _fields_ = [(n, ctypes.c_double) for n in
                ("gamma", "R_gas", "g", "L", "T_s", "rho_s", "Pr", "mu_ref", "T_ref", "S_suth", "mub_a", "mub_b")] + \
               [("viscous", ctypes.c_int32), ("gravity", ctypes.c_int32)]

    @classmethod
    def from_dict(cls, d):
        return cls(**{k: d[k] for k, _ in cls._fields_})


_D = ctypes.c_double
_I = ctypes.c_int
_P = ctypes.c_void_p
_PD = ctypes.c_ssize_t


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        for name in ("ora_alpha", "ora_b1", "ora_b2"):
            getattr(L, name).restype = _D
            getattr(L, name).argtypes = []
        L.ora_nb.restype = _I
        L.ora_thomas.argtypes = [_I, _P, _P, _P, _P, _P, _P]
        L.ora_d1_line.argtypes = [_I, _D, _P, _PD, _P, _PD, _P]
        L.ora_equiv_row.argtypes = [_I, _I, _P, _P]
        L.ora_d1_line_seg.argtypes = [_I, _D, _I, _P, _P, _PD, _P, _PD, _P]
        L.ora_d1_3d.argtypes = [_P, _P, _I, _P, _P]
        L.ora_d1_3d_seg.argtypes = [_P, _P, _I, _I, _P, _P, _P]
        L.ora_d2_3d.argtypes = [_P, _P, _I, _P, _P]
        L.ora_rhs.argtypes = [ctypes.POINTER(OraParams), _P, _P, _P, _P]
        L.ora_rhs_compact_visc.argtypes = [ctypes.POINTER(OraParams), _P, _P, _P, _P]
        L.ora_rhs_points.argtypes = [ctypes.POINTER(OraParams), _P, _P, _P, _I, _P, _P]
        L.ora_apply_bc.argtypes = [ctypes.POINTER(OraParams), _P, _P]
        L.ora_rk4.argtypes = [ctypes.POINTER(OraParams), _P, _P, _P, _D, _I]
        L.ora_rk4_compact_visc.argtypes = [ctypes.POINTER(OraParams), _P, _P, _P, _D, _I]
        L.ora_rk4_linear.argtypes = [_D, _D, _D, _I]
        L.ora_rk4_linear.restype = _D
        L.ora_scales.argtypes = [ctypes.POINTER(OraParams), _P]
        L.ora_num_threads.restype = _I
        L.ora_filter_line.argtypes = [_I, _D, _P, _PD, _P, _PD, _P]
        L.ora_filter_equiv_row.argtypes = [_I, _D, _I, _P, _P]
        L.ora_filter_line_seg.argtypes = [_I, _D, _I, _P, _P, _PD, _P, _PD, _P]
        L.ora_filter_dir.argtypes = [_P, _I, _D, _P, _P]
        L.ora_filter_dir_seg.argtypes = [_P, _I, _D, _I, _P, _P, _P]
        L.ora_filter_state.argtypes = [ctypes.POINTER(OraParams), _P, _D, _P]
        L.ora_rk4_filtered.argtypes = [ctypes.POINTER(OraParams), _P, _P, _P, _D, _I, _D, _I]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dims(shape):
    """(nz, ny, nx) -> int32[3] = (nx, ny, nz)."""
    nz, ny, nx = shape
    return np.array([nx, ny, nz], dtype=np.int32)


def _lens(length):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(length, dtype=np.float64), (3,)))


def alpha():
    return lib().ora_alpha()


def b1():
    return lib().ora_b1()


def b2():
    return lib().ora_b2()


def nb():
    return lib().ora_nb()


def thomas(sub, dia, sup, rhs):
    """General tridiagonal solve (sub[0], sup[-1] ignored)."""
    sub, dia, sup, rhs = (_f64(a) for a in (sub, dia, sup, rhs))
    m = len(dia)
    x = np.empty(m)
    w = np.empty(m)
    lib().ora_thomas(m, _ptr(sub), _ptr(dia), _ptr(sup), _ptr(rhs), _ptr(x), _ptr(w))
    return x


def d1_line(f, h=1.0):
    f = _f64(f)
    n = len(f)
    out = np.empty(n)
    w = np.empty(8 * n)
    lib().ora_d1_line(n, 1.0 / h, _ptr(f), 1, _ptr(out), 1, _ptr(w))
    return out


def equiv_row(n, e):
    """Row e of the global C = A^-1 B with h = 1 (length n)."""
    row = np.empty(n)
    w = np.empty(8 * n)
    lib().ora_equiv_row(n, e, _ptr(row), _ptr(w))
    return row


def segment_starts(n, nseg):
    """Near-equal split of n points into nseg segments (remainder to the first ones)."""
    base, rem = divmod(n, nseg)
    starts, s = [], 0
    for k in range(nseg):
        starts.append(s)
        s += base + (1 if k < rem else 0)
    return np.array(starts, dtype=np.int32)


def d1_line_seg(f, seg_lo, h=1.0):
    f = _f64(f)
    n = len(f)
    seg_lo = np.ascontiguousarray(seg_lo, dtype=np.int32)
    out = np.empty(n)
    w = np.empty(16 * n)
    lib().ora_d1_line_seg(n, 1.0 / h, len(seg_lo), _ptr(seg_lo), _ptr(f), 1, _ptr(out), 1, _ptr(w))
    return out


def d1(f, direction, length=1.0):
    """First derivative of a 3D field f[k, j, i] along direction 0 (x), 1 (y) or 2 (z)."""
    f = _f64(f)
    out = np.empty_like(f)
    lib().ora_d1_3d(_ptr(_dims(f.shape)), _ptr(_lens(length)), int(direction), _ptr(f), _ptr(out))
    return out


def d1_seg(f, direction, seg_lo, length=1.0):
    f = _f64(f)
    out = np.empty_like(f)
    seg_lo = np.ascontiguousarray(seg_lo, dtype=np.int32)
    lib().ora_d1_3d_seg(_ptr(_dims(f.shape)), _ptr(_lens(length)), int(direction), len(seg_lo), _ptr(seg_lo),
                        _ptr(f), _ptr(out))
    return out


def d2(f, direction, length=1.0):
    f = _f64(f)
    out = np.empty_like(f)
    lib().ora_d2_3d(_ptr(_dims(f.shape)), _ptr(_lens(length)), int(direction), _ptr(f), _ptr(out))
    return out


def rhs(params, Q, length=1.0):
    """Right-hand side R(Q) of ge17 for a state Q[5, nz, ny, nx]."""
    Q = _f64(Q)
    R = np.empty_like(Q)
    p = OraParams.from_dict(params)
    lib().ora_rhs(ctypes.byref(p), _ptr(_dims(Q.shape[1:])), _ptr(_lens(length)), _ptr(Q), _ptr(R))
    return R


def rhs_compact_viscous(params, Q, length=1.0):
    """Right-hand side of ge17 with the viscous terms differentiated by the
    compact first derivative (gradients of u, v, w, T and the divergence of
    Ev, Fv, Gv) instead of the explicit second-order differences."""
    Q = _f64(Q)
    R = np.empty_like(Q)
    p = OraParams.from_dict(params)
    lib().ora_rhs_compact_visc(ctypes.byref(p), _ptr(_dims(Q.shape[1:])), _ptr(_lens(length)), _ptr(Q), _ptr(R))
    return R


def rhs_points(params, Q, pts, length=1.0):
    """R(Q) at the points pts[m, 3] = (i, j, k); returns [5, m]."""
    Q = _f64(Q)
    pts = np.ascontiguousarray(pts, dtype=np.int32)
    out = np.empty((5, len(pts)))
    p = OraParams.from_dict(params)
    lib().ora_rhs_points(ctypes.byref(p), _ptr(_dims(Q.shape[1:])), _ptr(_lens(length)), _ptr(Q), len(pts),
                         _ptr(pts), _ptr(out))
    return out


def apply_bc(params, Q):
    Q = _f64(Q).copy()
    p = OraParams.from_dict(params)
    lib().ora_apply_bc(ctypes.byref(p), _ptr(_dims(Q.shape[1:])), _ptr(Q))
    return Q


def rk4(params, Q, dt, nsteps, length=1.0):
    """Advance Q by nsteps classical RK4 steps of size dt (returns a new array)."""
    Q = _f64(Q).copy()
    p = OraParams.from_dict(params)
    lib().ora_rk4(ctypes.byref(p), _ptr(_dims(Q.shape[1:])), _ptr(_lens(length)), _ptr(Q), float(dt), int(nsteps))
    return Q


def rk4_compact_viscous(params, Q, dt, nsteps, length=1.0):
    """rk4 with the D1-based viscous variant of the right-hand side."""
    Q = _f64(Q).copy()
    p = OraParams.from_dict(params)
    lib().ora_rk4_compact_visc(ctypes.byref(p), _ptr(_dims(Q.shape[1:])), _ptr(_lens(length)), _ptr(Q), float(dt),
                               int(nsteps))
    return Q


def rk4_linear(q0, lam, dt, nsteps):
    return lib().ora_rk4_linear(float(q0), float(lam), float(dt), int(nsteps))


def num_threads():
    """OpenMP threads the oracle's parallel loops use."""
    return lib().ora_num_threads()


def scales(params):
    """(U_s, t_s, Rh, M, Re, mu_s) as computed by the oracle."""
    out = np.empty(6)
    p = OraParams.from_dict(params)
    lib().ora_scales(ctypes.byref(p), _ptr(out))
    return tuple(out)


def vorticity_budget(params, Q, length=1.0):
    """Vorticity and the three source terms on the right of the inviscid
    vorticity transport equation (Eq. eqn12_1, the terms the paper's results
    section plots): omega = curl V; stretching (omega . grad) V; dilatation
    -omega (div V); baroclinic (grad rho x grad p) / rho^2.  Every derivative
    is the compact first derivative ``d1`` (global line solves); V = (rho u,
    rho v, rho w) / rho and p' = (gamma - 1)(E' - rho |V|^2 / 2) (ge12, ge13;
    the constant p - p' drops out of grad p).  Returns [12, nz, ny, nx]: omega,
    stretching, dilatation, baroclinic (x, y, z each); sums run over x, y, z.
    """
    Q = _f64(Q)
    rho = Q[0]
    V = [Q[1] / rho, Q[2] / rho, Q[3] / rho]
    ke = 0.5 * (Q[1] * V[0] + Q[2] * V[1] + Q[3] * V[2])
    pp = (params["gamma"] - 1.0) * (Q[4] - ke)
    g = [[d1(V[i], j, length) for j in range(3)] for i in range(3)]      # g[i][j] = d V_i / d x_j
    grho = [d1(rho, j, length) for j in range(3)]
    gp = [d1(pp, j, length) for j in range(3)]
    om = [g[2][1] - g[1][2], g[0][2] - g[2][0], g[1][0] - g[0][1]]
    div = (g[0][0] + g[1][1]) + g[2][2]
    out = np.empty((12,) + rho.shape)
    for i in range(3):
        out[i] = om[i]
        out[3 + i] = (om[0] * g[i][0] + om[1] * g[i][1]) + om[2] * g[i][2]
        out[6 + i] = -(om[i] * div)
    r2 = rho * rho
    out[9] = (grho[1] * gp[2] - grho[2] * gp[1]) / r2
    out[10] = (grho[2] * gp[0] - grho[0] * gp[2]) / r2
    out[11] = (grho[0] * gp[1] - grho[1] * gp[0]) / r2
    return out


def disturbance_pressure(params, Q, Q0):
    """Disturbance pressure p - p_h (Section 4: the instantaneous pressure minus
    the initial hydrostatic one): p' of Q minus p' of the initial state Q0, with
    p' = (gamma - 1)(E' - rho |V|^2 / 2) (ge12, ge13), taken as
    (gamma - 1)((E' - E'_0) - (k - k_0)) with k = (rho u u + rho v v + rho w w) / 2,
    the same difference without forming the two large pressures first."""
    Q = _f64(Q)
    Q0 = _f64(Q0)

    def ke(S):
        r = S[0]
        return 0.5 * ((S[1] * (S[1] / r) + S[2] * (S[2] / r)) + S[3] * (S[3] / r))

    return (params["gamma"] - 1.0) * ((Q[4] - Q0[4]) - (ke(Q) - ke(Q0)))


def line_spectrum(f):
    """Amplitude spectrum of a line of n samples (the Fourier transform of the
    disturbance pressure along y, Section 4): |sum_j f_j exp(-2 pi i j k / n)| / n
    for k = 0 .. n // 2, by the library FFT."""
    f = np.asarray(f, dtype=np.float64)
    return np.abs(np.fft.rfft(f)) / f.size


# ---------------------------------------------------------------------------
# Implicit filter of Section 4 (reading: fourth-order tridiagonal compact
# filter, wall rows unfiltered, applied along x, y, z in turn)
# ---------------------------------------------------------------------------
def filter_line(f, af=FILTER_ALPHA):
    """Filtered line (global solve)."""
    f = _f64(f)
    n = len(f)
    out = np.empty(n)
    work = np.empty(8 * n)
    lib().ora_filter_line(n, float(af), _ptr(f), 1, _ptr(out), 1, _ptr(work))
    return out


def filter_equiv_row(n, e, af=FILTER_ALPHA):
    """Row e of the filter's equivalent explicit operator A_f^-1 B_f on n points."""
    row = np.empty(n)
    work = np.empty(8 * n)
    lib().ora_filter_equiv_row(int(n), float(af), int(e), _ptr(row), _ptr(work))
    return row


def filter_line_seg(f, seg_lo, af=FILTER_ALPHA):
    """Segmented (NOHAP) filter of one line; seg_lo: segment starts."""
    f = _f64(f)
    n = len(f)
    lo = np.ascontiguousarray(seg_lo, dtype=np.int32)
    out = np.empty(n)
    work = np.empty(16 * n + n // 8 + 8)
    lib().ora_filter_line_seg(n, float(af), len(lo), _ptr(lo), _ptr(f), 1, _ptr(out), 1, _ptr(work))
    return out


def filter_dir(f, direction, af=FILTER_ALPHA):
    """Filter a 3D field f[nz, ny, nx] along one direction (global line solves)."""
    f = _f64(f)
    out = np.empty_like(f)
    lib().ora_filter_dir(_ptr(_dims(f.shape)), int(direction), float(af), _ptr(f), _ptr(out))
    return out


def filter_dir_seg(f, direction, nseg, af=FILTER_ALPHA):
    """Segmented (NOHAP) filter along one direction with nseg near-equal segments."""
    f = _f64(f)
    out = np.empty_like(f)
    n = f.shape[2 - direction]
    lo = np.ascontiguousarray(segment_starts(n, nseg), dtype=np.int32)
    lib().ora_filter_dir_seg(_ptr(_dims(f.shape)), int(direction), float(af), len(lo), _ptr(lo), _ptr(f), _ptr(out))
    return out


def filter_state(params, Q, af=FILTER_ALPHA):
    """3D filter of every conserved field (x, then y, then z), then the wall conditions."""
    Q = _f64(Q).copy()
    p = OraParams.from_dict(params)
    lib().ora_filter_state(ctypes.byref(p), _ptr(_dims(Q.shape[1:])), float(af), _ptr(Q))
    return Q


def rk4_filtered(params, Q, dt, nsteps, every=50, af=FILTER_ALPHA, length=1.0):
    """RK4 steps with the 3D filter after every `every`-th step (Section 4)."""
    Q = _f64(Q).copy()
    p = OraParams.from_dict(params)
    lib().ora_rk4_filtered(ctypes.byref(p), _ptr(_dims(Q.shape[1:])), _ptr(_lens(length)), _ptr(Q), float(dt),
                           int(nsteps), float(af), int(every))
    return Q
