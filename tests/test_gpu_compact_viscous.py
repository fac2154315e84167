"""GPU parity of the D1-based viscous variant of the right-hand side
(nse_rhs_compact_viscous) through the C ABI, against the oracle's
rhs_compact_viscous element by element: per field max|gpu - oracle| /
max|oracle| <= 1e-12.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2203_00879_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs an MI355X GPU", allow_module_level=True)

from paper_2203_00879_amd import nopcs  # noqa: E402

DEV = "cuda:0"
TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_rhs(params, Q, nseg, length, compact=True):
    nz, ny, nx = Q.shape[1:]
    g = nopcs.make_grid((nx, ny, nz), nseg, length)
    Qd = torch.from_numpy(np.ascontiguousarray(Q)).to(DEV)
    R = torch.empty_like(Qd)
    if compact:
        nopcs.nse_rhs_compact_viscous(nopcs.make_params(params), g, Qd, R)
    else:
        nopcs.nse_rhs(nopcs.make_params(params), g, Qd, R)
    torch.cuda.synchronize()
    return R.cpu().numpy()


def check(R, Ro):
    for c in range(5):
        scale = np.max(np.abs(Ro[c]))
        err = np.max(np.abs(R[c] - Ro[c])) / (scale if scale > 0 else 1.0)
        assert err <= TOL, (c, err)


CASES = [
    ((8, 8, 8), (1, 1, 1), 1.0, 1),
    ((40, 33, 37), (1, 2, 3), (1.0, 0.8, 1.1), 1),
    ((130, 70, 97), (3, 1, 2), 1.0, 1),
    ((40, 33, 37), (1, 2, 3), 1.0, 0),       # gravity off
]


@pytest.mark.parametrize("shape, nseg, length, gravity", CASES)
def test_compact_viscous_rhs_parity(shape, nseg, length, gravity):
    say("compact viscous parity", shape, nseg, length, gravity)
    p = dict(inputs.AIR, gravity=gravity)
    Q = inputs.smooth_state(shape, seed=13, length=length)
    R = gpu_rhs(p, Q, nseg, length)
    check(R, oracle.rhs_compact_viscous(p, Q, np.broadcast_to(np.asarray(length, float), (3,)).copy()))


@pytest.mark.parametrize("shape, nseg, length, gravity", CASES[1:3])
def test_compact_viscous_rhs_line_march_form(shape, nseg, length, gravity):
    """First derivatives along y and z by the line march (asked for on these
    small boxes): against the oracle, and within 1e-12 of the pencil form."""
    say("compact viscous parity, line march", shape, nseg, length, gravity)
    p = dict(inputs.AIR, gravity=gravity)
    Q = inputs.smooth_state(shape, seed=14, length=length)
    try:
        nopcs.set_deriv_form(nopcs.DERIV_MARCH)
        R = gpu_rhs(p, Q, nseg, length)
        nopcs.set_deriv_form(nopcs.DERIV_PENCIL)
        P = gpu_rhs(p, Q, nseg, length)
    finally:
        nopcs.set_deriv_form(nopcs.DERIV_BY_SIZE)
    check(R, oracle.rhs_compact_viscous(p, Q, np.broadcast_to(np.asarray(length, float), (3,)).copy()))
    check(R, P)


def test_compact_viscous_rhs_parity_rti():
    say("compact viscous parity RTI 32^3")
    p = dict(inputs.AIR)
    Q = oracle.rk4(p, inputs.rti_state(32, seed=3, noise_K=1e-3), 2e-5, 2)
    check(gpu_rhs(p, Q, (2, 2, 2), 1.0), oracle.rhs_compact_viscous(p, Q))


def test_inviscid_variant_equals_nse_rhs_bitwise():
    """With the viscous terms off the two entry points run the same kernels."""
    p = dict(inputs.AIR, viscous=0)
    Q = inputs.smooth_state((24, 20, 28), seed=14)
    assert np.array_equal(gpu_rhs(p, Q, (2, 1, 2), 1.0), gpu_rhs(p, Q, (2, 1, 2), 1.0, compact=False))


@pytest.mark.parametrize("shape, nseg", [((32, 32, 32), (2, 2, 2)), ((24, 40, 96), (1, 2, 3))])
def test_rk_step_compact_viscous_parity(shape, nseg):
    """Two RK4 steps with the variant against the oracle: fields <= 1e-12 and
    their change over the steps <= 1e-9 (relative to each field's maximum)."""
    say("rk compact viscous", shape, nseg)
    p = dict(inputs.AIR)
    Q0 = inputs.rti_state(shape, seed=4, noise_K=1e-3)
    nx, ny, nz = shape
    g = nopcs.make_grid(shape, nseg)
    Qd = torch.from_numpy(Q0.copy()).to(DEV)
    ws = torch.empty(nopcs.compact_viscous_workspace_bytes(g), dtype=torch.uint8, device=DEV)
    nopcs.rk_step_compact_viscous(nopcs.make_params(p), g, Qd, 2e-5, 2, ws)
    torch.cuda.synchronize()
    G = Qd.cpu().numpy()
    O = oracle.rk4_compact_viscous(p, Q0, 2e-5, 2)
    for c in range(5):
        s = np.max(np.abs(O[c]))
        assert np.max(np.abs(G[c] - O[c])) / s <= TOL, c
        ch = np.max(np.abs(O[c] - Q0[c]))
        if ch > 0:
            assert np.max(np.abs((G[c] - Q0[c]) - (O[c] - Q0[c]))) / ch <= 1e-9, c


def test_compact_viscous_512_quadratic_flow_closed_form():
    """Full size (512^3, 4 segments): rho = T = 1 and a quadratic V, for which
    every compact derivative is exact; the viscous momentum terms (the RHS with
    viscous terms on minus off) equal (mu lap V_i + (beta + mu/3) d_i div V) / Re
    everywhere, up to the rounding of second differences (h^-2 ~ 2.6e5;
    measured 9.4e-10 of the largest term)."""
    n = 512
    say("compact viscous 512 quadratic flow")
    rng = np.random.default_rng(12)
    a = rng.uniform(-0.01, 0.01, 3)
    B = rng.uniform(-0.01, 0.01, (3, 3))
    C = rng.uniform(-0.01, 0.01, (3, 3, 3))
    C = 0.5 * (C + C.transpose(0, 2, 1))
    c = torch.linspace(0.0, 1.0, n, dtype=torch.float64, device=DEV)
    X = (c.view(1, 1, n), c.view(1, n, 1), c.view(n, 1, 1))
    Q = torch.zeros((5, n, n, n), dtype=torch.float64, device=DEV)
    Q[0] = 1.0
    for i in range(3):
        Vi = torch.full((n, n, n), float(a[i]), dtype=torch.float64, device=DEV)
        for j in range(3):
            Vi += float(B[i, j]) * X[j]
            for k in range(3):
                Vi += float(C[i, j, k]) * (X[j] * X[k])
        Q[1 + i] = Vi
        Q[4] += 0.5 * Vi * Vi
        del Vi
    g = nopcs.make_grid(n, 4)
    R1 = torch.empty_like(Q)
    ws = torch.empty(nopcs.compact_viscous_workspace_bytes(g), dtype=torch.uint8, device=DEV)
    p_on, p_off = dict(inputs.AIR, gravity=0), dict(inputs.AIR, gravity=0, viscous=0)
    nopcs.nse_rhs_compact_viscous(nopcs.make_params(p_on), g, Q, R1, ws)
    R0 = torch.empty_like(Q)
    nopcs.nse_rhs_compact_viscous(nopcs.make_params(p_off), g, Q, R0, ws)
    torch.cuda.synchronize()
    Us, ts, Rh, M, Re, mu_s = oracle.scales(p_on)
    beta = (p_on["mub_a"] * p_on["T_s"] - p_on["mub_b"]) / mu_s
    lap = np.array([2.0 * np.trace(C[i]) for i in range(3)])
    gdiv = np.array([2.0 * sum(C[j, j, i] for j in range(3)) for i in range(3)])
    want = (lap + (beta + 1.0 / 3.0) * gdiv) / Re
    scale = np.max(np.abs(want))
    for i in range(3):
        err = float((R1[1 + i] - R0[1 + i] - want[i]).abs().max()) / scale
        say("  momentum", i, "err", err)
        assert err <= 1e-8
