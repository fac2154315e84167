"""GPU parity of the vorticity budget (Eq. eqn12_1) through the C ABI.

Small boxes: element by element against the oracle (global compact line
solves), per output component, max|gpu - oracle| / max|oracle| <= 1e-12.  The
512^3 box of the RK benchmark: a linear flow, for which every compact
derivative is exact, against its closed form at every point.
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
PARAMS = dict(inputs.AIR)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_budget(Q, nseg, length):
    nz, ny, nx = Q.shape[1:]
    g = nopcs.make_grid((nx, ny, nz), nseg, length)
    Qd = torch.from_numpy(np.ascontiguousarray(Q)).to(DEV)
    out = torch.empty((12, nz, ny, nx), dtype=torch.float64, device=DEV)
    nopcs.vorticity_budget(nopcs.make_params(PARAMS), g, Qd, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(G, O, tol=TOL):
    for c in range(12):
        scale = np.max(np.abs(O[c]))
        err = np.max(np.abs(G[c] - O[c])) / (scale if scale > 0 else 1.0)
        assert err <= tol, (c, err)


CASES = [
    ((8, 8, 8), (1, 1, 1), 1.0),                      # smallest grid
    ((40, 33, 37), (1, 2, 3), (1.0, 0.8, 1.1)),       # ragged, uneven segments, unequal lengths
    ((130, 70, 97), (3, 1, 2), 1.0),                  # crosses the 128-point class
]


@pytest.mark.parametrize("shape, nseg, length", CASES)
def test_vorticity_budget_parity_smooth_state(shape, nseg, length):
    say("vorticity parity", shape, nseg, length)
    Q = inputs.smooth_state(shape, seed=11, length=length)
    G = gpu_budget(Q, nseg, length)
    check(G, oracle.vorticity_budget(PARAMS, Q, np.broadcast_to(np.asarray(length, float), (3,)).copy()))


def test_vorticity_budget_parity_rti_after_steps():
    """An RTI box a few oracle RK4 steps after the partition is removed: the
    baroclinic term at the interface is the largest source (Section 5)."""
    say("vorticity parity RTI 24^3")
    Q = inputs.rti_state(24, seed=2, noise_K=1e-3)
    Q = oracle.rk4(PARAMS, Q, 2e-5, 3)
    G = gpu_budget(Q, (2, 2, 2), 1.0)
    O = oracle.vorticity_budget(PARAMS, Q)
    check(G, O)
    assert np.max(np.abs(O[9:12])) > 0.0


def test_vorticity_budget_512_linear_flow_closed_form():
    """Full size, 4 segments per direction: V = M x + v0, rho and p' linear.
    omega_i = eps_ijk M[k, j], stretching = M omega, dilatation = -omega tr M,
    baroclinic = (grad rho x grad p') / rho^2, at every point."""
    n, nseg = 512, 4
    say("vorticity closed form", n, nseg)
    rng = np.random.default_rng(5)
    M = rng.uniform(-0.3, 0.3, (3, 3))
    v0 = rng.uniform(-0.1, 0.1, 3)
    grho = rng.uniform(-0.2, 0.2, 3)
    gp = rng.uniform(-0.5, 0.5, 3)
    gamma = PARAMS["gamma"]
    c = torch.linspace(0.0, 1.0, n, dtype=torch.float64, device=DEV)
    X = (c.view(1, 1, n), c.view(1, n, 1), c.view(n, 1, 1))     # x, y, z on axes (z, y, x)
    Q = torch.empty((5, n, n, n), dtype=torch.float64, device=DEV)
    rho = 1.3 + (grho[0] * X[0] + grho[1] * X[1] + grho[2] * X[2])
    Q[0] = rho
    ke = torch.zeros((n, n, n), dtype=torch.float64, device=DEV)
    for i in range(3):
        Vi = v0[i] + (M[i, 0] * X[0] + M[i, 1] * X[1] + M[i, 2] * X[2])
        Q[1 + i] = rho * Vi
        ke += Vi * Vi
        del Vi
    Q[4] = (0.7 + (gp[0] * X[0] + gp[1] * X[1] + gp[2] * X[2])) / (gamma - 1.0) + 0.5 * rho * ke
    del ke
    g = nopcs.make_grid(n, nseg)
    out = torch.empty((12, n, n, n), dtype=torch.float64, device=DEV)
    nopcs.vorticity_budget(nopcs.make_params(PARAMS), g, Q, out)
    torch.cuda.synchronize()
    om = np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
    want = list(om) + list(M @ om) + list(-om * np.trace(M))
    scale = np.max(np.abs(want))
    for k in range(9):
        err = float((out[k] - want[k]).abs().max()) / scale
        say("component", k, "err", err)
        assert err <= 1e-11, (k, err)
    baro = np.cross(grho, gp)
    for k in range(3):
        err = float((out[9 + k] * rho * rho - baro[k]).abs().max()) / np.max(np.abs(baro))
        say("baroclinic", k, "err", err)
        assert err <= 1e-10, (k, err)
