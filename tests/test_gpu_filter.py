"""GPU: the implicit 3D filter of Section 4 (nopcs_filter) and RK4 stepping
with it (rk_step_filtered) against the FP64 oracle on the same seeded inputs.
The filter's reading (fourth-order tridiagonal compact filter, coefficient
0.135, wall rows unfiltered, x then y then z) is pinned in test_oracle_pins."""
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
P = dict(inputs.AIR)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    s = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (s if s > 0 else 1.0))


def _moving_state(shape, seed):
    Q = inputs.smooth_state(shape, seed=seed)
    Q[1:4] += np.random.default_rng(seed).normal(scale=1e-3, size=Q[1:4].shape)
    return Q


@pytest.mark.parametrize("shape, nseg", [((8, 8, 8), (1, 1, 1)), ((40, 33, 37), (1, 2, 3)),
                                         ((130, 70, 97), (3, 1, 2)), ((64, 64, 64), (2, 4, 16))])
def test_filter_parity(shape, nseg):
    say("filter", shape, nseg)
    Q = _moving_state(shape, sum(shape))
    g = nopcs.make_grid(shape, nseg)
    Qd = torch.from_numpy(Q).to(DEV)
    nopcs.nopcs_filter(nopcs.make_params(P), g, Qd)
    torch.cuda.synchronize()
    G = Qd.cpu().numpy()
    O = oracle.filter_state(P, Q)
    errs = [_rel(G[c], O[c]) for c in range(5)]
    say("  errors", ["%.2e" % e for e in errs])
    assert max(errs) <= TOL


def test_filter_512_bench_configuration():
    """The 512^3 box of the RK benchmark (4 segments per direction, default
    pieces), an RTI state with 1 K interface noise and small random momentum:
    every point of all 5 fields against the oracle's global line solves."""
    n = 512
    say("building 512^3 state")
    Q = inputs.rti_state(n, seed=2, noise_K=1.0)
    Q[1:4] = np.random.default_rng(3).normal(scale=1e-4, size=Q[1:4].shape)
    g = nopcs.make_grid(n, 4)
    Qd = torch.from_numpy(Q).to(DEV)
    nopcs.nopcs_filter(nopcs.make_params(P), g, Qd)
    torch.cuda.synchronize()
    G = Qd.cpu().numpy()
    del Qd
    torch.cuda.empty_cache()
    say("oracle filter at 512^3")
    O = oracle.filter_state(P, Q)
    for c in range(5):
        e = _rel(G[c], O[c])
        ch = float(np.max(np.abs(G[c] - O[c])) / max(np.max(np.abs(O[c] - Q[c])), 1e-300))
        say("  field", c, "err %.3e of the field, %.3e of its change" % (e, ch))
        assert e <= TOL and ch <= TOL


def test_filter_keeps_cubics_and_removes_the_two_point_mode_at_512():
    """Closed forms at full size: a field cubic in x, y and z passes the filter
    unchanged (fourth order, wall rows unfiltered), the three-dimensional
    two-point mode vanishes away from the walls."""
    n = 512
    g = nopcs.make_grid(n, 4)
    x = torch.linspace(-1.0, 1.0, n, dtype=torch.float64, device=DEV)
    cub = (0.3 + x - 0.7 * x ** 2 + 0.4 * x ** 3)
    Q = torch.empty((5, n, n, n), dtype=torch.float64, device=DEV)
    Q[0] = 1.0 + 0.1 * cub[None, None, :] * cub[None, :, None] * cub[:, None, None]
    Q[1:4] = 0.0
    Q[4] = 0.05 * cub[None, None, :] + 0.02 * cub[None, :, None] - 0.03 * cub[:, None, None]
    Q0 = Q.clone()
    nopcs.nopcs_filter(nopcs.make_params(P), g, Q)
    torch.cuda.synchronize()
    inner = (slice(1, n - 1),) * 3          # the wall conditions rewrite the wall nodes
    for c in (0, 4):
        e = float((Q[c][inner] - Q0[c][inner]).abs().max() / Q0[c].abs().max())
        say("  cubic field", c, "change %.2e" % e)
        assert e <= 1e-13
    i = torch.arange(n, device=DEV)
    alt = ((-1.0) ** (i[None, None, :] + i[None, :, None] + i[:, None, None])).to(torch.float64)
    Q[0] = 1.0 + 1e-3 * alt
    Q[4] = 1e-3 * alt
    nopcs.nopcs_filter(nopcs.make_params(P), g, Q)
    torch.cuda.synchronize()
    mid = (slice(24, n - 24),) * 3
    r = float((Q[0][mid] - 1.0).abs().max())
    e = float(Q[4][mid].abs().max())
    say("  two-point mode left: rho %.2e E' %.2e (of 1e-3)" % (r, e))
    assert r <= 1e-15 and e <= 1e-15
    del Q, Q0, alt
    torch.cuda.empty_cache()


def test_filtered_stepping_against_oracle():
    """rk_step_filtered: 110 RK4 steps with the filter after steps 50 and 100,
    on a box in motion (2 x 3 x 2 segments) and on the RTI box (4 segments;
    rho and E' only: its momentum is so small after a few steps that the
    filter's rounding of rho is of the order of 1e-12 of it)."""
    shape = (40, 36, 44)
    Q = inputs.smooth_state(shape, seed=9, amp_u=0.02)
    g = nopcs.make_grid(shape, (2, 3, 2))
    Qd = torch.from_numpy(Q).to(DEV)
    ws = nopcs.alloc_workspace(g)
    nopcs.rk_step_filtered(nopcs.make_params(P), g, Qd, 2e-6, 110, ws, filter_every=50)
    torch.cuda.synchronize()
    O = oracle.rk4_filtered(P, Q, 2e-6, 110, every=50)
    G = Qd.cpu().numpy()
    errs = [_rel(G[c], O[c]) for c in range(5)]
    say("  moving box errors", ["%.2e" % e for e in errs])
    assert max(errs) <= TOL
    n = 64
    Q = inputs.rti_state(n, seed=1, noise_K=1.0)
    g = nopcs.make_grid(n, 4)
    Qd = torch.from_numpy(Q).to(DEV)
    ws = nopcs.alloc_workspace(g)
    nopcs.rk_step_filtered(nopcs.make_params(P), g, Qd, 1e-5, 60, ws, filter_every=50)
    torch.cuda.synchronize()
    O = oracle.rk4_filtered(P, Q, 1e-5, 60, every=50)
    G = Qd.cpu().numpy()
    errs = [_rel(G[c], O[c]) for c in range(5)]
    say("  RTI box errors", ["%.2e" % e for e in errs])
    assert errs[0] <= TOL and errs[4] <= TOL
