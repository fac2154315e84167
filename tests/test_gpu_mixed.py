"""Mixed precision (NOPCS_MIXED) on the GPU.  rk_step: FP32 eliminations along
y and z, the x sweep staged and solved in FP32 on offset fluxes (each flux
less its line's first-row value), the viscous differences, stresses, heat
fluxes and their divergence in FP32, an FP32 RHS register; state, primitives,
known rows and the RK registers in FP64.  nse_rhs (FP64 output): the FP32
eliminations along y and z only.

Error budget: each FP32 run sees its right-hand side rounded once (unit
roundoff 6e-8: (B f)_i along y and z, the offset flux values along x, whose
size is the line's own variation) and amplifies it by at most the row sum of
|A^-1| (< 4.4), so the right-hand side is within about 3e-7 of each
component's maximum; the viscous terms carry FP32 roundings of the same size
relative to their own magnitude, and the RHS register in FP32 adds one more
rounding.  The tolerances below give a factor of 3-30 over that."""
import numpy as np
import pytest

import oracle
from paper_2203_00879_amd import inputs, nopcs

pytestmark = pytest.mark.gpu


def _rel(a, b):
    s = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (s if s > 0 else 1.0)


@pytest.mark.parametrize("shape, nseg", [((40, 130, 97), (1, 3, 2)), ((64, 64, 64), (2, 2, 2)),
                                         ((1024, 10, 9), (5, 1, 1)),    # longest x lines: FP32 1024-point pencils
                                         ((10, 1024, 9), (1, 7, 1)),    # longest y lines
                                         ((9, 10, 1024), (1, 1, 9))])   # longest z lines
def test_rhs_mixed_against_oracle(shape, nseg):
    import torch
    p = dict(inputs.AIR)
    Q = inputs.smooth_state(shape, seed=17)
    g = nopcs.make_grid(shape, nseg)
    Qd = torch.from_numpy(Q).to("cuda")
    Rd = torch.empty_like(Qd)
    nopcs.nse_rhs(nopcs.make_params(p), g, Qd, Rd, precision=nopcs.MIXED)
    torch.cuda.synchronize()
    R = Rd.cpu().numpy()
    Ro = oracle.rhs(p, Q)
    errs = [_rel(R[c], Ro[c]) for c in range(5)]
    print(shape, "mixed RHS relative errors", ["%.2e" % e for e in errs], flush=True)
    assert max(errs) <= 1e-6 and max(errs) > 0


@pytest.mark.parametrize("shape, nseg", [((40, 36, 70), (2, 3, 2)), ((130, 24, 40), (3, 1, 2))])
def test_rhs_mixed_uniform_motion_is_the_gravity_source(shape, nseg):
    """A uniform state in uniform motion has no derivative of any flux (the
    oracle's pin: R = [0, 0, -rho, 0, -rho v]).  nse_rhs in mixed precision
    (FP32 eliminations along y and z on (B f)_i formed in FP64) must keep every
    derivative exactly zero: rho, rho u and rho w come out exactly zero and the
    two source components within one FP32 rounding of the oracle."""
    import torch
    p = dict(inputs.AIR)
    rho, vel = 0.83, (0.31, -0.47, 0.19)
    Q = inputs.uniform_state(shape, T=1.3, rho=rho, velocity=vel, params=p)
    g = nopcs.make_grid(shape, nseg)
    Qd = torch.from_numpy(Q).to("cuda")
    Rd = torch.empty_like(Qd)
    nopcs.nse_rhs(nopcs.make_params(p), g, Qd, Rd, precision=nopcs.MIXED)
    torch.cuda.synchronize()
    R = Rd.cpu().numpy()
    Ro = oracle.rhs(p, Q)
    for c in (0, 1, 3):
        assert np.all(R[c] == 0.0), (c, np.max(np.abs(R[c])))
    for c in (2, 4):
        scale = np.max(np.abs(Ro[c]))
        assert scale > 0
        assert np.max(np.abs(R[c] - Ro[c])) <= 2.0 ** -23 * scale, (c, np.max(np.abs(R[c] - Ro[c])) / scale)


# Per-field bound of mixed-precision RK4 stepping, relative to the largest change
# of the field over the run: each stage's right-hand side carries about 3e-7
# of its components' maxima from the FP32 runs (see the module docstring), and
# the change over the run is the dt-weighted sum of those right-hand sides, so
# the change inherits the same relative error.  The FP32 viscous terms add up
# to a few times that where heat conduction or the bulk-viscosity dilatation
# term dominates a component's change: measured up to 1.1e-6 (rho v over the
# first 2 steps of the 100 K / 300 K setup) and 6.4e-7 at 512^3 over 5 steps.
MIXED_CHANGE_BOUND = 2e-6


def test_rk_mixed_against_oracle_and_fp64():
    """RTI box 64^3, 4 segments, 10 steps: the change of every field over the run,
    FP64 on the GPU against the oracle (<= 1e-12) and mixed precision against
    the oracle (<= MIXED_CHANGE_BOUND) and against GPU FP64."""
    import torch
    p = dict(inputs.AIR)
    n, steps, dt = 64, 10, 1e-5
    Q0 = inputs.rti_state(n, seed=3, noise_K=1.0)
    g = nopcs.make_grid(n, 4)
    out = {}
    for prec in (nopcs.FP64, nopcs.MIXED):
        Qd = torch.from_numpy(Q0).to("cuda")
        ws = nopcs.alloc_workspace(g, prec)
        nopcs.rk_step(nopcs.make_params(p), g, Qd, dt, steps, ws, precision=prec)
        torch.cuda.synchronize()
        out[prec] = Qd.cpu().numpy()
    O = oracle.rk4(p, Q0, dt, steps)
    do = O - Q0
    d64, d32 = out[nopcs.FP64] - Q0, out[nopcs.MIXED] - Q0
    e64 = [_rel(d64[c], do[c]) for c in range(5)]
    e32 = [_rel(d32[c], do[c]) for c in range(5)]
    e32_64 = [_rel(d32[c], d64[c]) for c in range(5)]
    print("change over 10 steps, relative max errors: FP64 vs oracle", ["%.2e" % e for e in e64],
          "mixed vs oracle", ["%.2e" % e for e in e32], "mixed vs FP64", ["%.2e" % e for e in e32_64], flush=True)
    assert np.isfinite(out[nopcs.MIXED]).all()
    assert max(e64) <= 1e-12
    assert max(e32) <= MIXED_CHANGE_BOUND and max(e32_64) <= MIXED_CHANGE_BOUND


def _gpu_rk(p, Q0, nseg, dt, steps, prec):
    import torch
    g = nopcs.make_grid(Q0.shape[1:][::-1], nseg)
    Qd = torch.from_numpy(Q0).to("cuda")
    ws = nopcs.alloc_workspace(g, prec)
    nopcs.rk_step(nopcs.make_params(p), g, Qd, dt, steps, ws, precision=prec)
    torch.cuda.synchronize()
    out = Qd.cpu().numpy()
    del Qd, ws
    torch.cuda.empty_cache()
    return out


def test_rk_mixed_paper_setup_uneven_segments():
    """The paper's own setup at small scale (Section 4: 100 K over 300 K, h_y =
    h_x / 2, uneven segments along every direction) in mixed precision: the
    change of every field over 2 RK4 steps against the oracle, within
    MIXED_CHANGE_BOUND of its largest value."""
    p = dict(inputs.AIR)
    Q0 = inputs.rti_state((32, 64, 32), T_upper=100.0, T_lower=300.0, seed=5, noise_K=1e-3)
    G = _gpu_rk(p, Q0, (3, 5, 3), 2e-6, 2, nopcs.MIXED)
    O = oracle.rk4(p, Q0, 2e-6, 2)
    errs = [_rel(G[c] - Q0[c], O[c] - Q0[c]) for c in range(5)]
    print("paper setup, mixed vs oracle (change)", ["%.2e" % e for e in errs], flush=True)
    assert np.isfinite(G).all()
    assert max(errs) <= MIXED_CHANGE_BOUND


def test_rk_mixed_512_bench_configuration():
    """The timed configuration (RTI box 512^3, 4 segments per direction, dt =
    1e-6) in mixed precision against GPU FP64 (itself held to the oracle at
    1e-12 in the parity tests): the change of every field over 5 steps within
    MIXED_CHANGE_BOUND of its largest value, over the whole box."""
    p = dict(inputs.AIR)
    n, steps, dt = 512, 5, 1e-6
    Q0 = inputs.rti_state(n, seed=0)
    G64 = _gpu_rk(p, Q0, 4, dt, steps, nopcs.FP64)
    d64 = G64 - Q0
    del G64
    G32 = _gpu_rk(p, Q0, 4, dt, steps, nopcs.MIXED)
    assert np.isfinite(G32).all()
    errs = []
    for c in range(5):
        d32 = G32[c] - Q0[c]
        errs.append(_rel(d32, d64[c]))
        del d32
    print("512^3, 5 steps, mixed vs FP64 (change)", ["%.2e" % e for e in errs], flush=True)
    assert max(errs) <= MIXED_CHANGE_BOUND


def test_rk_mixed_pencil_fallback_against_oracle():
    """Runs longer than a line march holds (48^3, one segment per direction:
    runs of 46 points) step through the LDS pencils along every direction, in
    mixed precision staged and solved in FP32 on offset fluxes (along y the
    offset leaves the hydrostatic variation of the line in the FP32 values),
    with the RK4 update as its own kernel on the FP32 R: the change of every
    field over 4 RK4 steps against the oracle, within MIXED_CHANGE_BOUND."""
    p = dict(inputs.AIR)
    Q0 = inputs.rti_state(48, seed=7, noise_K=1.0)
    G = _gpu_rk(p, Q0, 1, 1e-5, 4, nopcs.MIXED)
    O = oracle.rk4(p, Q0, 1e-5, 4)
    errs = [_rel(G[c] - Q0[c], O[c] - Q0[c]) for c in range(5)]
    print("48^3 one segment (pencils), mixed vs oracle (change)", ["%.2e" % e for e in errs], flush=True)
    assert np.isfinite(G).all()
    assert max(errs) <= MIXED_CHANGE_BOUND and max(errs) > 0.0


@pytest.mark.parametrize("shape, nseg", [((40, 36, 70), (2, 3, 2)), ((48, 48, 48), (1, 1, 1))])
def test_rk_mixed_uniform_rest_is_steady(shape, nseg):
    """A uniform state at rest without gravity is a steady solution, and in
    mixed precision every derivative of a uniform field must vanish exactly:
    the FP32 x sweep and pencils stage offset fluxes that are exact zeros, the
    y and z runs form (B f)_i from equal FP64 values, the FP32 viscous
    differences subtract equal numbers.  Over 3 RK4 steps the only change is
    the wall energy reset from the extrapolated wall temperature (a few ulps of
    E') and the momentum that drives next to the walls (measured 2.4e-15, the
    same in FP64); density and the interior energy stay bit for bit.  An FP32 rounding of the full fluxes (|E'| ~ 1e4) would show up as
    momentum changes many orders larger."""
    p = dict(inputs.AIR, gravity=0)
    Q0 = inputs.uniform_state(shape, T=1.3, rho=0.83, params=p)
    G = _gpu_rk(p, Q0, nseg, 1e-5, 3, nopcs.MIXED)
    assert np.array_equal(G[0], Q0[0])
    assert np.array_equal(G[4, 1:-1, 1:-1, 1:-1], Q0[4, 1:-1, 1:-1, 1:-1])
    # the wall energy as the kernel forms it from the wall temperature against
    # the generator's E' (measured 5 ulps, 9.1e-12 of 1.16e4)
    assert np.max(np.abs(G[4] - Q0[4])) <= 2e-15 * np.max(np.abs(Q0[4]))
    for c in (1, 2, 3):
        assert np.max(np.abs(G[c])) <= 1e-14, (c, np.max(np.abs(G[c])))
