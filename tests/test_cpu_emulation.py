"""The library's HIP kernels built for the host (CPU) and run under
AddressSanitizer/UBSan with guard pages around every device buffer and explicit
LDS index checks (tests/cpu_emul).  Catches out-of-bounds accesses on the CPU
before a kernel reaches the GPU, and checks the kernels' arithmetic against the
oracle.  No GPU needed."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2203_00879_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_00879_amd", "csrc")
EMU = os.path.join(ROOT, "tests", "cpu_emul")
BIN = os.path.join(ROOT, "tests", "cpu_emul", "nopcs_emul")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _sources():
    names = ("api.hip", "sweep.hip", "march.hip", "dmarch.hip", "visc.hip", "cvisc.hip", "diag.hip", "plan.cpp", "solver.cpp")
    return [os.path.join(CSRC, f) for f in names]


@pytest.fixture(scope="module")
def driver():
    deps = _sources() + [os.path.join(EMU, "driver.cpp"), os.path.join(EMU, "include", "hip", "hip_runtime.h")]
    deps += [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    if not os.path.exists(BIN) or os.path.getmtime(BIN) < max(os.path.getmtime(d) for d in deps):
        flags = ["-std=c++20", "-O1", "-g", "-DNOPCS_CPU_EMUL", "-fsanitize=address,undefined",
                 "-fno-omit-frame-pointer", "-fno-strict-aliasing", "-ffp-contract=off", "-pthread",
                 "-I", os.path.join(EMU, "include")]
        # one compiler per translation unit, in parallel, then one link
        srcs = _sources() + [os.path.join(EMU, "driver.cpp")]
        # per-process object and binary names: parallel workers may build at once
        objs = [BIN + ".%d.%d.o" % (os.getpid(), k) for k in range(len(srcs))]
        procs = [subprocess.Popen(["g++"] + flags + ["-x", "c++", "-c", src, "-o", obj]) for src, obj in zip(srcs, objs)]
        assert all(p.wait() == 0 for p in procs), "CPU build of the kernels failed"
        tmp = BIN + ".%d.tmp" % os.getpid()
        subprocess.check_call(["g++"] + flags + objs + ["-o", tmp])
        os.replace(tmp, BIN)
        for obj in objs:
            os.remove(obj)
    return BIN


def _run(driver, args, tmp_path, piece=None, mixed=False, deriv_form=None):
    env = dict(os.environ)
    if piece is not None:
        env["NOPCS_EMUL_PIECE"] = str(piece)
    if deriv_form is not None:
        env["NOPCS_EMUL_DERIV_FORM"] = str(deriv_form)
    if mixed:
        env["NOPCS_EMUL_PRECISION"] = "1"
    r = subprocess.run([driver] + [str(a) for a in args], capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, r.stderr[-4000:]


def _rel(a, b):
    s = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (s if s > 0 else 1.0)


@pytest.mark.parametrize("shape, nseg", [((27, 19, 22), (3, 2, 4)), ((16, 17, 20), (4, 4, 5)),
                                         ((10, 300, 9), (1, 3, 1)), ((9, 8, 520), (1, 1, 4)),
                                         ((1024, 9, 8), (7, 1, 1)), ((8, 1024, 9), (1, 13, 1)),
                                         ((9, 8, 1024), (1, 1, 60))])
def test_emulated_derivative_segmented(driver, tmp_path, shape, nseg):
    """Segmented lines, the second case with 4-point segments (Thomas runs of a
    single unknown, whose first row is also its last); the next two take the
    512-thread pencils of 300-point y lines (16 per block) and 520-point z
    lines (8 per block), with a ragged last pencil; the last three the longest
    lines (1024 points) along x, y and z, the last with 60 segments (118
    closure rows, near the pencil's capacity of 132)."""
    f = np.random.default_rng(1).normal(size=shape[::-1])
    fin, fout = tmp_path / "f.raw", tmp_path / "d.raw"
    f.tofile(fin)
    L = (1.0, 0.8, 1.1)
    for d in range(3):
        _run(driver, ["deriv", *shape, *nseg, *L, d, fin, fout], tmp_path)
        out = np.fromfile(fout).reshape(2, *f.shape)
        assert _rel(out[0], oracle.d1(f, d, L)) <= 1e-12
        assert _rel(out[1], oracle.d2(f, d, L)) <= 1e-12


@pytest.mark.parametrize("shape, nseg", [((27, 19, 22), (3, 2, 4)), ((16, 17, 20), (4, 4, 5)),
                                         ((130, 40, 33), (2, 3, 2)), ((9, 300, 70), (1, 3, 2)),
                                         ((8, 1024, 9), (1, 13, 1)), ((9, 8, 1024), (1, 1, 60))])
def test_emulated_first_derivative_line_march(driver, tmp_path, shape, nseg):
    """The first derivative alone with the line march asked for: along y and z
    the closure pass and line march (one thread per line, 128 lines per block:
    the third case has a ragged second x chunk), along x and with too many
    closure slots per row (the last case, 60 segments) the pencil solve; each
    within 1e-12 of the oracle and within 1e-13 of the pencil solve of the same
    field; an unknown form rejected."""
    f = np.random.default_rng(2).normal(size=shape[::-1])
    fin, fout = tmp_path / "f.raw", tmp_path / "d.raw"
    f.tofile(fin)
    L = (1.0, 0.8, 1.1)
    for d in range(3):
        _run(driver, ["deriv1", *shape, *nseg, *L, d, fin, fout], tmp_path)
        out = np.fromfile(fout).reshape(2, *f.shape)
        ref = oracle.d1(f, d, L)
        assert _rel(out[0], ref) <= 1e-12, d
        assert _rel(out[1], ref) <= 1e-12, d
        assert _rel(out[0], out[1]) <= 1e-13, d


def test_emulated_rhs(driver, tmp_path):
    p = dict(inputs.AIR)
    Q = inputs.smooth_state((20, 18, 22), seed=4)
    qin, rout = tmp_path / "q.raw", tmp_path / "r.raw"
    Q.tofile(qin)
    _run(driver, ["rhs", 20, 18, 22, 2, 1, 3, 1.0, 1.0, 1.0, 1, 1, qin, rout], tmp_path)
    R = np.fromfile(rout).reshape(Q.shape)
    Ro = oracle.rhs(p, Q)
    for c in range(5):
        assert _rel(R[c], Ro[c]) <= 1e-12


def test_emulated_rk_step_matches_oracle(driver, tmp_path):
    """One segment per direction: the kernels follow the oracle's operation order
    except in the Thomas elimination, which multiplies by reciprocal pivots
    (one rounding per row apart from the oracle's division)."""
    p = dict(inputs.AIR)
    Q = inputs.rti_state(16, seed=0)
    qin, qout = tmp_path / "q.raw", tmp_path / "o.raw"
    Q.tofile(qin)
    _run(driver, ["rk", 16, 16, 16, 1, 1, 1, 1.0, 1.0, 1.0, 1, 1, 2e-5, 2, qin, qout], tmp_path)
    G = np.fromfile(qout).reshape(Q.shape)
    O = oracle.rk4(p, Q, 2e-5, 2)
    assert np.array_equal(G[0], O[0])          # continuity: fluxes rho u_j, no elimination order
    for c in range(1, 5):
        assert _rel(G[c], O[c]) <= 1e-12


def test_emulated_rk_rti_32_config(driver, tmp_path):
    """The 32^3 Rayleigh-Taylor configuration exactly as the GPU case would run
    it: one segment per direction, 20 RK4 steps at dt = 1e-5, every point of all
    5 fields against the oracle (device buffers end flush with a guard page and
    every plan table sits in an allocation of its own)."""
    p = dict(inputs.AIR)
    Q = inputs.rti_state(32, seed=0)
    qin, qout = tmp_path / "q.raw", tmp_path / "o.raw"
    Q.tofile(qin)
    _run(driver, ["rk", 32, 32, 32, 1, 1, 1, 1.0, 1.0, 1.0, 1, 1, 1e-5, 20, qin, qout], tmp_path)
    G = np.fromfile(qout).reshape(Q.shape)
    O = oracle.rk4(p, Q, 1e-5, 20)
    assert np.array_equal(G[0], O[0])
    for c in range(5):
        ch = np.max(np.abs(O[c] - Q[c]))
        assert _rel(G[c], O[c]) <= 1e-12
        assert np.max(np.abs(G[c] - O[c])) <= 1e-12 * ch


@pytest.mark.parametrize("mixed", [False, True])
def test_emulated_rk_line_march(driver, tmp_path, mixed):
    """One RK4 step of a box whose y and z lines are cut into pieces (line
    marches; the stage update rides on the z march: in FP64 the stage state is
    written over R, so the two state buffers swap roles every stage; in mixed
    precision it alternates between two FP64 stage buffers), against the
    oracle's RK4 with global line solves.  The state change over the run is
    compared, relative to its largest value per field."""
    p = dict(inputs.AIR)
    shape = (8, 20, 44)
    Q = inputs.smooth_state(shape, seed=41)
    qin, qout = tmp_path / "q.raw", tmp_path / "o.raw"
    Q.tofile(qin)
    dt, steps = 5e-5, 1
    _run(driver, ["rk", *shape, 1, 2, 2, 1.0, 1.0, 1.0, 1, 1, dt, steps, qin, qout], tmp_path, piece=16, mixed=mixed)
    G = np.fromfile(qout).reshape(Q.shape)
    O = oracle.rk4(p, Q, dt, steps)
    tol = 1e-6 if mixed else 1e-11
    for c in range(5):
        d = np.max(np.abs(O[c] - Q[c]))
        assert np.max(np.abs(G[c] - O[c])) <= tol * d, (c, np.max(np.abs(G[c] - O[c])) / d)


@pytest.mark.parametrize("shape, v, g, chunk", [((60, 30, 20), 1, 1, 0), ((30, 14, 131), 1, 0, 0),
                                                ((30, 20, 41), 1, 1, 8)])
def test_emulated_rhs_tiles(driver, tmp_path, shape, v, g, chunk):
    """No extra cuts and one segment per direction: interior tiles (no wall
    inside the halo), wall tiles, shifted edge tiles and several z chunks of
    the viscous kernel (the last case: 8-plane chunks, the top one partial)
    all reproduce the oracle to rounding (the viscous terms and fluxes in the
    oracle's operation order, the Thomas elimination with reciprocal pivots)."""
    p = dict(inputs.AIR, viscous=v, gravity=g)
    Q = inputs.smooth_state(shape, seed=11)
    qin, rout = tmp_path / "q.raw", tmp_path / "r.raw"
    Q.tofile(qin)
    L = (1.0, 0.6, 1.4)
    os.environ["NOPCS_EMUL_VISC_CHUNK"] = str(chunk)
    try:
        _run(driver, ["rhs", *shape, 1, 1, 1, *L, v, g, qin, rout], tmp_path, piece=0)
    finally:
        del os.environ["NOPCS_EMUL_VISC_CHUNK"]
    R = np.fromfile(rout).reshape(Q.shape)
    Ro = oracle.rhs(p, Q, L)
    for c in range(5):
        assert _rel(R[c], Ro[c]) <= 4e-15


@pytest.mark.parametrize("shape, nseg, piece", [((8, 36, 100), (1, 2, 3), 16), ((8, 20, 200), (1, 1, 2), -1),
                                                ((1024, 9, 8), (5, 1, 1), -1), ((8, 1024, 9), (1, 7, 1), -1)])
def test_emulated_rhs_line_march_with_closures(driver, tmp_path, shape, nseg, piece):
    """Lines along y and z long enough to be cut into pieces: the line-march
    sweeps (closure pass with 16 or 8 accumulator slots, run march with one or
    several run groups per line) against the oracle's global solve."""
    p = dict(inputs.AIR)
    Q = inputs.smooth_state(shape, seed=21)
    qin, rout = tmp_path / "q.raw", tmp_path / "r.raw"
    Q.tofile(qin)
    L = (0.7, 1.3, 1.0)
    _run(driver, ["rhs", *shape, *nseg, *L, 1, 1, qin, rout], tmp_path, piece=piece)
    R = np.fromfile(rout).reshape(Q.shape)
    Ro = oracle.rhs(p, Q, L)
    for c in range(5):
        assert _rel(R[c], Ro[c]) <= 1e-13, c


@pytest.mark.parametrize("mode", ["serve", "serve_batched"])
def test_emulated_serving_runtime(driver, tmp_path, mode):
    """Serving runtime on 8^3 boxes, each request on its own stream or all
    resident requests in batched chunks: results in a mix equal each box run
    alone bit for bit, arrival-order admission under a one-box budget, a
    non-finite box flagged, EBUSY / ENOMEM / ENOTFOUND / EINVAL, destroy with
    pending work."""
    r = subprocess.run([driver, mode], capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ok mix equals alone bit for bit" in r.stdout
    assert "ok stream of 8 equals alone bit for bit" in r.stdout


@pytest.mark.parametrize("mixed", [False, True])
def test_emulated_batch_step(driver, tmp_path, mixed):
    """rk_step_batch over five uneven boxes (two of one shape sharing every
    launch, one taking the call's dt, the others their own), in every mode in
    FP64 (shared launches as a graph or issued directly, a graph branch per
    box, the hybrid) and in the direct and the default mode in mixed precision:
    each box bit-identical to rk_step on it alone, on the first call and on the
    cached second; grids that differ only in their padding bytes reuse the
    cached batch and lone graph steps; 8 distinct two-box batches through a
    step cache limited to 3 entries, each against the lone steps; duplicate states, misaligned
    workspaces, negative dt and an empty batch rejected."""
    env = dict(os.environ)
    if mixed:
        env["NOPCS_EMUL_PRECISION"] = "1"
    modes = (2, 3) if mixed else (2, 0, 1, 3)   # mixed precision: the direct and the default mode
    r = subprocess.run([driver, "batch", "".join(map(str, modes))], capture_output=True, text=True, timeout=900,
                       env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    for mode in modes:
        assert "ok batch mode %d call 1: 5 boxes bit-identical to their lone steps" % mode in r.stdout
    assert "ok grids differing in padding only reuse the cached steps" in r.stdout
    assert "ok 8 distinct batches through the cache" in r.stdout
    assert "ok batch argument errors" in r.stdout


def test_emulated_rhs_mixed_precision(driver, tmp_path):
    """nse_rhs in mixed precision (FP32 eliminations along y and z; its R is
    the caller's FP64 array, so the x sweep and viscous terms stay FP64)
    against the oracle's FP64 right-hand side.  Error budget: the FP32 runs
    see (B f)_i rounded once (relative 6e-8) and amplify it by at most the row
    sum of |A^-1| (< 4.4); the RHS error stays below 1e-6 of each component's
    maximum (measured 2.4e-7)."""
    p = dict(inputs.AIR)
    shape = (12, 40, 70)
    Q = inputs.smooth_state(shape, seed=31)
    qin, rout = tmp_path / "q.raw", tmp_path / "r.raw"
    Q.tofile(qin)
    _run(driver, ["rhs", *shape, 1, 2, 2, 1.0, 1.0, 1.0, 1, 1, qin, rout], tmp_path, mixed=True)
    R = np.fromfile(rout).reshape(Q.shape)
    Ro = oracle.rhs(p, Q)
    errs = [_rel(R[c], Ro[c]) for c in range(5)]
    print("mixed rhs rel errors", errs)
    assert max(errs) <= 1e-6
    assert max(errs) > 0.0     # the FP32 path really ran


def test_emulated_rhs_mixed_uniform_motion(driver, tmp_path):
    """nse_rhs in mixed precision on a uniform state in uniform motion: every
    derivative vanishes exactly ((B f)_i and the closure and wall rows of the
    FP32 y and z runs formed from equal FP64 values), so rho, rho u, rho w are
    exactly zero and the gravity source components within one FP32 rounding of
    the oracle's closed form."""
    p = dict(inputs.AIR)
    shape = (12, 40, 70)
    Q = inputs.uniform_state(shape, T=1.3, rho=0.83, velocity=(0.31, -0.47, 0.19), params=p)
    qin, rout = tmp_path / "q.raw", tmp_path / "r.raw"
    Q.tofile(qin)
    _run(driver, ["rhs", *shape, 1, 2, 2, 1.0, 1.0, 1.0, 1, 1, qin, rout], tmp_path, mixed=True)
    R = np.fromfile(rout).reshape(Q.shape)
    Ro = oracle.rhs(p, Q)
    for c in (0, 1, 3):
        assert np.all(R[c] == 0.0), c
    for c in (2, 4):
        s = np.max(np.abs(Ro[c]))
        assert np.max(np.abs(R[c] - Ro[c])) <= 2.0 ** -23 * s, c


@pytest.mark.parametrize("form", [0, 2])
def test_emulated_vorticity_budget(driver, tmp_path, form):
    """Vorticity budget of Eq. eqn12_1 on a ragged box with segmented lines and
    unequal lengths, against the oracle's global line solves; first
    derivatives along y and z by the pencil solve (form 0 on this small box)
    and by the line march (form 2)."""
    p = dict(inputs.AIR)
    shape = (18, 13, 16)   # x, y, z
    Q = inputs.smooth_state(shape, seed=6)
    L = (1.0, 0.8, 1.1)
    qin, oout = tmp_path / "q.raw", tmp_path / "o.raw"
    Q.tofile(qin)
    _run(driver, ["vort", *shape, 3, 1, 2, *L, qin, oout], tmp_path, deriv_form=form)
    G = np.fromfile(oout).reshape((12,) + Q.shape[1:])
    O = oracle.vorticity_budget(p, Q, np.array(L))
    for c in range(12):
        assert _rel(G[c], O[c]) <= 1e-12, c


def test_emulated_disturbance_pressure_and_line_spectrum(driver, tmp_path):
    """p - p_h of an RTI box two oracle steps after release, and the amplitude
    spectrum of its vertical centre line (odd length)."""
    p = dict(inputs.AIR)
    shape = (9, 37, 10)   # x, y, z
    Q0 = inputs.rti_state(shape, seed=1, noise_K=1e-3)
    Q = oracle.rk4(p, Q0, 2e-5, 2)
    qin, q0in, dout, aout = (tmp_path / s for s in ("q.raw", "q0.raw", "d.raw", "a.raw"))
    Q.tofile(qin)
    Q0.tofile(q0in)
    _run(driver, ["dpress", *shape, 1, 1, 1, 1.0, 1.0, 1.0, qin, q0in, dout, aout], tmp_path)
    dp = np.fromfile(dout).reshape(Q.shape[1:])
    want = oracle.disturbance_pressure(p, Q, Q0)
    assert _rel(dp, want) <= 1e-12
    amp = np.fromfile(aout)
    # the emulated twiddles use the host libm, so compare at 1e-12 of the largest amplitude
    assert _rel(amp, oracle.line_spectrum(want[shape[2] // 2, :, shape[0] // 2])) <= 1e-12


@pytest.mark.parametrize("form", [0, 2])
def test_emulated_rhs_compact_viscous(driver, tmp_path, form):
    """D1-based viscous variant on a ragged, segmented box with unequal
    lengths; first derivatives along y and z by the pencil solve (form 0) and
    by the line march (form 2)."""
    p = dict(inputs.AIR)
    shape = (17, 14, 19)   # x, y, z
    L = (1.0, 0.9, 1.2)
    Q = inputs.smooth_state(shape, seed=9, length=L)
    qin, rout = tmp_path / "q.raw", tmp_path / "r.raw"
    Q.tofile(qin)
    _run(driver, ["cvisc", *shape, 2, 1, 3, *L, 1, 1, qin, rout], tmp_path, deriv_form=form)
    R = np.fromfile(rout).reshape(Q.shape)
    Ro = oracle.rhs_compact_viscous(p, Q, np.array(L))
    for c in range(5):
        assert _rel(R[c], Ro[c]) <= 1e-12, c


@pytest.mark.parametrize("form", [0, 2])
def test_emulated_rk_step_compact_viscous(driver, tmp_path, form):
    """One RK4 step with the D1-based viscous variant (z line march carrying
    the stage update on an 8 x 10 x 24 box with pieces), against the oracle:
    the fields and their change over the step; first derivatives along y and z
    by the pencil solve (form 0) and by the line march (form 2)."""
    p = dict(inputs.AIR)
    shape = (8, 10, 24)
    Q = inputs.rti_state(shape, seed=2, noise_K=1e-3)
    qin, qout = tmp_path / "q.raw", tmp_path / "o.raw"
    Q.tofile(qin)
    _run(driver, ["cvisc", *shape, 1, 2, 2, 1.0, 1.0, 1.0, 1, 1, qin, qout, "2e-5:1"], tmp_path, piece=16,
         deriv_form=form)
    G = np.fromfile(qout).reshape(Q.shape)
    O = oracle.rk4_compact_viscous(p, Q, 2e-5, 1)
    for c in range(5):
        assert _rel(G[c], O[c]) <= 1e-12, c
        assert _rel(G[c] - Q[c], O[c] - Q[c]) <= 1e-9, c


@pytest.mark.parametrize("shape, nseg, piece", [((27, 19, 22), (3, 2, 4), None), ((9, 130, 10), (1, 3, 1), None),
                                                ((72, 20, 16), (2, 1, 2), 16)])
def test_emulated_filter(driver, tmp_path, shape, nseg, piece):
    """The implicit 3D filter (nopcs_filter) against the oracle's global line
    solves, segmented lines (the second case's 130-point y lines are cut into
    pieces), every point of all 5 fields."""
    p = dict(inputs.AIR)
    Q = inputs.smooth_state(shape, seed=13)
    Q[1:4] += np.random.default_rng(2).normal(scale=1e-3, size=Q[1:4].shape)
    qin, qout = tmp_path / "q.raw", tmp_path / "o.raw"
    Q.tofile(qin)
    _run(driver, ["filter", *shape, *nseg, 1.0, 1.0, 1.0, oracle.FILTER_ALPHA, 0, 0.0, 0, qin, qout], tmp_path,
         piece=piece)
    G = np.fromfile(qout).reshape(Q.shape)
    O = oracle.filter_state(p, Q)
    for c in range(5):
        assert _rel(G[c], O[c]) <= 1e-12


def test_emulated_filtered_stepping(driver, tmp_path):
    """RK4 with the filter after every 2nd step (5 steps: filtered twice) on a
    segmented box in motion, against the oracle, every point of all 5 fields.
    (On a resting RTI box the momentum after a few steps is so small that the
    filter's rounding of rho, ~1e-16 of rho, is 1e-12 of the momentum's
    maximum: that case is checked on rho and E' only.)"""
    p = dict(inputs.AIR)
    shape = (20, 24, 18)
    Q = inputs.smooth_state(shape, seed=6, amp_u=0.02)
    qin, qout = tmp_path / "q.raw", tmp_path / "o.raw"
    Q.tofile(qin)
    _run(driver, ["filter", *shape, 2, 2, 1, 1.0, 1.0, 1.0, oracle.FILTER_ALPHA, 2, 2e-6, 5, qin, qout], tmp_path)
    G = np.fromfile(qout).reshape(Q.shape)
    O = oracle.rk4_filtered(p, Q, 2e-6, 5, every=2)
    for c in range(5):
        assert _rel(G[c], O[c]) <= 1e-12
    Q = inputs.rti_state(shape, seed=6, noise_K=1.0)
    Q.tofile(qin)
    _run(driver, ["filter", *shape, 2, 2, 1, 1.0, 1.0, 1.0, oracle.FILTER_ALPHA, 2, 1e-5, 5, qin, qout], tmp_path)
    G = np.fromfile(qout).reshape(Q.shape)
    O = oracle.rk4_filtered(p, Q, 1e-5, 5, every=2)
    for c in (0, 4):
        assert _rel(G[c], O[c]) <= 1e-12
