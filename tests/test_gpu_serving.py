"""Serving runtime on the GPU (solver_create / submit / poll / destroy), each
request on its own stream (batched chunks: skipped, see BATCHED).

Parity here is with the library's own single-box path: a request served in a
mix of boxes must equal the same box advanced alone by rk_step, bit for bit
(rk_step itself is checked against the oracle in test_gpu_parity)."""
import numpy as np
import pytest

import oracle
from paper_2203_00879_amd import inputs, nopcs

pytestmark = pytest.mark.gpu

# Batched serving (solver_config.batched = 1) is switched off on the GPU: a
# stream of 256 boxes ended in a segmentation fault in a non-Python thread,
# twice, without an explained cause.  Its cases stay here, skipped; the CPU
# build of the kernels runs batched serving under AddressSanitizer.
BATCHED = [False, pytest.param(True, marks=pytest.mark.skip(
    reason="batched serving switched off on the GPU: unexplained host segfault in a 256-box stream"))]


def _alone(params, grid, Q0, steps, dt, precision=nopcs.FP64):
    import torch
    Q = torch.from_numpy(Q0).to("cuda")
    ws = nopcs.alloc_workspace(grid, precision)
    nopcs.rk_step(params, grid, Q, dt, steps, ws, precision=precision)
    torch.cuda.synchronize()
    return Q.cpu().numpy()


def _wait(S, rid):
    import time
    while True:
        rc, res, Q = S.poll(rid)
        if rc != nopcs.NOPCS_EAGAIN:
            return rc, res, Q
        time.sleep(0.002)


BOXES = [(32, 1, 7, 0), (48, 1, 5, 1), (64, 2, 9, 2), (40, 2, 6, 3), (72, 1, 4, 4)]


@pytest.mark.parametrize("batched", BATCHED)
def test_mix_equals_alone_bitwise(batched):
    params = nopcs.make_params(inputs.AIR)
    dt = 1e-5
    work = []
    for n, nseg, steps, seed in BOXES:
        Q0 = inputs.rti_state(n, seed=seed, T_lower=420.0)
        g = nopcs.make_grid(n, nseg)
        work.append((g, Q0, steps, _alone(params, g, Q0, steps, dt)))
    with nopcs.Solver(16 << 30, max_slots=3, max_queue=16, batched=batched) as S:
        ids = [S.submit(params, g, Q0, steps, dt) for g, Q0, steps, _ in work]
        for rid, (g, Q0, steps, ref) in zip(ids, work):
            rc, res, Q = _wait(S, rid)
            print("request", rid, "status", rc, "steps", res.steps_done, flush=True)
            assert rc == nopcs.NOPCS_OK and res.steps_done == steps
            assert np.array_equal(Q, ref)
            assert res.t_submit <= res.t_admit <= res.t_done
            if g.n[0] == 72:
                # the 72^3 box (one segment cut into pieces, 4 steps) against the FP64 oracle
                O = oracle.rk4(inputs.AIR, Q0, dt, steps)
                for c in range(5):
                    err = float(np.max(np.abs(Q[c] - O[c])))
                    print("  oracle field", c, "err %.3e of the field, %.3e of its change"
                          % (err / np.max(np.abs(O[c])), err / np.max(np.abs(O[c] - Q0[c]))), flush=True)
                    assert err <= 1e-12 * np.max(np.abs(O[c])) and err <= 1e-12 * np.max(np.abs(O[c] - Q0[c]))


@pytest.mark.parametrize("batched", BATCHED)
def test_mixed_precision_requests_equal_alone_bitwise(batched):
    """Mixed-precision requests (FP32 eliminations and RHS register) served beside
    FP64 ones: each equals its box advanced alone by rk_step in its precision."""
    params = nopcs.make_params(inputs.AIR)
    dt = 1e-5
    work = []
    for n, nseg, steps, seed, prec in [(48, 1, 5, 7, nopcs.MIXED), (72, 1, 4, 8, nopcs.FP64),
                                        (96, 2, 3, 9, nopcs.MIXED)]:
        Q0 = inputs.rti_state(n, seed=seed, T_lower=420.0)
        g = nopcs.make_grid(n, nseg)
        work.append((g, Q0, steps, prec, _alone(params, g, Q0, steps, dt, prec)))
    with nopcs.Solver(16 << 30, max_slots=3, max_queue=8, batched=batched) as S:
        ids = [S.submit(params, g, Q0, steps, dt, precision=prec) for g, Q0, steps, prec, _ in work]
        for rid, (g, Q0, steps, prec, ref) in zip(ids, work):
            rc, res, Q = _wait(S, rid)
            print("request", rid, "precision", prec, "status", rc, flush=True)
            assert rc == nopcs.NOPCS_OK and res.steps_done == steps
            assert np.array_equal(Q, ref)


@pytest.mark.parametrize("batched", BATCHED)
def test_admission_order_and_budget(batched):
    params = nopcs.make_params(inputs.AIR)
    g = nopcs.make_grid(32, 1)
    fp = nopcs.workspace_bytes(g) + 5 * 32 ** 3 * 8
    with nopcs.Solver(fp + 1024, max_slots=4, max_queue=8, batched=batched) as S:
        ids = [S.submit(params, g, inputs.rti_state(32, seed=s), 3, 1e-5) for s in range(3)]
        res = [_wait(S, i)[1] for i in ids]
        for a, b in zip(res, res[1:]):
            assert a.t_done <= b.t_admit      # one box at a time, in arrival order
        with pytest.raises(nopcs.NopcsError) as e:
            S.submit(params, nopcs.make_grid(64, 1), inputs.rti_state(64), 1, 1e-5)
        assert e.value.code == nopcs.NOPCS_ENOMEM
        with pytest.raises(nopcs.NopcsError) as e:
            S.poll(123456789)
        assert e.value.code == nopcs.NOPCS_ENOTFOUND


@pytest.mark.parametrize("batched", BATCHED)
def test_nonfinite_request_flagged_others_unaffected(batched):
    params = nopcs.make_params(inputs.AIR)
    g = nopcs.make_grid(32, 1)
    good = inputs.rti_state(32, seed=5)
    bad = good.copy()
    bad[4, 3, 4, 5] = np.inf
    ref = _alone(params, g, good, 3, 1e-5)
    with nopcs.Solver(8 << 30, max_slots=2, max_queue=8, batched=batched) as S:
        ib = S.submit(params, g, bad, 3, 1e-5)
        ig = S.submit(params, g, good, 3, 1e-5)
        assert _wait(S, ib)[0] == nopcs.NOPCS_ENONFINITE
        rc, _, Q = _wait(S, ig)
        assert rc == nopcs.NOPCS_OK and np.array_equal(Q, ref)


@pytest.mark.parametrize("batched", BATCHED)
def test_serving_bench_small_stream(batched):
    from paper_2203_00879_amd import serve_bench
    out = serve_bench.run(n_req=12, step_scale=0.02, slots=4, budget_gb=40.0, check=3, batched=batched)
    print(out, flush=True)
    assert out["all_ok"] and out["mix_equals_alone"]
    assert 0 < out["p50_latency_s"] <= out["p99_latency_s"]


def test_batched_serving_refused_on_the_gpu():
    with pytest.raises(nopcs.NopcsError) as e:
        nopcs.Solver(1 << 30, max_slots=2, max_queue=4, batched=True)
    assert e.value.code == nopcs.NOPCS_EINVAL
