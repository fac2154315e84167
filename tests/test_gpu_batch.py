"""GPU: RK4 stepping of a batch of uneven boxes (rk_step_batch: one launch per
stage kernel over all boxes, as a graph or issued directly, one graph branch
per box, or branches for large boxes beside shared launches for small ones)
gives every box exactly the result of rk_step on it alone."""
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
P = dict(inputs.AIR)
BOXES = [((32, 32, 32), (1, 1, 1), 0), ((48, 40, 36), (2, 1, 3), 1), ((24, 64, 28), (1, 2, 1), 2),
         ((80, 20, 72), (2, 1, 2), 3)]
BIG = ((132, 128, 128), (2, 2, 2), 5)   # 2^21 points or more: a branch of its own in the default mode


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make(shape, nseg, seed, prec):
    g = nopcs.make_grid(shape, nseg)
    Q = torch.from_numpy(inputs.rti_state(shape, seed=seed, noise_K=1e-3)).to(DEV)
    return g, Q, nopcs.alloc_workspace(g, prec)


def lone(shape, nseg, seed, prec, dt, nsteps):
    g, Q, ws = make(shape, nseg, seed, prec)
    nopcs.rk_step(nopcs.make_params(P), g, Q, dt, nsteps, ws, precision=prec)
    torch.cuda.synchronize()
    return Q.cpu().numpy()


@pytest.fixture
def batch_mode(request):
    nopcs.set_batch_mode(request.param)
    yield request.param
    nopcs.set_batch_mode(3)


@pytest.mark.parametrize("batch_mode", [0, 1, 2, 3], indirect=True)
@pytest.mark.parametrize("prec", [nopcs.FP64, nopcs.MIXED])
def test_batch_equals_lone_runs_bitwise_over_replays(prec, batch_mode):
    """Four uneven boxes, a fifth of the second's shape (so launches hold
    several boxes of one configuration) with its own dt, and a large sixth,
    2 + 1 + 1 steps in three calls (the step is captured or collected on the
    first and replayed after), with unrelated eager work in between."""
    say("batch of", len(BOXES) + 2, "precision", prec, "mode", batch_mode)
    dt, dt5 = 1e-5, 2.5e-5
    nopcs.lib().nopcs_set_graphs(0)
    specs = BOXES + [(BOXES[1][0], BOXES[1][1], 9), BIG]
    dts = [dt] * len(BOXES) + [dt5, dt]
    want = [lone(s, n, seed, prec, d, 4) for (s, n, seed), d in zip(specs, dts)]
    boxes = [make(s, n, seed, prec) for s, n, seed in specs]
    boxes[4] = boxes[4] + (dt5,)
    prm = nopcs.make_params(P)
    junk = torch.ones(1 << 20, dtype=torch.float64, device=DEV)
    for k in (2, 1, 1):
        nopcs.rk_step_batch(prm, boxes, dt, k, precision=prec)
        junk.mul_(1.5).add_(1.0)
        torch.cuda.synchronize()
    for box, w, (shape, _, _) in zip(boxes, want, specs):
        got = box[1].cpu().numpy()
        say("  box", shape, "max diff", float(np.max(np.abs(got - w))))
        assert np.array_equal(got, w)


def test_batch_single_box_equals_rk_step():
    g, Q, ws = make((40, 36, 44), (2, 3, 2), 7, nopcs.FP64)
    nopcs.rk_step_batch(nopcs.make_params(P), [(g, Q, ws)], 1e-5, 3)
    torch.cuda.synchronize()
    assert np.array_equal(Q.cpu().numpy(), lone((40, 36, 44), (2, 3, 2), 7, nopcs.FP64, 1e-5, 3))


def test_batch_box_against_oracle():
    """A box stepped inside a batch against the FP64 oracle: the 48 x 40 x 36
    box (2 x 1 x 3 segments) of an FP64 batch, 3 steps, every point of all 5
    fields within 1e-12 of the field's maximum and of its change."""
    dt, steps = 1e-5, 3
    boxes = [make(s, n, seed, nopcs.FP64) for s, n, seed in BOXES]
    nopcs.rk_step_batch(nopcs.make_params(P), boxes, dt, steps)
    torch.cuda.synchronize()
    shape, nseg, seed = BOXES[1]
    Q0 = inputs.rti_state(shape, seed=seed, noise_K=1e-3)
    O = oracle.rk4(P, Q0, dt, steps)
    G = boxes[1][1].cpu().numpy()
    for c in range(5):
        scale = np.max(np.abs(O[c]))
        ch = np.max(np.abs(O[c] - Q0[c]))
        err = float(np.max(np.abs(G[c] - O[c])))
        say("  field", c, "err %.3e of the field, %.3e of its change" % (err / scale, err / ch))
        assert err <= 1e-12 * scale and err <= 1e-12 * ch
