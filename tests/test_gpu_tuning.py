"""Autotuner of the piece lengths and the viscous z chunk (nopcs_autotune):
leaves the state untouched, picks admissible settings, and the tuned stepping
differs from the default stepping by round-off only (the closure rows are the
same global-row sums; the chunk changes nothing)."""
import numpy as np
import pytest

from paper_2203_00879_amd import inputs, nopcs

pytestmark = pytest.mark.gpu


def test_autotune_keeps_state_and_results():
    import torch
    p = nopcs.make_params(inputs.AIR)
    n = 96
    g = nopcs.make_grid(n, 2)
    Q0 = inputs.smooth_state(n, seed=8)
    try:
        ws = nopcs.alloc_workspace(g)
        ref = torch.from_numpy(Q0).to("cuda")
        nopcs.rk_step(p, g, ref, 1e-5, 3, ws)
        Q = torch.from_numpy(Q0).to("cuda")
        chosen = nopcs.autotune(p, g, Q, ws)
        torch.cuda.synchronize()
        print("chosen piece lengths", chosen, flush=True)
        assert np.array_equal(Q.cpu().numpy(), Q0)
        assert all(c in (16, 24, 32) for c in chosen)
        assert nopcs.visc_chunk(g) in (16, 32, 64)   # 128 exceeds nz = 96: capped, the same as one chunk
        ws2 = nopcs.alloc_workspace(g)
        nopcs.rk_step(p, g, Q, 1e-5, 3, ws2)
        torch.cuda.synchronize()
        a, b = Q.cpu().numpy(), ref.cpu().numpy()
        for c in range(5):
            s = np.max(np.abs(b[c] - Q0[c])) or 1.0
            assert np.max(np.abs(a[c] - b[c])) / s <= 1e-10, c
    finally:
        for d in range(3):
            nopcs.set_piece_length(d, -1)
        nopcs.set_visc_chunk(0)


@pytest.mark.parametrize("prec", [nopcs.FP64, nopcs.MIXED])
def test_visc_chunk_does_not_change_results(prec):
    """Three RK4 steps of a 40 x 36 x 100 box with the viscous kernel's z chunk
    at 8, the default (16 here) and 128 planes: bit for bit the same state."""
    import torch
    p = nopcs.make_params(inputs.AIR)
    g = nopcs.make_grid((40, 36, 100), (2, 1, 3))
    Q0 = inputs.smooth_state((40, 36, 100), seed=3)
    out = []
    try:
        for zc in (8, 0, 128):
            nopcs.set_visc_chunk(zc)
            Q = torch.from_numpy(Q0).to("cuda")
            nopcs.rk_step(p, g, Q, 1e-5, 3, nopcs.alloc_workspace(g, prec), precision=prec)
            torch.cuda.synchronize()
            out.append(Q.cpu().numpy())
    finally:
        nopcs.set_visc_chunk(0)
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[1], out[2])
