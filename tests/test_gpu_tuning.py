"""Autotuner of the piece lengths (nopcs_autotune): leaves the state untouched,
picks admissible lengths, and the tuned stepping differs from the default
stepping by round-off only (the closure rows are the same global-row sums)."""
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
