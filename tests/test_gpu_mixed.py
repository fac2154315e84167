"""Mixed precision (NOPCS_MIXED) on the GPU: FP32 eliminations along y and z
and an FP32 RHS register, FP64 everything else.

Error budget: each FP32 run sees (B f)_i rounded once (unit roundoff 6e-8)
and amplifies it by at most the row sum of |A^-1| (< 4.4), so the right-hand
side is within about 3e-7 of each component's maximum; the RHS register in FP32
adds one more rounding.  The tolerances below give a factor of 3-30 over that."""
import numpy as np
import pytest

import oracle
from paper_2203_00879_amd import inputs, nopcs

pytestmark = pytest.mark.gpu


def _rel(a, b):
    s = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (s if s > 0 else 1.0)


@pytest.mark.parametrize("shape, nseg", [((40, 130, 97), (1, 3, 2)), ((64, 64, 64), (2, 2, 2))])
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


def test_rk_mixed_against_fp64():
    """RTI box 64^3, 4 segments, 10 steps: the change of every field over the run
    in mixed precision against FP64 on the GPU (itself checked against the oracle)."""
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
    d64, d32 = out[nopcs.FP64] - Q0, out[nopcs.MIXED] - Q0
    errs = [_rel(d32[c], d64[c]) for c in range(5)]
    print("mixed vs FP64, change over 10 steps, relative max errors", ["%.2e" % e for e in errs], flush=True)
    assert np.isfinite(out[nopcs.MIXED]).all()
    assert max(errs) <= 1e-4
