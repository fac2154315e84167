"""rk_step replayed from a captured HIP graph (nopcs_set_graphs) equals the
directly launched kernels bit for bit, on every replay, with the program's
own eager work and synchronisations between the replays."""
import numpy as np
import pytest

from paper_2203_00879_amd import inputs, nopcs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n, nseg, prec", [(32, 1, nopcs.FP64), (48, 2, nopcs.FP64), (40, 2, nopcs.MIXED)])
def test_graph_replays_equal_direct_launches(n, nseg, prec):
    import torch
    lib = nopcs.lib()
    p = nopcs.make_params(inputs.AIR)
    g = nopcs.make_grid(n, nseg)
    Q0 = inputs.rti_state(n, seed=2, noise_K=0.5)
    dt = 1e-5
    # reference: direct launches, 3 calls of 2 steps
    lib.nopcs_set_graphs(0)
    Qr = torch.from_numpy(Q0).to("cuda")
    wr = nopcs.alloc_workspace(g, prec)
    refs = []
    for _ in range(3):
        nopcs.rk_step(p, g, Qr, dt, 2, wr, precision=prec)
        torch.cuda.synchronize()
        refs.append(Qr.cpu().numpy())
    # graphs: the same calls, eager torch work and syncs in between
    lib.nopcs_set_graphs(1)
    try:
        Qg = torch.from_numpy(Q0).to("cuda")
        wg = nopcs.alloc_workspace(g, prec)
        scratch = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
        for k in range(3):
            nopcs.rk_step(p, g, Qg, dt, 2, wg, precision=prec)
            scratch.add_(1.0)
            torch.cuda.synchronize()
            got = Qg.cpu().numpy()
            print("replay", k, "max diff", float(np.max(np.abs(got - refs[k]))), flush=True)
            assert np.array_equal(got, refs[k])
        assert float(scratch[0]) == 3.0
    finally:
        lib.nopcs_set_graphs(0)
