"""nse_rhs_noalloc: nse_rhs with its closure array in the library's static
device scratch array (no allocation), called through the C ABI and compared
with nse_rhs on the same inputs: two calls in a row, the second on a smaller
box, each bit for bit equal to nse_rhs and within 1e-12 of the oracle."""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    s = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (s if s > 0 else 1.0))


def test_noalloc_equals_nse_rhs_on_two_calls():
    p = dict(inputs.AIR)
    prm = nopcs.make_params(p)
    # the larger box first (both sweeps along y and z march with closures), then a smaller one
    for shape, nseg, prec in [((96, 80, 72), (2, 3, 2), nopcs.FP64), ((40, 36, 44), (2, 3, 2), nopcs.FP64),
                              ((64, 72, 80), (1, 2, 2), nopcs.MIXED)]:
        say("noalloc", shape, nseg, "precision", prec)
        Q = inputs.smooth_state(shape, seed=sum(shape))
        g = nopcs.make_grid(shape, nseg)
        Qd = torch.from_numpy(Q).to(DEV)
        Rref = torch.empty_like(Qd)
        nopcs.nse_rhs(prm, g, Qd, Rref, precision=prec)          # builds and caches the plans
        Rna = torch.full_like(Qd, float("nan"))
        nopcs.nse_rhs_noalloc(prm, g, Qd, Rna, precision=prec)
        torch.cuda.synchronize()
        a, b = Rna.cpu().numpy(), Rref.cpu().numpy()
        assert np.array_equal(a, b)
        if prec == nopcs.FP64:
            Ro = oracle.rhs(p, Q)
            errs = [_rel(a[c], Ro[c]) for c in range(5)]
            say("  oracle errors", ["%.2e" % e for e in errs])
            assert max(errs) <= 1e-12


def test_noalloc_errors_before_device_work():
    p = dict(inputs.AIR)
    prm = nopcs.make_params(p)
    # a grid whose plans were never built on this device: refused, nothing launched
    shape = (28, 44, 36)
    Qd = torch.from_numpy(inputs.smooth_state(shape, seed=1)).to(DEV)
    R = torch.zeros_like(Qd)
    with pytest.raises(nopcs.NopcsError) as e:
        nopcs.nse_rhs_noalloc(prm, nopcs.make_grid(shape, (1, 3, 5)), Qd, R)
    assert e.value.code == nopcs.NOPCS_EINVAL and "plan" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(R == 0)
    # a grid whose closure array exceeds the static array: refused with the sizes
    shape = (192, 512, 288)
    g = nopcs.make_grid(shape, 4)
    need = nopcs.workspace_bytes(g) - 3 * ((5 * 192 * 512 * 288 * 8 + 255) // 256 * 256)
    assert need > nopcs.NOALLOC_SCRATCH_BYTES
    Qd = torch.zeros((5, 288, 512, 192), dtype=torch.float64, device=DEV)
    Qd[0] = 1.0
    R = torch.zeros_like(Qd)
    f = torch.zeros((288, 512, 192), dtype=torch.float64, device=DEV)
    d1 = torch.empty_like(f)
    for d in range(3):
        nopcs.nopcs_derivative(g, d, f, d1)                     # caches the plans of this grid
    torch.cuda.synchronize()
    with pytest.raises(nopcs.NopcsError) as e:
        nopcs.nse_rhs_noalloc(prm, g, Qd, R)
    assert e.value.code == nopcs.NOPCS_EINVAL and "static array" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(R == 0)
