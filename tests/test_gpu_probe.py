"""The MFMA rate probe (measurement support, strassen_probe_mfma) computes
what it claims: with constant operands 0.25 every MFMA adds k * 0.0625 to
each of the 16 accumulator elements of each of a lane's four accumulators
(k = 16 for the 16-bit 32x32x16 forms, 2 for the fp32 32x32x2 form), so each
thread writes 64 * iters * k * 0.0625."""
import pytest
import torch

import paper_1808_07984_amd as sg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("op,k", [(0, 16), (1, 16), (2, 2)])
def test_probe_constant_operands(op, k):
    wgs, iters = 3, 37
    out = torch.full((wgs * 256,), float("nan"), device="cuda")
    print("probe op=%d iters=%d workgroups=%d" % (op, iters, wgs), flush=True)
    assert sg.strassen_probe_mfma(op, 0, iters, wgs, out.data_ptr(), None) == 0
    torch.cuda.synchronize()
    assert torch.all(out == 64.0 * iters * k * 0.0625)


def test_probe_random_operands_finite():
    out = torch.full((2 * 256,), float("nan"), device="cuda")
    assert sg.strassen_probe_mfma(0, 1, 11, 2, out.data_ptr(), None) == 0
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
    assert float(out.abs().max()) > 0.0
