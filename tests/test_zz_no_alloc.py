"""strassen_gemm_formed_noalloc (fixed device scratch, no allocation) against
strassen_gemm_formed (caller workspace) through the C ABI: the same kernels
on the same sums, so the results are bit-identical; two calls in a row, the
second smaller, so the second reuses scratch the first left behind; a call
beyond the scratch size is refused before anything runs."""
import numpy as np
import pytest
import torch

import oracle
import paper_1808_07984_amd as sg
from parity import make_problem, to_device

pytestmark = pytest.mark.gpu

DT = {"f32": sg.STRASSEN_F32, "bf16": sg.STRASSEN_BF16, "f16": sg.STRASSEN_F16, "bf16x3": sg.STRASSEN_F32}
MODE = {"f32": sg.STRASSEN_MODE_PLAIN, "bf16": sg.STRASSEN_MODE_PLAIN, "f16": sg.STRASSEN_MODE_PLAIN,
        "bf16x3": sg.STRASSEN_MODE_BF16X3}


def _call(fam, dev, alpha, beta, noalloc):
    A, B, C = dev["A"], dev["B"], dev["C"]
    m, k = A.shape
    n = B.shape[1]
    if noalloc:
        rc = sg.strassen_gemm_formed_noalloc(m, n, k, A.data_ptr(), A.stride(0), DT[fam], B.data_ptr(),
                                             B.stride(0), DT[fam], C.data_ptr(), C.stride(0), alpha, beta,
                                             MODE[fam], torch.cuda.current_stream().cuda_stream)
    else:
        need = sg.strassen_formed_workspace_size(m, n, k, DT[fam], MODE[fam])
        ws = torch.empty(max(need, 16), dtype=torch.uint8, device="cuda")
        rc = sg.strassen_gemm_formed(m, n, k, A.data_ptr(), A.stride(0), DT[fam], B.data_ptr(), B.stride(0),
                                     DT[fam], C.data_ptr(), C.stride(0), alpha, beta, MODE[fam],
                                     ws.data_ptr(), need, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return rc


@pytest.mark.parametrize("fam", ["f32", "bf16", "f16", "bf16x3"])
def test_noalloc_matches_workspace_entry_point(fam):
    for (m, n, k) in ((2050, 1790, 2300), (777, 1030, 515)):  # second call smaller
        prob = make_problem(m, n, k, kind="uniform", dtype=fam, c_kind="uniform")
        d1, d2 = to_device(prob), to_device(prob)
        print("noalloc %s m=%d n=%d k=%d" % (fam, m, n, k), flush=True)
        assert _call(fam, d1, 1.25, 0.5, True) == 0
        assert _call(fam, d2, 1.25, 0.5, False) == 0
        assert torch.equal(d1["C"], d2["C"])
    # integers: exact against the oracle
    prob = make_problem(300, 260, 520, kind="integers", dtype=fam, c_kind="integers")
    dev = to_device(prob)
    assert _call(fam, dev, 1.0, 1.0, True) == 0
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(dev["C"].cpu().double().numpy(), want)


def test_noalloc_allocates_nothing_and_refuses_oversize():
    prob = make_problem(1024, 1024, 1024, kind="uniform", dtype="bf16x3", c_kind="uniform")
    dev = to_device(prob)
    assert _call("bf16x3", dev, 1.0, 1.0, True) == 0  # first call on this device: symbol lookup
    free0, _ = torch.cuda.mem_get_info()
    assert _call("bf16x3", dev, 1.0, 1.0, True) == 0
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    # fp32 6144^3 needs 10 * 6144^2 bytes of sums, more than the 256 MiB scratch:
    # refused before anything is read or launched (the pointers are never used)
    C = torch.zeros(4, 4, device="cuda")
    rc = sg.strassen_gemm_formed_noalloc(6144, 6144, 6144, 1 << 20, 6144, sg.STRASSEN_F32, 1 << 40, 6144,
                                         sg.STRASSEN_F32, C.data_ptr(), 6144, 1.0, 1.0,
                                         sg.STRASSEN_MODE_PLAIN, None)
    assert rc == sg.STRASSEN_ERROR_SCRATCH_LIMIT
    assert "scratch" in sg.strassen_error_string(rc)
    assert bool((C == 0).all())
