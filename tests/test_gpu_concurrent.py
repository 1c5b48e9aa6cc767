"""Concurrent schedule (element-wise atomic update, Task Parallelism
section): beta applied first, products of mixed variants launched together,
outputs added with fp32 atomics.  Integer inputs stay exact (sums of
integers below 2^24 are exact in any order); reals within tau_L; two runs
agree within the tolerance (not bitwise: atomic order varies)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1808_07984_amd as sg
from parity import EPS, e_norm, make_problem, stratified_entries, tau, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def concurrent():
    assert sg.strassen_set_schedule(sg.STRASSEN_SCHEDULE_CONCURRENT) == 0
    yield
    sg.strassen_set_schedule(sg.STRASSEN_SCHEDULE_BATCHED)


@pytest.fixture
def tile_mode(request):
    assert sg.strassen_set_tile(request.param) == 0
    yield request.param
    sg.strassen_set_tile(sg.STRASSEN_TILE_AUTO)


def _run(prob, levels, alpha, beta):
    dev = to_device(prob)
    print("concurrent m=%d n=%d k=%d L=%d" % (prob["A"].shape[0], prob["B"].shape[1],
                                              prob["A"].shape[1], levels), flush=True)
    sg.gemm(dev["A"], dev["B"], dev["C"], alpha, beta, levels=levels)
    torch.cuda.synchronize()
    return dev


@pytest.mark.parametrize("tile_mode", [sg.STRASSEN_TILE_128, sg.STRASSEN_TILE_256], indirect=True)
@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (3, 5, 7), (65, 67, 63), (301, 257, 190),
                                   (520, 700, 333)])
def test_concurrent_integer_exact(tile_mode, levels, m, n, k):
    prob = make_problem(m, n, k, kind="integers", c_kind="integers")
    dev = _run(prob, levels, 1.0, 1.0)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(dev["C"].cpu().double().numpy(), want)


@pytest.mark.parametrize("levels", [1, 2])
def test_concurrent_padded_alpha_beta(levels):
    m, n, k = 375, 501, 313
    prob = make_problem(m, n, k, kind="integers", c_kind="integers", lda=k + 11, ldb=n + 9,
                        ldc=n + 7)
    dev = _run(prob, levels, 1.5, 0.5)
    assert np.array_equal(dev["C"].cpu().double().numpy(),
                          oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.5, 0.5))
    assert torch.isnan(dev["C_storage"][:, n:]).all()


@pytest.mark.parametrize("levels", [1, 2])
def test_concurrent_beta_zero_ignores_nan(levels):
    prob = make_problem(130, 70, 90, kind="integers", c_kind="zeros")
    prob["C"] = torch.full((130, 70), float("nan"))
    dev = _run(prob, levels, 1.0, 0.0)
    assert np.array_equal(dev["C"].cpu().double().numpy(), oracle.gemm_f64(prob["A"], prob["B"]))


@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("m,n,k", [(1024, 1024, 1024), (2048, 1536, 1000)])
def test_concurrent_float_within_tolerance_and_repeatable(levels, m, n, k):
    prob = make_problem(m, n, k, kind="uniform", c_kind="uniform")
    d1 = _run(prob, levels, 1.0, 1.0)
    d2 = _run(prob, levels, 1.0, 1.0)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    for d in (d1, d2):
        en = e_norm(d["C"].cpu().double().numpy(), want, prob["A"], prob["B"], prob["C"], k, 1.0,
                    1.0, EPS["f32"])
        print("e_norm %.4f" % en, flush=True)
        assert en <= tau(levels)


def test_concurrent_matches_batched_on_integers_large():
    """Both schedules give the exact product on an integer workload large
    enough for 256x256 tiles: stratified entries (every tile of every C
    block, corners, whole accumulator blocks) equal the oracle's, and the two
    schedules agree everywhere."""
    prob = make_problem(4096, 4096, 2048, kind="integers", c_kind="integers", int_range=(-1, 1))
    dev = _run(prob, 2, 1.0, 1.0)
    rows, cols = stratified_entries(4096, 4096, 2, 11)
    want = oracle.gemm_entries(prob["A"], prob["B"], prob["C"], rows, cols, 1.0, 1.0)
    got = dev["C"][torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")]
    assert np.array_equal(got.cpu().double().numpy(), want)
    sg.strassen_set_schedule(sg.STRASSEN_SCHEDULE_BATCHED)
    d2 = to_device(prob)
    sg.gemm(d2["A"], d2["B"], d2["C"], 1.0, 1.0, levels=2)
    torch.cuda.synchronize()
    assert torch.equal(dev["C"], d2["C"])
