"""GPU parity of the stream-by-stage schedule (strassen_set_schedule(
STRASSEN_SCHEDULE_STREAMS), table tab:gpu_streaming of the Task Parallelism
section): one launch per one-level product on two streams, stage barriers.

* integer inputs: exact (every family, ragged sizes, alpha/beta, padding);
* real inputs: within tau_1 of the oracle and reproducible run to run;
* the launches follow the paper's table (product, stage, stream), read from
  the library's own launch records and compared with the golden fixture;
* two-level calls keep the batched schedule.
"""
import re

import numpy as np
import pytest
import torch

import oracle
import paper_1808_07984_amd as sg
from conftest import read_golden
from parity import EPS, e_norm, make_problem, tau, to_device

pytestmark = pytest.mark.gpu

FAMILIES = {"f32": ("f32", "plain"), "bf16": ("bf16", "plain"), "bf16x3": ("bf16x3", "bf16x3")}
GATE_EPS = {"f32": 2.0 ** -23, "bf16": 2.0 ** -7, "bf16x3": 2.0 ** -16}


@pytest.fixture(autouse=True)
def streams():
    assert sg.strassen_set_schedule(sg.STRASSEN_SCHEDULE_STREAMS) == 0
    yield
    sg.strassen_set_schedule(sg.STRASSEN_SCHEDULE_BATCHED)


def _run(prob, levels, alpha, beta, mode):
    dev = to_device(prob)
    print("streams m=%d n=%d k=%d L=%d dtype=%s mode=%s" % (prob["A"].shape[0], prob["B"].shape[1],
                                                           prob["A"].shape[1], levels, prob["A"].dtype, mode),
          flush=True)
    sg.gemm(dev["A"], dev["B"], dev["C"], alpha=alpha, beta=beta, levels=levels, mode=mode)
    torch.cuda.synchronize()
    return dev


@pytest.mark.parametrize("fam", sorted(FAMILIES))
@pytest.mark.parametrize("m,n,k", [(3, 5, 7), (64, 64, 64), (257, 130, 300), (1030, 1100, 1500),
                                   (2048, 2048, 1024)])
def test_streams_integer_exact(fam, m, n, k):
    dtype, mode = FAMILIES[fam]
    prob = make_problem(m, n, k, kind="integers", dtype=dtype, c_kind="integers")
    dev = _run(prob, 1, 1.0, 1.0, mode)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(dev["C"].cpu().double().numpy(), want)


def test_streams_integer_exact_padded_alpha_beta():
    m, n, k = 375, 501, 313
    prob = make_problem(m, n, k, kind="integers", c_kind="integers", lda=k + 11, ldb=n + 9, ldc=n + 7)
    dev = _run(prob, 1, 1.5, 0.5, "plain")
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.5, 0.5)
    assert np.array_equal(dev["C"].cpu().double().numpy(), want)
    assert torch.isnan(dev["C_storage"][:, n:]).all()


@pytest.mark.parametrize("fam", sorted(FAMILIES))
def test_streams_float_and_reproducible(fam):
    dtype, mode = FAMILIES[fam]
    m, n, k = 1500, 1400, 1300
    prob = make_problem(m, n, k, kind="uniform", dtype=dtype, c_kind="uniform")
    d1 = _run(prob, 1, 1.0, 1.0, mode)
    d2 = _run(prob, 1, 1.0, 1.0, mode)
    assert torch.equal(d1["C"], d2["C"])
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    en = e_norm(d1["C"].cpu().numpy(), want, prob["A"], prob["B"], prob["C"], k, 1.0, 1.0, GATE_EPS[fam])
    print("e_norm %.4g" % en, flush=True)
    assert en <= tau(1)


def test_streams_follow_the_paper_table():
    """Launch records (one per product, in launch order) carry the stream;
    the products are identified by their (W_A, W_B, W_C) variant and output
    blocks through strassen_plan_instances, and must be the table's."""
    table = [tuple(map(int, ln.split())) for ln in read_golden("streaming_stages.txt")]  # stage product stream
    m = n = k = 2048
    prob = make_problem(m, n, k, kind="uniform", c_kind="uniform")
    dev = to_device(prob)
    sg.strassen_profile_start()
    sg.gemm(dev["A"], dev["B"], dev["C"], levels=1)
    rc, recs = sg.strassen_profile_stop()
    assert rc == 7
    # the variant of each one-level product M0..M6 (eq. gpu_allops)
    variant = {0: (2, 2, 2), 1: (2, 1, 2), 2: (1, 2, 2), 3: (1, 2, 2), 4: (2, 1, 2), 5: (2, 2, 1), 6: (2, 2, 1)}
    order = sorted(table, key=lambda t: (t[0], t[2]))  # stage, then stream; file order within a stream
    by_stage = {}
    for st, prod, stream in table:
        by_stage.setdefault(st, {}).setdefault(stream, []).append(prod)
    got = []
    for r in recs:
        name = r.kernel.decode()
        mm = re.search(r"<(\d),(\d),(\d),stream (\d)>", name)
        assert mm, name
        got.append((tuple(int(x) for x in mm.groups()[:3]), int(mm.group(4))))
    # launches grouped by stage, streams as the table assigns, variants match
    i = 0
    for st in sorted(by_stage):
        launched = got[i:i + sum(len(v) for v in by_stage[st].values())]
        i += len(launched)
        for stream, prods in by_stage[st].items():
            on = [v for v, s in launched if s == stream]
            assert on == [variant[p] for p in prods], (st, stream, on)
    assert i == 7 and len(order) == 7


def test_streams_two_levels_keep_batched():
    prob = make_problem(300, 260, 520, kind="uniform", c_kind="uniform")
    d1 = _run(prob, 2, 1.0, 1.0, "plain")
    sg.strassen_set_schedule(sg.STRASSEN_SCHEDULE_BATCHED)
    d2 = _run(prob, 2, 1.0, 1.0, "plain")
    assert torch.equal(d1["C"], d2["C"])
