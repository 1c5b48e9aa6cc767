"""GPU parity of the 16-bit MFMA path: bf16 and fp16 operands (sums rounded
once to the operand type), and the compensated bf16x3 mode on fp32 operands.

* integer inputs: every operand sum (at most four terms of magnitude <= 3) and
  every bf16 hi/lo split is exact, so the result equals the classical product
  bit for bit;
* real inputs: within tau_L * eps * (k |alpha| |A| |B| + |beta| |C|) of the
  fp64 oracle evaluated on the exact stored operands, eps = 2^-7 (bf16),
  2^-10 (fp16), 2^-16 (bf16x3: hi + lo carries 16 significant bits);
* the compensated mode is far more accurate than plain bf16 on the same data.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1808_07984_amd as sg
from parity import EPS, e_norm, make_problem, stratified_entries, tau, to_device

pytestmark = pytest.mark.gpu

MODES = {"bf16": ("bf16", "plain"), "f16": ("f16", "plain"), "bf16x3": ("bf16x3", "bf16x3")}
GATE_EPS = {"bf16": 2.0 ** -7, "f16": 2.0 ** -10, "bf16x3": 2.0 ** -16}


def _run(prob, levels, alpha, beta, mode):
    dev = to_device(prob)
    print("case m=%d n=%d k=%d L=%d dtype=%s mode=%s" % (
        prob["A"].shape[0], prob["B"].shape[1], prob["A"].shape[1], levels, prob["A"].dtype, mode),
        flush=True)
    sg.gemm(dev["A"], dev["B"], dev["C"], alpha=alpha, beta=beta, levels=levels, mode=mode)
    torch.cuda.synchronize()
    return dev


@pytest.mark.parametrize("kind", sorted(MODES))
@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("m,n,k", [(64, 64, 64), (65, 67, 63), (200, 129, 77), (3, 5, 7),
                                   (257, 130, 300)])
def test_lowp_integer_exact(kind, levels, m, n, k):
    dtype, mode = MODES[kind]
    prob = make_problem(m, n, k, kind="integers", dtype=dtype, c_kind="integers")
    dev = _run(prob, levels, 1.0, 1.0, mode)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(dev["C"].cpu().double().numpy(), want)


@pytest.mark.parametrize("kind", sorted(MODES))
@pytest.mark.parametrize("levels", [0, 1, 2])
def test_lowp_integer_exact_padded_alpha_beta(kind, levels):
    dtype, mode = MODES[kind]
    m, n, k = 375, 501, 313
    prob = make_problem(m, n, k, kind="integers", dtype=dtype, c_kind="integers",
                        lda=k + 11, ldb=n + 9, ldc=n + 7)
    dev = _run(prob, levels, 1.5, 0.5, mode)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.5, 0.5)
    assert np.array_equal(dev["C"].cpu().double().numpy(), want)
    assert torch.isnan(dev["C_storage"][:, n:]).all()


@pytest.mark.parametrize("kind", sorted(MODES))
@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("m,n,k", [(512, 384, 640), (1000, 1100, 900)])
def test_lowp_float_within_tolerance(kind, levels, m, n, k):
    dtype, mode = MODES[kind]
    dist = "uniform" if kind == "bf16x3" else "normal"
    prob = make_problem(m, n, k, kind=dist, dtype=dtype, c_kind="uniform")
    dev = _run(prob, levels, 1.0, 1.0, mode)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    got = dev["C"].cpu().double().numpy()
    en = e_norm(got, want, prob["A"], prob["B"], prob["C"], k, 1.0, 1.0, GATE_EPS[kind])
    en23 = e_norm(got, want, prob["A"], prob["B"], prob["C"], k, 1.0, 1.0, EPS["f32"])
    print("e_norm=%.4f at eps=%g (tau=%g); %.3f at 2^-23" % (en, GATE_EPS[kind], tau(levels), en23),
          flush=True)
    assert en <= tau(levels)


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_bf16x3_far_more_accurate_than_bf16(levels):
    """Same fp32 operands: the compensated mode's error is at least 32x below
    plain bf16 on the bf16-rounded operands."""
    m = n = k = 768
    prob = make_problem(m, n, k, kind="uniform", dtype="bf16x3", c_kind="zeros")
    exact = oracle.gemm_f64(prob["A"], prob["B"])
    d3 = _run(prob, levels, 1.0, 0.0, "bf16x3")
    err3 = np.abs(d3["C"].cpu().double().numpy() - exact).max()
    pb = dict(prob, A=prob["A"].to(torch.bfloat16), B=prob["B"].to(torch.bfloat16))
    db = _run(pb, levels, 1.0, 0.0, "plain")
    errb = np.abs(db["C"].cpu().double().numpy() - exact).max()
    print("err bf16x3 %.3e  bf16 %.3e" % (err3, errb), flush=True)
    assert err3 * 32 <= errb


@pytest.mark.parametrize("kind", ["bf16", "f16"])
@pytest.mark.parametrize("levels", [0, 1, 2])
def test_lowp_scaled_rows_and_columns(kind, levels):
    """Rows of A and columns of B with 2-norms 10^u, u ~ U[-3, 3] (the
    precision workload's scaled variant).  Strassen's error bound is normwise:
    the gate is e_norm <= tau_L.  Without operand sums (L = 0) the error of
    each entry is also within the gate relative to its own row and column
    (componentwise); at L >= 1 a sum mixes rows of different blocks, so only
    the normwise bound is claimed and the row-relative error is reported."""
    from paper_1808_07984_amd import inputs
    dtype = MODES[kind][0]
    tdt = {"bf16": torch.bfloat16, "f16": torch.float16}[kind]
    m = n = k = 1536
    A = inputs.scaled(m, k, inputs.SEED_A, axis=0, dtype=tdt)
    B = inputs.scaled(k, n, inputs.SEED_B, axis=1, dtype=tdt)
    prob = dict(A=A, B=B, C=torch.zeros(m, n), lda=k, ldb=n, ldc=n, fill=float("nan"))
    dev = _run(prob, levels, 1.0, 0.0, "plain")
    want = oracle.gemm_f64(A, B)
    got = dev["C"].cpu().double().numpy()
    en = e_norm(got, want, A, B, None, k, 1.0, 0.0, GATE_EPS[kind])
    ra = np.abs(oracle._f64(A)).max(axis=1)
    cb = np.abs(oracle._f64(B)).max(axis=0)
    comp = np.abs(got - want) / (GATE_EPS[kind] * k * np.outer(ra, cb))
    rel_fro = np.linalg.norm(got - want) / np.linalg.norm(want)
    print("e_norm %.4f  componentwise max %.4f  relative Frobenius %.3e" % (en, comp.max(), rel_fro),
          flush=True)
    assert en <= tau(levels)
    if levels == 0:
        assert comp.max() <= tau(0)


def test_lowp_deterministic():
    prob = make_problem(600, 520, 700, kind="normal", dtype="bf16", c_kind="uniform")
    d1 = _run(prob, 2, 1.0, 1.0, "plain")
    d2 = _run(prob, 2, 1.0, 1.0, "plain")
    assert torch.equal(d1["C"], d2["C"])


@pytest.mark.parametrize("kind,levels", [("bf16", 2), ("f16", 1), ("bf16x3", 2)])
def test_lowp_full_size_sampled(kind, levels):
    """m = n = k = 16384 (the precision configuration's largest size),
    stratified entries (every tile of every C block, block corners, whole
    32 x 32 accumulator blocks) against the classical fp64 definition on the
    stored operands."""
    dtype, mode = MODES[kind]
    N = 16384
    dist = "uniform" if kind == "bf16x3" else "normal"
    prob = make_problem(N, N, N, kind=dist, dtype=dtype, c_kind="zeros")
    dev = _run(prob, levels, 1.0, 0.0, mode)
    rows, cols = stratified_entries(N, N, levels, levels)
    want = oracle.gemm_entries(prob["A"], prob["B"], None, rows, cols, 1.0, 0.0)
    got = dev["C"][torch.as_tensor(rows, device="cuda"),
                   torch.as_tensor(cols, device="cuda")].double().cpu().numpy()
    scale = N * float(prob["A"].float().abs().max()) * float(prob["B"].float().abs().max())
    en = float(np.abs(got - want).max()) / (GATE_EPS[kind] * scale)
    print("sampled e_norm %.4f at eps=%g" % (en, GATE_EPS[kind]), flush=True)
    assert en <= tau(levels)
    assert bool(torch.isfinite(dev["C"]).all())


@pytest.fixture
def tile_mode(request):
    assert sg.strassen_set_tile(request.param) == 0
    yield request.param
    sg.strassen_set_tile(sg.STRASSEN_TILE_AUTO)


@pytest.mark.parametrize("tile_mode", [sg.STRASSEN_TILE_128, sg.STRASSEN_TILE_256], indirect=True)
@pytest.mark.parametrize("kind", sorted(MODES))
@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("m,n,k", [(3, 5, 7), (65, 67, 63), (301, 257, 190), (520, 700, 333),
                                   (1100, 1060, 600), (512, 512, 128), (600, 300, 100), (512, 256, 64)])
def test_lowp_integer_exact_each_tile(tile_mode, kind, levels, m, n, k):
    """Integers exact against the oracle on both tile sizes.  On 256 x 256
    tiles the interior tiles of the bf16 and fp16 single-term products load
    their whole 64-deep k-tiles straight into LDS (at level 0 here): one
    such k-tile without a ragged end (512 x 256 x 64) and with one (600 x
    300 x 100), two without (512^2 x 128) and two or more with one (301 x
    257 x 190 and the larger shapes)."""
    dtype, mode = MODES[kind]
    prob = make_problem(m, n, k, kind="integers", dtype=dtype, c_kind="integers")
    dev = _run(prob, levels, 1.0, 1.0, mode)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(dev["C"].cpu().double().numpy(), want)


@pytest.mark.parametrize("tile_mode", [sg.STRASSEN_TILE_128, sg.STRASSEN_TILE_256], indirect=True)
@pytest.mark.parametrize("ta,tb", [(0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("aligned", [False, True])
def test_bf16x3_transposed_integer_exact(tile_mode, ta, tb, levels, aligned):
    from paper_1808_07984_amd import inputs
    m, n, k = 301, 257, 190
    prob = make_problem(m, n, k, kind="integers", dtype="bf16x3", c_kind="integers")

    def stored(x, trans, extra):
        s = x.t().contiguous() if trans else x.contiguous()
        pad = (-s.shape[1]) % 4 + 4 if aligned else extra
        st, _ = inputs.padded(s, s.shape[1] + pad)
        return st.cuda()[:, : s.shape[1]]

    A = stored(prob["A"], ta, 5)
    B = stored(prob["B"], tb, 3)
    C = prob["C"].cuda()
    sg.gemm(A, B, C, 1.5, 0.5, levels=levels, mode="bf16x3", trans_a=bool(ta), trans_b=bool(tb))
    torch.cuda.synchronize()
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.5, 0.5)
    assert np.array_equal(C.cpu().double().numpy(), want)


def test_lowp_transposed_16bit_storage_rejected():
    A = torch.zeros(8, 8, dtype=torch.bfloat16, device="cuda")
    C = torch.zeros(8, 8, device="cuda")
    with pytest.raises(sg.StrassenError):
        sg.gemm(A, A, C, trans_a=True)
