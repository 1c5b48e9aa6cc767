"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

* integer inputs: Strassen equals the classical product exactly, so the GPU
  result must be bit-identical to the oracle (all levels, ragged sizes);
* real inputs: within tau_L * eps * (k |alpha| |A| |B| + |beta| |C|) of the
  fp64 oracle (tests/parity.py);
* fringes and memory safety: ld padding poisoned with NaN stays untouched,
  guard rows around C are not written, beta = 0 ignores NaN in C, k = 0 and
  alpha = 0 give beta*C, sizes below 2^levels;
* determinism (no atomics) and zero device allocation by the library;
* the full sizes of the benchmark workloads, on sampled entries.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1808_07984_amd as sg
from paper_1808_07984_amd import inputs
from parity import EPS, e_norm, make_problem, stratified_entries, tau, to_device

pytestmark = pytest.mark.gpu


def _run(prob, levels, alpha, beta, mode="plain"):
    dev = to_device(prob)
    print("case m=%d n=%d k=%d L=%d alpha=%g beta=%g dtype=%s mode=%s" % (
        prob["A"].shape[0], prob["B"].shape[1], prob["A"].shape[1], levels, alpha, beta,
        prob["A"].dtype, mode), flush=True)
    sg.gemm(dev["A"], dev["B"], dev["C"], alpha=alpha, beta=beta, levels=levels, mode=mode)
    torch.cuda.synchronize()
    return dev


@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("m,n,k", [(64, 64, 64), (65, 67, 63), (200, 129, 77), (3, 5, 7),
                                   (1, 1, 1), (257, 130, 300)])
def test_integer_exact(m, n, k, levels):
    prob = make_problem(m, n, k, kind="integers", c_kind="integers")
    dev = _run(prob, levels, 1.0, 1.0)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    got = dev["C"].cpu().double().numpy()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_integer_exact_alpha_beta_padded(levels):
    """alpha = 1.5, beta = 0.5 (exact on integers), padded leading dimensions
    with NaN in the padding, which must stay NaN and never leak in."""
    m, n, k = 375, 501, 313
    prob = make_problem(m, n, k, kind="integers", c_kind="integers",
                        lda=k + 11, ldb=n + 9, ldc=n + 7)
    dev = _run(prob, levels, 1.5, 0.5)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.5, 0.5)
    assert np.array_equal(dev["C"].cpu().double().numpy(), want)
    pad = dev["C_storage"][:, n:].cpu()
    assert torch.isnan(pad).all()


@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("m,n,k", [(1024, 1024, 1024), (1000, 1100, 900), (384, 256, 2048)])
def test_float_within_tolerance(m, n, k, levels):
    prob = make_problem(m, n, k, kind="uniform", c_kind="uniform")
    dev = _run(prob, levels, 1.0, 1.0)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    got = dev["C"].cpu().double().numpy()
    en = e_norm(got, want, prob["A"], prob["B"], prob["C"], k, 1.0, 1.0, EPS["f32"])
    print("e_norm=%.4f (tau=%g)" % (en, tau(levels)), flush=True)
    assert en <= tau(levels)


@pytest.mark.parametrize("levels", [1, 2])
def test_float_matches_f32_emulation_level(levels):
    """The GPU error is of the size the binary32 emulation of the same scheme
    predicts (within a factor 8), not merely inside the tolerance."""
    n = 512
    prob = make_problem(n, n, n, kind="uniform", c_kind="zeros")
    dev = _run(prob, levels, 1.0, 0.0)
    exact = oracle.gemm_f64(prob["A"], prob["B"])
    emu = oracle.strassen(prob["A"], prob["B"], levels=levels, f32emu=True)
    err_gpu = np.abs(dev["C"].cpu().double().numpy() - exact).max()
    err_emu = np.abs(emu - exact).max()
    print("err gpu %.3e emu %.3e" % (err_gpu, err_emu), flush=True)
    assert err_gpu <= 8 * err_emu + 1e-30


def test_guard_rows_untouched():
    """C is a window inside a larger buffer: rows above/below and columns
    outside the window keep their values."""
    m, n, k = 300, 260, 200
    prob = make_problem(m, n, k, kind="integers", c_kind="integers")
    big = torch.full((m + 8, n + 16), 7.0, device="cuda")
    C = big[4:4 + m, 8:8 + n]
    C.copy_(prob["C"].cuda())
    A, B = prob["A"].cuda(), prob["B"].cuda()
    for L in (0, 1, 2):
        C.copy_(prob["C"].cuda())
        sg.gemm(A, B, C, 1.0, 1.0, levels=L)
        torch.cuda.synchronize()
        want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
        assert np.array_equal(C.cpu().double().numpy(), want)
        host = big.cpu()
        mask = torch.ones_like(host, dtype=torch.bool)
        mask[4:4 + m, 8:8 + n] = False
        assert (host[mask] == 7.0).all(), L


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_beta_zero_ignores_nan(levels):
    prob = make_problem(130, 70, 90, kind="integers", c_kind="zeros")
    prob["C"] = torch.full((130, 70), float("nan"))
    dev = _run(prob, levels, 1.0, 0.0)
    want = oracle.gemm_f64(prob["A"], prob["B"])
    assert np.array_equal(dev["C"].cpu().double().numpy(), want)


def test_k_zero_and_alpha_zero():
    C0 = inputs.integers(33, 45, 2).cuda()
    A = torch.empty(33, 0, device="cuda")
    B = torch.empty(0, 45, device="cuda")
    for L in (0, 1, 2):
        C = C0.clone()
        sg.gemm(A, B, C, 1.0, 2.0, levels=L)
        torch.cuda.synchronize()
        assert torch.equal(C, 2 * C0)
    An = torch.full((33, 10), float("nan"), device="cuda")
    Bn = torch.full((10, 45), float("nan"), device="cuda")
    C = C0.clone()
    sg.gemm(An, Bn, C, 0.0, 0.5, levels=2)
    torch.cuda.synchronize()
    assert torch.equal(C, 0.5 * C0)
    C = C0.clone()
    sg.gemm(An, Bn, C, 0.0, 0.0, levels=1)
    torch.cuda.synchronize()
    assert torch.equal(C, torch.zeros_like(C0))


def test_empty_outputs_untouched():
    A = torch.ones(0, 5, device="cuda")
    B = torch.ones(5, 4, device="cuda")
    C = torch.ones(0, 4, device="cuda")
    sg.gemm(A, B, C, 1.0, 1.0, levels=2)
    torch.cuda.synchronize()


@pytest.mark.parametrize("levels", [1, 2])
def test_deterministic(levels):
    prob = make_problem(700, 650, 600, kind="uniform", c_kind="uniform")
    d1 = _run(prob, levels, 1.0, 1.0)
    d2 = _run(prob, levels, 1.0, 1.0)
    assert torch.equal(d1["C"], d2["C"])


def test_no_device_allocation():
    """The library allocates no workspace: free device memory is unchanged
    across calls (E5 of the paper's memory-capacity discussion)."""
    prob = make_problem(2048, 2048, 2048, kind="uniform", c_kind="uniform")
    dev = to_device(prob)
    sg.gemm(dev["A"], dev["B"], dev["C"], 1.0, 1.0, levels=2)  # loads the code object
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for L in (0, 1, 2):
        sg.gemm(dev["A"], dev["B"], dev["C"], 1.0, 1.0, levels=L)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0


def _check_entries(prob, Cg, rows, cols, k, levels, alpha, beta, exact):
    want = oracle.gemm_entries(prob["A"], prob["B"], prob["C"], rows, cols, alpha, beta)
    got = Cg[torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")].cpu().double().numpy()
    if exact:
        bad = int((got != want).sum())
        print("stratified: %d entries, %d differ (exact)" % (len(rows), bad), flush=True)
        assert bad == 0
        return
    amax = float(prob["A"].abs().max())
    bmax = float(prob["B"].abs().max())
    cmax = float(prob["C"].abs().max())
    scale = k * abs(alpha) * amax * bmax + abs(beta) * cmax
    en = float(np.abs(got - want).max()) / (EPS["f32"] * scale)
    print("stratified: %d entries, e_norm=%.4f (tau=%g)" % (len(rows), en, tau(levels)), flush=True)
    assert en <= tau(levels)


def _sampled(m, n, k, levels, alpha, beta, lda=None, ldb=None, ldc=None, kind="uniform",
             exact=False, call=None):
    """Full-size call, compared against oracle.gemm_entries on the
    stratified entries (every tile of every C block, block corners, whole
    32 x 32 accumulator blocks)."""
    prob = make_problem(m, n, k, kind=kind, c_kind=kind, lda=lda, ldb=ldb, ldc=ldc,
                        int_range=(-1, 1))
    if call is None:
        dev = _run(prob, levels, alpha, beta)
    else:
        dev = to_device(prob)
        call(dev, alpha, beta)
        torch.cuda.synchronize()
    rows, cols = stratified_entries(m, n, levels, m + n + k + levels)
    Cg = dev["C"]
    _check_entries(prob, Cg, rows, cols, k, levels, alpha, beta, exact)
    assert bool(torch.isfinite(Cg).all())
    if ldc and ldc > n:
        assert bool(torch.isnan(dev["C_storage"][:, n:]).all())


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_full_size_square_16384(levels):
    _sampled(16384, 16384, 16384, levels, 1.0, 1.0)


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_full_size_square_16384_integer_exact(levels):
    """Entries in {-1, 0, 1}: the largest intermediate (about 1.0e6 at two
    levels) is below 2^24, so every checked entry is exact."""
    _sampled(16384, 16384, 16384, levels, 1.0, 1.0, kind="integers", exact=True)


def test_full_size_hybrid_16384():
    def call(dev, alpha, beta):
        print("case hybrid 16384^3", flush=True)
        sg.gemm_hybrid(dev["A"], dev["B"], dev["C"], alpha, beta)
    _sampled(16384, 16384, 16384, 2, 1.0, 1.0, call=call)


def test_full_size_hybrid_16384_integer_exact():
    def call(dev, alpha, beta):
        print("case hybrid 16384^3 integers", flush=True)
        sg.gemm_hybrid(dev["A"], dev["B"], dev["C"], alpha, beta)
    _sampled(16384, 16384, 16384, 2, 1.0, 1.0, kind="integers", exact=True, call=call)


@pytest.mark.parametrize("k", [512, 1024, 2048, 4096])
@pytest.mark.parametrize("levels", [0, 1, 2])
def test_full_size_rank_k(k, levels):
    """Rank-k updates m = n = 16384 (k = 512 at two levels: 128-deep blocks,
    fewer than one 256-row k-slab of the plain kernel)."""
    _sampled(16384, 16384, k, levels, 1.0, 1.0)


@pytest.mark.parametrize("levels", [1, 2])
def test_full_size_square_12288(levels):
    _sampled(12288, 12288, 12288, levels, 1.0, 1.0)


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_full_size_awkward_15001(levels):
    _sampled(15001, 17003, 9007, levels, 1.5, 0.5, lda=9024, ldb=17024, ldc=17024)


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_full_size_awkward_3000(levels):
    _sampled(3000, 20000, 5000, levels, 1.5, 0.5, lda=5056, ldb=20032, ldc=20032)


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_full_size_awkward_integer_exact(levels):
    """Entries in {-1, 0, 1}: exact at every checked entry (largest
    intermediate well below 2^23)."""
    _sampled(15001, 17003, 9007, levels, 1.5, 0.5, lda=9024, ldb=17024, ldc=17024,
             kind="integers", exact=True)


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_base_entry_point_on_a_set_stream(levels):
    """strassen_gemm (the fp32 entry point without dtype, mode or stream
    arguments) on a stream chosen with strassen_set_stream: exact on
    integers, and the work is ordered on that stream."""
    m, n, k = 1100, 1060, 600
    prob = make_problem(m, n, k, kind="integers", c_kind="integers")
    dev = to_device(prob)
    A, B, C = dev["A"], dev["B"], dev["C"]
    s = torch.cuda.Stream()
    assert sg.strassen_set_stream(s.cuda_stream) == 0
    try:
        print("case strassen_gemm on a set stream L=%d" % levels, flush=True)
        rc = sg.strassen_gemm(m, n, k, A.data_ptr(), A.stride(0), B.data_ptr(), B.stride(0),
                              C.data_ptr(), C.stride(0), 1.0, 1.0, levels)
        assert rc == 0
        done = torch.cuda.Event()
        done.record(s)
        done.synchronize()
    finally:
        sg.strassen_set_stream(None)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(C.cpu().double().numpy(), want)


def _wide(x, ld):
    """Device view of x inside a rows x ld storage whose tail is NaN, built on
    the device (the storages here are several GiB)."""
    st = torch.full((x.shape[0], ld), float("nan"), dtype=x.dtype, device="cuda")
    st[:, : x.shape[1]] = x.cuda()
    return st[:, : x.shape[1]]


@pytest.fixture
def tile256():
    assert sg.strassen_set_tile(sg.STRASSEN_TILE_256) == 0
    yield
    sg.strassen_set_tile(sg.STRASSEN_TILE_AUTO)
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind,levels", [("f32", 0), ("f32", 1), ("bf16", 0), ("bf16", 1)])
def test_a_leading_dimension_past_32bit_tile_offsets(tile256, kind, levels):
    """lda so large that 256 rows of A span more than 2^32 bytes: the
    in-bounds loop addresses a tile with 32-bit per-thread byte offsets, so
    these calls must take the guarded loop, and stay exact."""
    esz = 4 if kind == "f32" else 2
    lda = (1 << 32) // (256 * esz) + 8
    m, n, k = 256 << levels, 256 << levels, 64 << levels
    prob = make_problem(m, n, k, kind="integers", dtype=kind, c_kind="integers")
    A = _wide(prob["A"], lda)
    B, C = prob["B"].cuda(), prob["C"].cuda()
    print("case lda=%d m=%d n=%d k=%d L=%d %s" % (lda, m, n, k, levels, kind), flush=True)
    sg.gemm(A, B, C, 1.0, 1.0, levels=levels)
    torch.cuda.synchronize()
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(C.cpu().double().numpy(), want)


@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_b_leading_dimension_past_32bit_tile_offsets(tile256, kind):
    """ldb so large that one k-tile of B rows spans more than 2^32 bytes."""
    esz = 4 if kind == "f32" else 2
    kt = 32 if kind == "f32" else 64
    ldb = (1 << 32) // (kt * esz) + 8
    m, n, k = 256, 256, 2 * kt
    prob = make_problem(m, n, k, kind="integers", dtype=kind, c_kind="integers")
    B = _wide(prob["B"], ldb)
    A, C = prob["A"].cuda(), prob["C"].cuda()
    print("case ldb=%d m=%d n=%d k=%d %s" % (ldb, m, n, k, kind), flush=True)
    sg.gemm(A, B, C, 1.0, 1.0, levels=0)
    torch.cuda.synchronize()
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(C.cpu().double().numpy(), want)


@pytest.fixture
def tile_mode(request):
    """Forces the fp32 tile shape for one test, then restores automatic."""
    assert sg.strassen_set_tile(request.param) == 0
    yield request.param
    sg.strassen_set_tile(sg.STRASSEN_TILE_AUTO)


TILES = [sg.STRASSEN_TILE_128, sg.STRASSEN_TILE_256]


@pytest.mark.parametrize("tile_mode", TILES, indirect=True)
@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (3, 5, 7), (65, 67, 63), (301, 257, 190),
                                   (520, 700, 333), (1100, 1060, 600)])
def test_integer_exact_each_tile(tile_mode, m, n, k, levels):
    # 1100 x 1060 x 600: at two levels the 275 x 265 x 150 blocks still have
    # interior 256 x 256 tiles with several in-bounds k-tiles, so the
    # steady-state loops of every two-level variant run and are checked exactly
    prob = make_problem(m, n, k, kind="integers", c_kind="integers")
    dev = _run(prob, levels, 1.0, 1.0)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(dev["C"].cpu().double().numpy(), want)


def _stored(x, trans, pad, fill=float("nan")):
    """Device storage of operand x (as used in the product) -- transposed when
    trans -- with `pad` extra NaN columns; returns the view passed to gemm."""
    s = x.t().contiguous() if trans else x.contiguous()
    st, view = inputs.padded(s, s.shape[1] + pad, fill=fill)
    return st.cuda()[:, : s.shape[1]]


@pytest.mark.parametrize("tile_mode", TILES, indirect=True)
@pytest.mark.parametrize("ta,tb", [(0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("levels", [0, 1, 2])
@pytest.mark.parametrize("aligned", [False, True])
def test_transposed_integer_exact(tile_mode, ta, tb, levels, aligned):
    """op(X) = X^T read from the stored transpose (ld padded with NaN, either
    to a multiple of 4 -- 16-byte loads -- or not): exact against the oracle
    on op(A), op(B)."""
    m, n, k = 301, 257, 190
    prob = make_problem(m, n, k, kind="integers", c_kind="integers")

    def pad(cols, extra):
        return (-cols) % 4 + 4 if aligned else extra

    A = _stored(prob["A"], ta, pad(m if ta else k, 5))
    B = _stored(prob["B"], tb, pad(k if tb else n, 3))
    C = prob["C"].cuda()
    print("case trans_a=%d trans_b=%d L=%d tile=%d" % (ta, tb, levels, tile_mode), flush=True)
    sg.gemm(A, B, C, 1.5, 0.5, levels=levels, trans_a=bool(ta), trans_b=bool(tb))
    torch.cuda.synchronize()
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.5, 0.5)
    assert np.array_equal(C.cpu().double().numpy(), want)


@pytest.mark.parametrize("ta,tb", [(0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("levels", [1, 2])
def test_transposed_float_within_tolerance(ta, tb, levels):
    m, n, k = 1000, 700, 1100
    prob = make_problem(m, n, k, kind="uniform", c_kind="uniform")
    A = _stored(prob["A"], ta, 0)
    B = _stored(prob["B"], tb, 0)
    C = prob["C"].cuda()
    sg.gemm(A, B, C, 1.0, 1.0, levels=levels, trans_a=bool(ta), trans_b=bool(tb))
    torch.cuda.synchronize()
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    en = e_norm(C.cpu().double().numpy(), want, prob["A"], prob["B"], prob["C"], k, 1.0, 1.0,
                EPS["f32"])
    print("e_norm=%.4f (tau=%g)" % (en, tau(levels)), flush=True)
    assert en <= tau(levels)


@pytest.mark.parametrize("tile_mode", TILES, indirect=True)
@pytest.mark.parametrize("levels", [1, 2])
def test_float_each_tile(tile_mode, levels):
    prob = make_problem(1536, 1280, 1024, kind="uniform", c_kind="uniform")
    dev = _run(prob, levels, 1.0, 1.0)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    en = e_norm(dev["C"].cpu().double().numpy(), want, prob["A"], prob["B"], prob["C"], 1024,
                1.0, 1.0, EPS["f32"])
    assert en <= tau(levels)
