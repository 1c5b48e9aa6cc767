"""GPU parity of the formed schedules (strassen_gemm_formed,
strassen_gemm_formed_ex): the multi-term operand sums of eq. gpu_allops
(applied once or twice) formed once into caller workspace, then single-term
products scattered into C.

* integer inputs: equal to the classical product bit for bit (oracle);
* real inputs: equal bit for bit to the fused one-level call
  (strassen_gemm_ex, levels = 1), whose sums are formed in the same order
  and precision, where no chain applies (fp32, and 16-bit C blocks of fewer
  than 128 tiles of 256 x 256); with chains (M5 and M6 accumulated after M2
  and M3 and added into C with them) C0 and C3 may differ in the last bits
  and C1, C2 stay equal; always within tau_1 of the fp64 oracle at the gate
  eps of the format (bf16x3 at 2^-16: hi + lo carries 16 significant bits;
  its figure at 2^-23 is printed, not gated);
* two levels: integers exact; real inputs equal bit for bit to the fused
  two-level call (no chains there, the same batches in the same order);
* the library allocates nothing; the workspace is the caller's.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1808_07984_amd as sg
from parity import EPS, e_norm, make_problem, stratified_entries, tau, to_device

pytestmark = pytest.mark.gpu

FAMILIES = {"f32": ("f32", "plain"), "bf16": ("bf16", "plain"), "f16": ("f16", "plain"),
            "bf16x3": ("bf16x3", "bf16x3")}
GATE_EPS = {"f32": 2.0 ** -23, "bf16": 2.0 ** -7, "f16": 2.0 ** -10, "bf16x3": 2.0 ** -16}


def _formed(dev, alpha, beta, mode, ws=None, levels=1):
    A, B, C = dev["A"], dev["B"], dev["C"]
    print("formed m=%d n=%d k=%d L=%d dtype=%s mode=%s" % (A.shape[0], B.shape[1], A.shape[1], levels, A.dtype,
                                                           mode), flush=True)
    sg.gemm_formed(A, B, C, alpha=alpha, beta=beta, mode=mode, workspace=ws, levels=levels)
    torch.cuda.synchronize()
    return C


@pytest.mark.parametrize("fam", sorted(FAMILIES))
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (3, 5, 7), (64, 64, 64), (65, 67, 63), (200, 129, 77),
                                   (257, 130, 300), (1100, 1060, 600)])
def test_formed_integer_exact(fam, m, n, k):
    dtype, mode = FAMILIES[fam]
    prob = make_problem(m, n, k, kind="integers", dtype=dtype, c_kind="integers")
    dev = to_device(prob)
    got = _formed(dev, 1.0, 1.0, mode)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(got.cpu().double().numpy(), want)


@pytest.mark.parametrize("fam", sorted(FAMILIES))
def test_formed_integer_exact_padded_alpha_beta(fam):
    dtype, mode = FAMILIES[fam]
    m, n, k = 375, 501, 313
    prob = make_problem(m, n, k, kind="integers", dtype=dtype, c_kind="integers",
                        lda=k + 11, ldb=n + 9, ldc=n + 7)
    dev = to_device(prob)
    got = _formed(dev, 1.5, 0.5, mode)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.5, 0.5)
    assert np.array_equal(got.cpu().double().numpy(), want)
    assert torch.isnan(dev["C_storage"][:, n:]).all()


@pytest.mark.parametrize("fam", sorted(FAMILIES))
@pytest.mark.parametrize("kind", ["uniform", "normal"])
@pytest.mark.parametrize("m,n,k", [(300, 260, 520), (513, 257, 1000), (1030, 1100, 1500)])
def test_formed_equals_fused_one_level(fam, kind, m, n, k):
    """Same sums, same rounding, same accumulation order: bit-identical."""
    dtype, mode = FAMILIES[fam]
    prob = make_problem(m, n, k, kind=kind, dtype=dtype, c_kind=kind)
    d1 = to_device(prob)
    d2 = to_device(prob)
    got = _formed(d1, 1.25, 0.75, mode)
    sg.gemm(d2["A"], d2["B"], d2["C"], alpha=1.25, beta=0.75, levels=1, mode=mode)
    torch.cuda.synchronize()
    assert torch.equal(got, d2["C"])
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.25, 0.75)
    en = e_norm(got.cpu().numpy(), want, prob["A"], prob["B"], prob["C"], k, 1.25, 0.75, GATE_EPS[fam])
    en23 = en * GATE_EPS[fam] / EPS["f32"]
    print("e_norm=%.4g (gate eps of %s), %.4g at 2^-23" % (en, fam, en23), flush=True)
    assert en <= tau(1)


@pytest.mark.parametrize("fam", ["bf16", "f16", "bf16x3"])
@pytest.mark.parametrize("kind", ["integers", "uniform"])
def test_formed_chained_16bit(fam, kind):
    """C blocks of 16 x 8 tiles of 256 x 256: M5 and M6 run chained after M2
    and M3.  Integers: exact.  Reals: C1 and C2 (not chained) equal the fused
    call bit for bit; C0 and C3 within a few roundings of it; all within
    tau_1 of the oracle."""
    dtype, mode = FAMILIES[fam]
    m, n, k = 8192, 4096, 1024
    prob = make_problem(m, n, k, kind=kind, dtype=dtype, c_kind=kind, int_range=(-1, 1))
    d1, d2 = to_device(prob), to_device(prob)
    assert sg.strassen_profile_start() == 0
    got = _formed(d1, 1.0, 1.0, mode)
    rc, recs = sg.strassen_profile_stop()
    names = [r.kernel.decode() for r in recs[:rc]]
    # two sum-forming launches, M1 and M4 as one batch, M0 alone, and one
    # chained launch of the two chains M2 -> M5 and M3 -> M6
    assert sum(nm.startswith("form_sums") for nm in names) == 2
    assert sum("<chained,2," in nm for nm in names) == 1
    assert len(names) == 5, names
    if kind == "integers":
        rows, cols = stratified_entries(m, n, 1, 7)
        want = oracle.gemm_entries(prob["A"], prob["B"], prob["C"], rows, cols, 1.0, 1.0)
        g = got[torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")].cpu().double().numpy()
        assert np.array_equal(g, want)
        return
    sg.gemm(d2["A"], d2["B"], d2["C"], levels=1, mode=mode)
    torch.cuda.synchronize()
    ref = d2["C"]
    hm, hn = m // 2, n // 2
    assert torch.equal(got[:hm, hn:], ref[:hm, hn:])      # C1
    assert torch.equal(got[hm:, :hn], ref[hm:, :hn])      # C2
    diff = float((got - ref).abs().max())
    scale = k * float(prob["A"].float().abs().max()) * float(prob["B"].float().abs().max()) + \
        float(prob["C"].abs().max())
    print("chained vs fused: max |diff| %.3g = %.3g of eps scale" % (diff, diff / (GATE_EPS[fam] * scale)), flush=True)
    assert diff <= tau(1) * GATE_EPS[fam] * scale


def test_formed_beta_zero_ignores_nan_and_degenerate():
    prob = make_problem(130, 140, 150, kind="uniform", c_kind="uniform")
    dev = to_device(prob)
    dev["C"].fill_(float("nan"))
    got = _formed(dev, 1.0, 0.0, "bf16x3")
    assert bool(torch.isfinite(got).all())
    # k = 0 and alpha = 0: C := beta * C, no workspace needed
    C = torch.ones(33, 17, device="cuda")
    A = torch.empty(33, 0, device="cuda")
    B = torch.empty(0, 17, device="cuda")
    rc = sg.strassen_gemm_formed(33, 17, 0, A.data_ptr(), 1, sg.STRASSEN_F32, B.data_ptr(), 17,
                                 sg.STRASSEN_F32, C.data_ptr(), 17, 1.0, 0.5, sg.STRASSEN_MODE_PLAIN,
                                 None, 0, None)
    torch.cuda.synchronize()
    assert rc == 0 and bool((C == 0.5).all())
    A = torch.rand(33, 9, device="cuda")
    B = torch.rand(9, 17, device="cuda")
    rc = sg.strassen_gemm_formed(33, 17, 9, A.data_ptr(), 9, sg.STRASSEN_F32, B.data_ptr(), 17,
                                 sg.STRASSEN_F32, C.data_ptr(), 17, 0.0, 2.0, sg.STRASSEN_MODE_PLAIN,
                                 None, 0, None)
    torch.cuda.synchronize()
    assert rc == 0 and bool((C == 1.0).all())


def test_formed_no_device_allocation_and_stream():
    """Nothing is allocated by the library; the call runs on the given stream."""
    prob = make_problem(1024, 1024, 1024, kind="integers", dtype="bf16x3", c_kind="integers")
    dev = to_device(prob)
    need = sg.api.formed_workspace_bytes(1024, 1024, 1024, torch.float32, "bf16x3")
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    C0 = dev["C"].clone()
    s = torch.cuda.Stream()  # created (and its queue allocated) before the measurement
    with torch.cuda.stream(s):
        sg.gemm_formed(dev["A"], dev["B"], dev["C"], mode="bf16x3", workspace=ws)
    s.synchronize()
    dev["C"].copy_(C0)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    with torch.cuda.stream(s):
        sg.gemm_formed(dev["A"], dev["B"], dev["C"], mode="bf16x3", workspace=ws)
    s.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(dev["C"].cpu().double().numpy(), want)


@pytest.mark.parametrize("size", [8192, 16384])
def test_formed_full_size_bf16x3_equals_fused(size):
    """Benchmark sizes: C1 and C2 equal the fused one-level result (C0 and
    C3 take the chained products), and sampled entries (one per 256 x 256 tile of every C block, plus corners)
    are within tau_1 of the fp64 oracle at the bf16x3 gate (2^-16); the
    figure at 2^-23 is printed."""
    m = n = k = size
    prob = make_problem(m, n, k, kind="normal", dtype="bf16x3", c_kind="normal", fill=0.0)
    d1 = to_device(prob)
    C0 = d1["C"].clone()
    _formed(d1, 1.0, 1.0, "bf16x3")
    got = d1["C"].clone()
    d1["C"].copy_(C0)
    del C0
    sg.gemm(d1["A"], d1["B"], d1["C"], levels=1, mode="bf16x3")
    torch.cuda.synchronize()
    h = size // 2  # chained products add into C0 and C3 only
    assert torch.equal(got[:h, h:], d1["C"][:h, h:]) and torch.equal(got[h:, :h], d1["C"][h:, :h])
    rng = np.random.default_rng(size)
    ti = np.arange(0, m, 256)
    tj = np.arange(0, n, 256)
    rows = (np.repeat(ti, len(tj)) + rng.integers(0, 256, len(ti) * len(tj))).clip(0, m - 1)
    cols = (np.tile(tj, len(ti)) + rng.integers(0, 256, len(ti) * len(tj))).clip(0, n - 1)
    rows = np.concatenate([rows, [0, m - 1, 0, m - 1]])
    cols = np.concatenate([cols, [0, n - 1, n - 1, 0]])
    want = oracle.gemm_entries(prob["A"], prob["B"], prob["C"], rows, cols, 1.0, 1.0)
    g = got[torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")].cpu().double().numpy()
    scale = k * float(prob["A"].abs().max()) * float(prob["B"].abs().max()) + float(prob["C"].abs().max())
    en = float(np.abs(g - want).max()) / (GATE_EPS["bf16x3"] * scale)
    print("sampled e_norm=%.4g at 2^-16, %.4g at 2^-23 (tau=%g), %d entries"
          % (en, en * 128, tau(1), len(rows)), flush=True)
    assert en <= tau(1)


def _bf16_rne_bits(x):
    """bf16 bits of fp32 values x rounded to nearest even (finite x)."""
    u = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint32) & 0xFFFF


def _pre_split_words(s):
    """The compensated mode's pre-split layout of fp32 values s (rows x
    cols, cols a multiple of 4): per unit of four elements the words
    (hi0 | hi1 << 16, hi2 | hi3 << 16, lo0 | lo1 << 16, lo2 | lo3 << 16), hi
    = bf16(s) and lo = bf16(s - hi), both rounded to nearest even."""
    hi = _bf16_rne_bits(s)
    lo = _bf16_rne_bits(s - (hi << 16).view(np.float32))
    r, c = s.shape
    hi = hi.reshape(r, c // 4, 2, 2)
    lo = lo.reshape(r, c // 4, 2, 2)
    w = np.concatenate([hi[..., 0] | (hi[..., 1] << 16), lo[..., 0] | (lo[..., 1] << 16)], axis=2)
    return w.reshape(r, c).astype(np.uint32)


@pytest.mark.parametrize("m,n,k", [(64, 64, 64), (70, 66, 62)])
def test_formed_bf16x3_workspace_holds_pre_split_operands(m, n, k):
    """One level, bf16x3: the workspace holds A's seven operands (five sums,
    the two single quadrants) and B's five sums, each stored pre-split: the
    fp32 sum of the stored quadrants with the first term's sign factored
    out, zero outside the operands' extents, split into bf16 hi and lo
    halves of each 16-byte unit."""
    prob = make_problem(m, n, k, kind="uniform", dtype="bf16x3", c_kind="uniform")
    dev = to_device(prob)
    need = sg.api.formed_workspace_bytes(m, n, k, torch.float32, "bf16x3")
    ws = torch.zeros(need, dtype=torch.uint8, device="cuda")
    _formed(dev, 1.0, 1.0, "bf16x3", ws=ws)
    words = ws.cpu().numpy().view(np.uint32)
    sm, sk, sn = -(-m // 2), -(-(-(-k // 2)) // 4) * 4, -(-(-(-n // 2)) // 4) * 4
    assert need == 4 * (7 * sm * sk + 5 * sk * sn)

    def quadrant(X, rows, cols, q):
        R, Cc = q // 2, q % 2
        out = np.zeros((rows, cols), np.float32)
        blk = X[R * rows:(R + 1) * rows, Cc * cols:(Cc + 1) * cols]
        out[:blk.shape[0], :blk.shape[1]] = blk
        return out

    rc, ins = sg.strassen_plan_instances(1)
    assert rc >= 0
    A = prob["A"].float().numpy()
    B = prob["B"].float().numpy()
    want_a, want_b = [], []
    for p in ins:
        for X, rows, cols, nt, blocks, signs, want, single in (
                (A, sm, sk, p.n_a, p.a_block, p.a_sign, want_a, True),
                (B, sk, sn, p.n_b, p.b_block, p.b_sign, want_b, False)):
            if nt == 1 and not single:
                continue
            s = quadrant(X, rows, cols, blocks[0])
            if nt == 2:
                s = (s + np.float32(signs[1] * signs[0]) * quadrant(X, rows, cols, blocks[1])).astype(np.float32)
            want.append(_pre_split_words(s))
    assert len(want_a) == 7 and len(want_b) == 5
    got_a = words[:7 * sm * sk].reshape(7, sm, sk)
    got_b = words[7 * sm * sk:].reshape(5, sk, sn)
    for got, want in ((got_a, want_a), (got_b, want_b)):
        # every stored block is one of the operands, each operand stored once
        matched = sorted(next(i for i, w in enumerate(want) if np.array_equal(g, w)) for g in got)
        assert matched == list(range(len(want)))


def test_formed_workspace_errors_on_device():
    prob = make_problem(96, 80, 72, kind="uniform", c_kind="uniform")
    dev = to_device(prob)
    need = sg.api.formed_workspace_bytes(96, 80, 72)
    ws = torch.empty(need + 64, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        sg.gemm_formed(dev["A"], dev["B"], dev["C"], workspace=ws[: need - 4])
    A, B, C = dev["A"], dev["B"], dev["C"]
    rc = sg.strassen_gemm_formed(96, 80, 72, A.data_ptr(), A.stride(0), sg.STRASSEN_F32, B.data_ptr(),
                                 B.stride(0), sg.STRASSEN_F32, C.data_ptr(), C.stride(0), 1.0, 1.0,
                                 sg.STRASSEN_MODE_PLAIN, ws.data_ptr() + 4, need, None)
    assert rc == -15


# ---- two levels (strassen_gemm_formed_ex, levels = 2) ----

@pytest.mark.parametrize("fam", sorted(FAMILIES))
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (3, 5, 7), (65, 67, 63), (257, 130, 300), (1100, 1060, 600)])
def test_formed2_integer_exact(fam, m, n, k):
    dtype, mode = FAMILIES[fam]
    prob = make_problem(m, n, k, kind="integers", dtype=dtype, c_kind="integers")
    dev = to_device(prob)
    got = _formed(dev, 1.0, 1.0, mode, levels=2)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(got.cpu().double().numpy(), want)


@pytest.mark.parametrize("fam", sorted(FAMILIES))
def test_formed2_integer_exact_padded_alpha_beta(fam):
    dtype, mode = FAMILIES[fam]
    m, n, k = 375, 501, 313
    prob = make_problem(m, n, k, kind="integers", dtype=dtype, c_kind="integers",
                        lda=k + 11, ldb=n + 9, ldc=n + 7)
    dev = to_device(prob)
    got = _formed(dev, 1.5, 0.5, mode, levels=2)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.5, 0.5)
    assert np.array_equal(got.cpu().double().numpy(), want)
    assert torch.isnan(dev["C_storage"][:, n:]).all()


@pytest.mark.parametrize("fam", sorted(FAMILIES))
@pytest.mark.parametrize("m,n,k", [(300, 260, 520), (1030, 1100, 1500), (12288, 12288, 512)])
def test_formed2_equals_fused_two_level(fam, m, n, k):
    """Four-term sums in the fused kernels' order and precision, the same
    batches in the same order, single-term products accumulating in the
    same k order: bit-identical to strassen_gemm_ex at levels = 2 (12288:
    C blocks of 144 tiles of 256 x 256, the large-tile launches)."""
    dtype, mode = FAMILIES[fam]
    prob = make_problem(m, n, k, kind="uniform", dtype=dtype, c_kind="uniform")
    d1 = to_device(prob)
    d2 = to_device(prob)
    assert sg.strassen_profile_start() == 0
    got = _formed(d1, 1.25, 0.75, mode, levels=2)
    rc, recs = sg.strassen_profile_stop()
    names = [r.kernel.decode() for r in recs[:rc]]
    # 16 product launches (the fused schedule's batches) and one sum-forming
    # launch per multi-term level-1 operand of A and of B
    assert sum(not nm.startswith("form_terms") for nm in names) == 16, names
    assert sum(nm.startswith("form_terms") for nm in names) == 14, names
    sg.gemm(d2["A"], d2["B"], d2["C"], alpha=1.25, beta=0.75, levels=2, mode=mode)
    torch.cuda.synchronize()
    assert torch.equal(got, d2["C"])
    if m * n <= 2 ** 22:
        want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.25, 0.75)
        en = e_norm(got.cpu().numpy(), want, prob["A"], prob["B"], prob["C"], k, 1.25, 0.75, GATE_EPS[fam])
        print("e_norm=%.4g (gate eps of %s)" % (en, fam), flush=True)
        assert en <= tau(2)


def test_formed2_workspace_and_errors():
    m, n, k = 1000, 900, 700
    sm, sk, sn = 250, 176, 232   # ceil(/4), k and n rounded up to 8 (16-bit) elements
    assert sg.api.formed_workspace_bytes(m, n, k, torch.bfloat16, "plain", levels=2) == 2 * 45 * (sm * sk + sk * sn)
    sm, sk, sn = 250, 176, 228   # fp32: rounded up to 4
    # compensated: the single blocks are stored (pre-split) too
    assert sg.api.formed_workspace_bytes(m, n, k, torch.float32, "bf16x3", levels=2) == 4 * 49 * (sm * sk + sk * sn)
    assert sg.api.formed_workspace_bytes(m, n, k, torch.float32, "plain", levels=2) == 4 * 45 * (sm * sk + sk * sn)
    prob = make_problem(96, 80, 72, kind="uniform", c_kind="uniform")
    dev = to_device(prob)
    A, B, C = dev["A"], dev["B"], dev["C"]
    need = sg.api.formed_workspace_bytes(96, 80, 72, levels=2)
    ws = torch.empty(need + 64, dtype=torch.uint8, device="cuda")
    common = (96, 80, 72, A.data_ptr(), A.stride(0), sg.STRASSEN_F32, B.data_ptr(), B.stride(0), sg.STRASSEN_F32,
              C.data_ptr(), C.stride(0), 1.0, 1.0)
    for bad in (-1, 3):
        assert sg.strassen_gemm_formed_ex(*common, bad, sg.STRASSEN_MODE_PLAIN, ws.data_ptr(), need, None) == -14
    assert sg.strassen_gemm_formed_ex(*common, 2, sg.STRASSEN_MODE_PLAIN, ws.data_ptr() + 4, need, None) == -16
    assert sg.strassen_gemm_formed_ex(*common, 2, sg.STRASSEN_MODE_PLAIN, ws.data_ptr(), need - 16, None) == -17
    assert sg.strassen_gemm_formed_ex(*common, 2, 7, ws.data_ptr(), need, None) == -15
    torch.cuda.synchronize()


@pytest.mark.parametrize("fam", ["bf16", "bf16x3"])
def test_formed2_full_size_equals_fused(fam):
    """16384^3 (the precision configuration's largest size), two levels:
    equal to the fused two-level call bit for bit, and stratified entries
    (every 256 x 256 tile of every C block, block corners, whole 32 x 32
    accumulator blocks) within tau_2 of the fp64 oracle at the gate eps."""
    dtype, mode = FAMILIES[fam]
    N = 16384
    prob = make_problem(N, N, N, kind="normal", dtype=dtype, c_kind="zeros")
    dev = to_device(prob)
    _formed(dev, 1.0, 0.0, mode, levels=2)
    got = dev["C"].clone()
    sg.gemm(dev["A"], dev["B"], dev["C"], 1.0, 0.0, levels=2, mode=mode)
    torch.cuda.synchronize()
    assert torch.equal(got, dev["C"])
    rows, cols = stratified_entries(N, N, 2, 2)
    want = oracle.gemm_entries(prob["A"], prob["B"], None, rows, cols, 1.0, 0.0)
    g = got[torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")].double().cpu().numpy()
    scale = N * float(prob["A"].float().abs().max()) * float(prob["B"].float().abs().max())
    en = float(np.abs(g - want).max()) / (GATE_EPS[fam] * scale)
    print("sampled e_norm %.4g at eps=%g, %d entries" % (en, GATE_EPS[fam], len(rows)), flush=True)
    assert en <= tau(2)


def _random_shapes(count, seed):
    rng = np.random.default_rng(seed)
    return [tuple(int(v) for v in rng.integers(1, 700, 3)) for _ in range(count)]


@pytest.mark.parametrize("fam", sorted(FAMILIES))
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (65, 67, 63), (257, 130, 301), (1030, 1100, 1503)])
def test_formed0_equals_plain(fam, m, n, k):
    """Level 0: the plain product (on pre-split copies of A and B in the
    bf16x3 mode), bit for bit the plain call's result, alpha and beta
    applied; integers exact against the oracle."""
    dtype, mode = FAMILIES[fam]
    prob = make_problem(m, n, k, kind="uniform", dtype=dtype, c_kind="uniform")
    d1, d2 = to_device(prob), to_device(prob)
    got = _formed(d1, 1.25, 0.5, mode, levels=0)
    sg.gemm(d2["A"], d2["B"], d2["C"], alpha=1.25, beta=0.5, levels=0, mode=mode)
    torch.cuda.synchronize()
    assert torch.equal(got, d2["C"])
    prob = make_problem(m, n, k, kind="integers", dtype=dtype, c_kind="integers")
    dev = to_device(prob)
    got = _formed(dev, 1.0, 1.0, mode, levels=0)
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(got.cpu().double().numpy(), want)


def test_formed0_full_size_bf16x3_equals_plain():
    """8192^3, bf16x3: the pre-split plain product (direct-to-LDS loads)
    equals the plain call bit for bit."""
    n = 8192
    prob = make_problem(n, n, n, kind="normal", dtype="bf16x3", c_kind="normal", fill=0.0)
    d1 = to_device(prob)
    C0 = d1["C"].clone()
    got = _formed(d1, 1.0, 1.0, "bf16x3", levels=0).clone()
    d1["C"].copy_(C0)
    sg.gemm(d1["A"], d1["B"], d1["C"], levels=0, mode="bf16x3")
    torch.cuda.synchronize()
    assert torch.equal(got, d1["C"])


@pytest.mark.parametrize("levels,m,n,k", [(0, 4200, 4100, 1001), (1, 5800, 6000, 2566)])
def test_formed_bf16x3_direct_loads_ragged_integer_exact(levels, m, n, k):
    """Shapes whose products run the 256 x 256 tiles (direct-to-LDS loads of
    the pre-split operands) with a ragged last k-tile and edge tiles (both
    taking the staged loop) and, at one level, the chained launch: integers
    exact against the oracle, every entry."""
    prob = make_problem(m, n, k, kind="integers", dtype="bf16x3", c_kind="integers")
    dev = to_device(prob)
    assert sg.strassen_profile_start() == 0
    got = _formed(dev, 1.0, 1.0, "bf16x3", levels=levels)
    rc, recs = sg.strassen_profile_stop()
    names = [r.kernel.decode() for r in recs[:rc]]
    assert any("bf16x3p,256x256" in nm for nm in names), names
    want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.0, 1.0)
    assert np.array_equal(got.cpu().double().numpy(), want)


def test_formed2_bf16x3_direct_loads_ragged_sampled():
    """Two levels at 11600 x 12000 x 2566 (blocks 2900 x 3000 x 644 on 256 x
    256 tiles: a ragged last k-tile and edge tiles): integer entries sampled
    in every tile of every C block, exact against the oracle."""
    m, n, k = 11600, 12000, 2566
    prob = make_problem(m, n, k, kind="integers", dtype="bf16x3", c_kind="integers")
    dev = to_device(prob)
    got = _formed(dev, 1.0, 1.0, "bf16x3", levels=2)
    rows, cols = stratified_entries(m, n, 2, 3)
    want = oracle.gemm_entries(prob["A"], prob["B"], prob["C"], rows, cols, 1.0, 1.0)
    g = got[torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")].cpu().double().numpy()
    assert np.array_equal(g, want)


@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("fam", sorted(FAMILIES))
def test_formed_random_shapes_integer_exact(fam, levels):
    """Twelve seeded random shapes up to 700 per dimension (ragged blocks,
    virtual padding in every operand), alpha 1.5, beta 0.5: exact against
    the classical product."""
    dtype, mode = FAMILIES[fam]
    for (m, n, k) in _random_shapes(12, 1000 * levels + len(fam)):
        prob = make_problem(m, n, k, kind="integers", dtype=dtype, c_kind="integers")
        dev = to_device(prob)
        got = _formed(dev, 1.5, 0.5, mode, levels=levels)
        want = oracle.gemm_f64(prob["A"], prob["B"], prob["C"], 1.5, 0.5)
        assert np.array_equal(got.cpu().double().numpy(), want), (m, n, k)
