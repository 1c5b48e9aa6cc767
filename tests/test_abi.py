"""The C-ABI library loads, exports every symbol its header declares, and
validates arguments with the documented codes -- all without a GPU (no call
here reaches a kernel launch)."""
import ctypes
import os
import re

import pytest

import paper_1808_07984_amd as sg
from paper_1808_07984_amd import _binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"\b(strassen_\w+)\s*\(", src)
    return sorted(set(names))


def test_header_symbols_exported_and_bound():
    names = _declared_functions()
    assert "strassen_gemm" in names and "strassen_gemm_ex" in names
    lib = ctypes.CDLL(_binding.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
        assert name in _binding.SIGNATURES, name
        assert hasattr(sg, name), name


def test_no_oracle_in_product_path():
    """The product package neither imports nor loads the oracle."""
    pkg = os.path.join(ROOT, "paper_1808_07984_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "liboracle" not in src, f


N = None  # null pointer
P = 4096  # any non-null value: validation rejects before anything is dereferenced


@pytest.mark.parametrize("args,code", [
    ((-1, 4, 4, P, 4, P, 4, P, 4, 1.0, 1.0, 1), -1),
    ((4, -1, 4, P, 4, P, 4, P, 4, 1.0, 1.0, 1), -2),
    ((4, 4, -1, P, 4, P, 4, P, 4, 1.0, 1.0, 1), -3),
    ((4, 4, 4, N, 4, P, 4, P, 4, 1.0, 1.0, 1), -4),
    ((4, 4, 8, P, 7, P, 4, P, 4, 1.0, 1.0, 1), -5),
    ((4, 4, 4, P, 4, N, 4, P, 4, 1.0, 1.0, 1), -6),
    ((4, 8, 4, P, 4, P, 7, P, 8, 1.0, 1.0, 1), -7),
    ((4, 4, 4, P, 4, P, 4, N, 4, 1.0, 1.0, 1), -8),
    ((4, 8, 4, 1 << 20, 4, 1 << 21, 8, P, 7, 1.0, 1.0, 1), -9),
    ((4, 4, 4, 1 << 20, 4, 1 << 21, 4, P, 4, 1.0, 1.0, 3), -12),
    ((4, 4, 4, 1 << 20, 4, 1 << 21, 4, P, 4, 1.0, 1.0, -1), -12),
    # A overlaps C
    ((4, 4, 4, 1 << 20, 4, 1 << 21, 4, (1 << 20) + 16, 4, 1.0, 1.0, 1), -8),
    # B overlaps C
    ((4, 4, 4, 1 << 20, 4, 1 << 21, 4, (1 << 21) - 8, 4, 1.0, 1.0, 1), -8),
    # m == 0 / n == 0: nothing to do, success without touching the GPU
    ((0, 4, 4, N, 4, N, 4, N, 4, 1.0, 1.0, 1), 0),
    ((4, 0, 4, N, 4, N, 4, N, 4, 1.0, 1.0, 1), 0),
])
def test_strassen_gemm_validation(args, code):
    assert sg.strassen_gemm(*args) == code


def test_ex_validation():
    base = dict(m=4, n=4, k=4, A=1 << 20, lda=4, a_type=0, trans_a=0, B=1 << 21, ldb=4, b_type=0,
                trans_b=0, C=1 << 22, ldc=4, alpha=1.0, beta=1.0, levels=1, mode=0, hip_stream=None)

    def call(**kw):
        a = dict(base, **kw)
        return sg.strassen_gemm_ex(*a.values())

    assert call(a_type=7) == -6
    assert call(trans_a=2) == -7
    assert call(b_type=1) == -10
    assert call(trans_b=-1) == -11
    assert call(ldc=3) == -13
    assert call(levels=5) == -16
    assert call(mode=9) == -17
    assert call(mode=1, a_type=1, b_type=1) == -17   # compensated mode needs fp32 operands
    assert call(trans_a=1, lda=3, m=4, k=4) == -5    # stored A is k x m
    assert call(C=(1 << 20) + 4) == -12               # overlap reported on C


def test_error_strings():
    assert sg.strassen_error_string(0) == "success"
    assert "argument 4" in sg.strassen_error_string(-4)
    assert sg.strassen_error_string(-99) == "invalid argument"
    assert isinstance(sg.strassen_error_string(1), str)


def test_plan_info_validation():
    rc, _ = sg.strassen_plan_info(-1, 1, 1, 1)
    assert rc == -1
    rc, _ = sg.strassen_plan_info(1, 1, 1, 3)
    assert rc == -4
    rc, _ = sg.strassen_plan_info(1, 1, 1, 1, 0, 1)
    assert rc == 0
    rc, _ = sg.strassen_plan_info(1, 1, 1, 1, 1, 1)
    assert rc == -6
    rc, _ = sg.strassen_plan_instances(3)
    assert rc == -1


def test_profile_records_nothing_without_launches():
    assert sg.strassen_profile_start() == 0
    rc, recs = sg.strassen_profile_stop()
    assert rc == 0 and recs == []


def test_hybrid_workspace_size():
    # (2 sm)(2 sk) + (2 sk)(2 sn) floats with sm = ceil(m/4), sn/sk = ceil(./4) rounded to 4
    assert sg.strassen_hybrid_workspace_size(16384, 16384, 16384) == 4 * 2 * 8192 * 8192
    m, n, k = 15001, 17003, 9007
    sm, sn, sk = -(-m // 4), -(-(-(-n // 4)) // 4) * 4, -(-(-(-k // 4)) // 4) * 4
    assert sg.strassen_hybrid_workspace_size(m, n, k) == 4 * (4 * sm * sk + 4 * sk * sn)
    assert sg.strassen_hybrid_workspace_size(-1, 1, 1) == -1
    assert sg.strassen_hybrid_workspace_size(1, 1, -1) == -3


def test_hybrid_validation():
    need = sg.strassen_hybrid_workspace_size(64, 64, 64)
    A, B, C, W = 1 << 20, 1 << 22, 1 << 24, 1 << 26
    base = [64, 64, 64, A, 64, B, 64, C, 64, 1.0, 1.0, W, need, None]

    def call(**kw):
        a = list(base)
        idx = dict(m=0, lda=4, ldb=6, ldc=8, ws=11, wsb=12, A=3, C=7)
        for key, v in kw.items():
            a[idx[key]] = v
        return sg.strassen_gemm_hybrid(*a)

    assert call(m=-1) == -1
    assert call(lda=3) == -5
    assert call(ldc=3) == -9
    assert call(ws=None) == -12
    assert call(ws=W + 4) == -12          # not 16-byte aligned
    assert call(wsb=need - 4) == -13
    assert call(ws=C + 64) == -12         # workspace overlaps C
    assert call(C=A + 128) == -8          # A overlaps C


def test_formed_workspace_size():
    # e * (5 sm sk + 5 sk sn), one-level extents, sk and sn rounded to the
    # 16-byte vector width (4 fp32, 8 16-bit elements); the compensated mode
    # stores A's two single quadrants (pre-split) too: 4 * (7 sm sk + 5 sk sn)
    def want(m, n, k, e, v, na=5):
        sm = -(-m // 2)
        sk = -(-(-(-k // 2)) // v) * v
        sn = -(-(-(-n // 2)) // v) * v
        return e * (na * sm * sk + 5 * sk * sn)
    f = sg.strassen_formed_workspace_size
    assert f(16384, 16384, 16384, sg.STRASSEN_F32, sg.STRASSEN_MODE_BF16X3) == 4 * 12 * 8192 * 8192
    assert f(16384, 16384, 16384, sg.STRASSEN_F32, sg.STRASSEN_MODE_PLAIN) == 4 * 10 * 8192 * 8192
    for (m, n, k) in ((15001, 17003, 9007), (3, 5, 7), (1, 1, 1), (3000, 20000, 5000)):
        assert f(m, n, k, sg.STRASSEN_F32, sg.STRASSEN_MODE_PLAIN) == want(m, n, k, 4, 4)
        assert f(m, n, k, sg.STRASSEN_F32, sg.STRASSEN_MODE_BF16X3) == want(m, n, k, 4, 4, na=7)
        assert f(m, n, k, sg.STRASSEN_BF16, sg.STRASSEN_MODE_PLAIN) == want(m, n, k, 2, 8)
        assert f(m, n, k, sg.STRASSEN_F16, sg.STRASSEN_MODE_PLAIN) == want(m, n, k, 2, 8)
    assert f(-1, 1, 1, 0, 0) == -1
    assert f(1, -1, 1, 0, 0) == -2
    assert f(1, 1, -1, 0, 0) == -3
    assert f(1, 1, 1, 7, 0) == -4
    assert f(1, 1, 1, sg.STRASSEN_BF16, sg.STRASSEN_MODE_BF16X3) == -5


def test_formed_workspace_size_two_levels():
    # e * 45 (sm sk + sk sn), two-level extents (ceil(/4), sk and sn rounded
    # to the vector width), 49 blocks per operand in the compensated mode
    # (its single blocks stored pre-split too); one level as
    # strassen_formed_workspace_size
    def want(m, n, k, e, v, nb=45):
        sm = -(-m // 4)
        sk = -(-(-(-k // 4)) // v) * v
        sn = -(-(-(-n // 4)) // v) * v
        return e * nb * (sm * sk + sk * sn)
    f = sg.strassen_formed_workspace_size_ex
    assert f(16384, 16384, 16384, 2, sg.STRASSEN_F32, sg.STRASSEN_MODE_BF16X3) == 4 * 98 * 4096 * 4096
    assert f(16384, 16384, 16384, 2, sg.STRASSEN_F32, sg.STRASSEN_MODE_PLAIN) == 4 * 90 * 4096 * 4096
    for (m, n, k) in ((15001, 17003, 9007), (3, 5, 7), (1, 1, 1), (3000, 20000, 5000)):
        assert f(m, n, k, 2, sg.STRASSEN_F32, sg.STRASSEN_MODE_PLAIN) == want(m, n, k, 4, 4)
        assert f(m, n, k, 2, sg.STRASSEN_F32, sg.STRASSEN_MODE_BF16X3) == want(m, n, k, 4, 4, nb=49)
        assert f(m, n, k, 2, sg.STRASSEN_BF16, sg.STRASSEN_MODE_PLAIN) == want(m, n, k, 2, 8)
        assert f(m, n, k, 1, sg.STRASSEN_F16, sg.STRASSEN_MODE_PLAIN) == \
            sg.strassen_formed_workspace_size(m, n, k, sg.STRASSEN_F16, sg.STRASSEN_MODE_PLAIN)
    assert f(-1, 1, 1, 2, 0, 0) == -1
    assert f(1, 1, -1, 2, 0, 0) == -3
    assert f(1, 1, 1, -1, 0, 0) == -4
    assert f(1, 1, 1, 3, 0, 0) == -4
    # level 0: nothing formed in the PLAIN mode, pre-split copies of A and B in BF16X3
    assert f(1000, 900, 700, 0, sg.STRASSEN_F32, sg.STRASSEN_MODE_PLAIN) == 0
    assert f(1000, 900, 700, 0, sg.STRASSEN_BF16, sg.STRASSEN_MODE_PLAIN) == 0
    assert f(1000, 900, 701, 0, sg.STRASSEN_F32, sg.STRASSEN_MODE_BF16X3) == 4 * (1000 * 704 + 704 * 900)
    assert f(1, 1, 1, 2, 7, 0) == -5
    assert f(1, 1, 1, 2, sg.STRASSEN_BF16, sg.STRASSEN_MODE_BF16X3) == -6


def test_formed_ex_validation():
    need = sg.strassen_formed_workspace_size_ex(64, 64, 64, 2, 0, 0)
    A, B, C, W = 1 << 20, 1 << 22, 1 << 24, 1 << 26
    names = ["m", "n", "k", "A", "lda", "a_type", "B", "ldb", "b_type", "C", "ldc", "alpha",
             "beta", "levels", "mode", "ws", "wsb", "stream"]
    base = dict(zip(names, [64, 64, 64, A, 64, 0, B, 64, 0, C, 64, 1.0, 1.0, 2, 0, W, need, None]))

    def call(**kw):
        return sg.strassen_gemm_formed_ex(*dict(base, **kw).values())

    assert call(m=-1) == -1
    assert call(A=None) == -4
    assert call(b_type=1) == -9
    assert call(ldc=3) == -11
    assert call(levels=-1) == -14
    assert call(levels=3) == -14
    assert call(mode=4) == -15
    assert call(ws=None) == -16
    assert call(wsb=need - 1) == -17
    assert call(ws=C + 256) == -16        # workspace overlaps C


def test_formed_validation():
    need = sg.strassen_formed_workspace_size(64, 64, 64, 0, 0)
    A, B, C, W = 1 << 20, 1 << 22, 1 << 24, 1 << 26
    names = ["m", "n", "k", "A", "lda", "a_type", "B", "ldb", "b_type", "C", "ldc", "alpha",
             "beta", "mode", "ws", "wsb", "stream"]
    base = dict(zip(names, [64, 64, 64, A, 64, 0, B, 64, 0, C, 64, 1.0, 1.0, 0, W, need, None]))

    def call(**kw):
        return sg.strassen_gemm_formed(*dict(base, **kw).values())

    assert call(m=-1) == -1
    assert call(k=-1) == -3
    assert call(A=None) == -4
    assert call(lda=63) == -5
    assert call(a_type=5) == -6
    assert call(B=None) == -7
    assert call(ldb=3) == -8
    assert call(b_type=1) == -9
    assert call(C=None) == -10
    assert call(ldc=3) == -11
    assert call(mode=4) == -14
    assert call(mode=1, a_type=1, b_type=1) == -14
    assert call(ws=None) == -15
    assert call(ws=W + 8) == -15          # not 16-byte aligned
    assert call(wsb=need - 1) == -16
    assert call(ws=C + 256) == -15        # workspace overlaps C
    assert call(ws=A - 64) == -15         # workspace overlaps A
    assert call(C=A + 128) == -10         # A overlaps C
    assert call(m=0, A=None, B=None, C=None, ws=None) == 0
    assert call(n=0, A=None, B=None, C=None, ws=None) == 0


def test_build_id_matches_sources():
    """The loaded library was built from the sources in the tree (the binding
    refuses to load one that was not)."""
    assert sg.strassen_build_id() == _binding.source_id()
    assert len(sg.strassen_build_id()) == 64


def test_probe_mfma_validation():
    # argument errors return before anything is launched
    assert sg.strassen_probe_mfma(3, 0, 10, 1, 1 << 20) == -1
    assert sg.strassen_probe_mfma(0, 2, 10, 1, 1 << 20) == -2
    assert sg.strassen_probe_mfma(0, 0, -1, 1, 1 << 20) == -3
    assert sg.strassen_probe_mfma(0, 0, 10, 0, 1 << 20) == -4
    assert sg.strassen_probe_mfma(0, 0, 10, 1, None) == -5
