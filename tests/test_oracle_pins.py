"""Pins for the CPU oracle: facts fixed by the paper and by mathematics, not by
the oracle itself.

* basis brute force: for bilinear maps, agreeing with A@B on every pair of
  matrix units E_ab, E_cd is the same as satisfying the Brent equations of
  the scheme, so a dropped term, a wrong sign or a wrong quadrant index in the
  oracle's copy of the seven products (Method section, eq. gpu_allops) fails;
* exact equality with the classical product on integer inputs, also for odd
  and rectangular sizes (zero padding, Fringes section) and three levels;
* the classical definition against a textbook library product (numpy) on
  rectangular shapes, which catches transposed operands;
* closed-form special cases of C = alpha*A*B + beta*C (Introduction, eq.
  prime) and the BLAS conventions for alpha = 0, beta = 0, k = 0;
* the binary32 emulation against numpy's binary32 arithmetic;
* planted mistakes: mutated copies of oracle.c, built on the CPU, must each
  fail at least one of these pins.
"""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ints(rng, r, c, lo=-3, hi=3):
    return rng.integers(lo, hi + 1, size=(r, c)).astype(np.float64)


def _unit(r, c, a, b):
    e = np.zeros((r, c))
    e[a, b] = 1.0
    return e


@pytest.mark.parametrize("levels,dim", [(1, 2), (2, 4), (1, 3), (2, 5)])
def test_basis_brute_force(levels, dim):
    """Strassen on every pair of matrix units equals the classical product:
    the bilinear identities of the scheme hold (2x2 and, by recursion, 4x4;
    odd dims exercise the zero padding)."""
    for a in range(dim):
        for b in range(dim):
            A = _unit(dim, dim, a, b)
            for c in range(dim):
                for d in range(dim):
                    B = _unit(dim, dim, c, d)
                    got = oracle.strassen(A, B, levels=levels)
                    assert np.array_equal(got, A @ B), (levels, dim, a, b, c, d)


def test_basis_brute_force_rectangular():
    """Unit-matrix pairs on a 4x2 @ 2x6 product at two levels."""
    m, k, n = 4, 2, 6
    for a in range(m):
        for b in range(k):
            A = _unit(m, k, a, b)
            for c in range(k):
                for d in range(n):
                    B = _unit(k, n, c, d)
                    assert np.array_equal(oracle.strassen(A, B, levels=2), A @ B)


SHAPES = [(1, 1, 1), (2, 2, 2), (3, 2, 5), (7, 5, 9), (33, 17, 65), (64, 64, 64),
          (50, 1, 3), (1, 40, 7), (13, 31, 1)]


@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("levels", [1, 2, 3])
def test_strassen_exact_on_integers(m, n, k, levels):
    rng = np.random.default_rng(1000 * m + 10 * n + k)
    A, B, C = _ints(rng, m, k), _ints(rng, k, n), _ints(rng, m, n)
    want = A @ B + 2.0 * C
    got = oracle.strassen(A, B, C, alpha=1.0, beta=2.0, levels=levels)
    assert np.array_equal(got, want)
    assert np.array_equal(oracle.gemm_f64(A, B, C, 1.0, 2.0), want)


@pytest.mark.parametrize("m,n,k", [(5, 7, 3), (31, 17, 64), (64, 48, 80), (1, 9, 4)])
def test_classical_matches_library(m, n, k):
    """Classical definition vs numpy's product (a textbook routine) on
    rectangular real inputs; also the f64 Strassen within rounding."""
    rng = np.random.default_rng(7)
    A, B, C = rng.uniform(-1, 1, (m, k)), rng.uniform(-1, 1, (k, n)), rng.uniform(-1, 1, (m, n))
    want = 1.5 * (A @ B) + 0.5 * C
    np.testing.assert_allclose(oracle.gemm_f64(A, B, C, 1.5, 0.5), want, rtol=0, atol=1e-13 * k)
    for L in (1, 2):
        np.testing.assert_allclose(oracle.strassen(A, B, C, 1.5, 0.5, levels=L), want,
                                   rtol=0, atol=1e-12 * k)


def test_alpha_beta_half_integers_exact():
    rng = np.random.default_rng(3)
    A, B, C = _ints(rng, 9, 11), _ints(rng, 11, 6), _ints(rng, 9, 6)
    want = 1.5 * (A @ B) + 0.5 * C
    for L in (0, 1, 2):
        assert np.array_equal(oracle.strassen(A, B, C, 1.5, 0.5, levels=L), want)
    assert np.array_equal(oracle.gemm_f64(A, B, C, 1.5, 0.5), want)


def test_special_cases():
    rng = np.random.default_rng(5)
    A, B, C = _ints(rng, 6, 4), _ints(rng, 4, 5), _ints(rng, 6, 5)
    # k = 0: C := beta * C
    A0, B0 = np.zeros((6, 0)), np.zeros((0, 5))
    for f in (lambda *a, **k: oracle.gemm_f64(*a, **k),
              lambda *a, **k: oracle.strassen(*a, levels=2, **k)):
        assert np.array_equal(f(A0, B0, C, alpha=1.0, beta=3.0), 3.0 * C)
        # alpha = 0: A and B are not read (NaN there does not propagate)
        An = A.copy()
        An[0, 0] = np.nan
        assert np.array_equal(f(An, B, C, alpha=0.0, beta=0.5), 0.5 * C)
        # beta = 0: C is write-only
        Cn = np.full_like(C, np.nan)
        assert np.array_equal(f(A, B, Cn, alpha=1.0, beta=0.0), A @ B)
    # empty outputs
    assert oracle.gemm_f64(np.zeros((0, 3)), np.zeros((3, 4))).shape == (0, 4)
    assert oracle.strassen(np.zeros((3, 2)), np.zeros((2, 0)), levels=1).shape == (3, 0)


def test_gemm_entries_matches_dot():
    rng = np.random.default_rng(11)
    A, B, C = _ints(rng, 40, 30), _ints(rng, 30, 20), _ints(rng, 40, 20)
    rows, cols = rng.integers(0, 40, 25), rng.integers(0, 20, 25)
    got = oracle.gemm_entries(A, B, C, rows, cols, alpha=-1.0, beta=2.0)
    want = np.array([-np.dot(A[i], B[:, j]) + 2 * C[i, j] for i, j in zip(rows, cols)])
    assert np.array_equal(got, want)


def test_f32emu_level0_matches_binary32_serial_sum():
    """At zero levels the emulation is a serial binary32 dot product: numpy's
    float32 arithmetic (one rounding per product and per sum) reproduces it."""
    rng = np.random.default_rng(13)
    m, n, k = 5, 7, 33
    A = rng.uniform(-1, 1, (m, k)).astype(np.float32)
    B = rng.uniform(-1, 1, (k, n)).astype(np.float32)
    acc = np.zeros((m, n), dtype=np.float32)
    for l in range(k):
        acc = acc + np.outer(A[:, l], B[l, :]).astype(np.float32)
    got = oracle.strassen(A, B, levels=0, f32emu=True)
    assert np.array_equal(got, acc.astype(np.float64))


def test_f32emu_one_level_matches_binary32_scheme():
    """One level in numpy float32, built from the fixture of eq. gpu_allops
    (not from the oracle's own table), equals the emulation bit for bit."""
    from conftest import parse_scheme
    rng = np.random.default_rng(17)
    h = 6
    A = rng.uniform(-1, 1, (2 * h, 2 * h)).astype(np.float32)
    B = rng.uniform(-1, 1, (2 * h, 2 * h)).astype(np.float32)

    def quad(X, q):
        r, c = divmod(q, 2)
        return X[r * h:(r + 1) * h, c * h:(c + 1) * h]

    def serial(P, Q):
        acc = np.zeros((h, h), dtype=np.float32)
        for l in range(h):
            acc = acc + np.outer(P[:, l], Q[l, :]).astype(np.float32)
        return acc

    Cq = [np.zeros((h, h), dtype=np.float32) for _ in range(4)]
    for _, at, bt, ct in parse_scheme():
        P = np.float32(at[0][1]) * quad(A, at[0][0])
        for q, s in at[1:]:
            P = P + np.float32(s) * quad(A, q)
        Q = np.float32(bt[0][1]) * quad(B, bt[0][0])
        for q, s in bt[1:]:
            Q = Q + np.float32(s) * quad(B, q)
        M = serial(P, Q)
        for q, s in ct:
            Cq[q] = Cq[q] + np.float32(s) * M
    want = np.block([[Cq[0], Cq[1]], [Cq[2], Cq[3]]]).astype(np.float64)
    got = oracle.strassen(A, B, levels=1, f32emu=True)
    assert np.array_equal(got, want)


def test_f32emu_error_within_classical_bound():
    """fp32 rounding of the scheme stays inside k * 2^-23 * |A|max |B|max times
    the level factor used by the parity tests."""
    rng = np.random.default_rng(19)
    n = 256
    A = rng.uniform(-1, 1, (n, n)).astype(np.float32)
    B = rng.uniform(-1, 1, (n, n)).astype(np.float32)
    exact = oracle.gemm_f64(A, B)
    for L in (0, 1, 2):
        err = np.abs(oracle.strassen(A, B, levels=L, f32emu=True) - exact).max()
        e_norm = err / (2.0 ** -23 * n)
        assert 0 < e_norm <= 2 ** (L + 1) / 2, (L, e_norm)


# ---------------------------------------------------------------------------
# Planted mistakes: each mutant of oracle.c must fail a pin.
# ---------------------------------------------------------------------------

MUTANTS = {
    # wrong sign in M3's right factor (B2 + B0 instead of B2 - B0)
    "sign": ("{1, {3, 0}, {+1, 0}, 2, {2, 0}, {+1, -1}",
             "{1, {3, 0}, {+1, 0}, 2, {2, 0}, {+1, +1}"),
    # M0 dropped from C3
    "dropped_output": ("{2, {0, 3}, {+1, +1}, 2, {0, 3}, {+1, +1}, 2, {0, 3}, {+1, +1}}",
                       "{2, {0, 3}, {+1, +1}, 2, {0, 3}, {+1, +1}, 1, {0, 3}, {+1, +1}}"),
    # wrong quadrant index in M6's left factor
    "index": ("{2, {1, 3}, {+1, -1}, 2, {2, 3}", "{2, {1, 2}, {+1, -1}, 2, {2, 3}"),
    # dropped term of M5's left factor
    "dropped_term": ("{2, {2, 0}, {+1, -1}, 2, {0, 1}", "{1, {2, 0}, {+1, -1}, 2, {0, 1}"),
    # transposed A in the classical kernel
    "transpose": ("const double a = A[i * lda + l];\n            const double *b = B + l * ldb;\n            for (i64 j = 0; j < n; ++j)\n                c[j]",
                  "const double a = A[l * lda + i];\n            const double *b = B + l * ldb;\n            for (i64 j = 0; j < n; ++j)\n                c[j]"),
    # padding quadrant origin off by one
    "padding": ("const i64 r0 = (i64)(q / 2) * hr, c0", "const i64 r0 = (i64)(q / 2) * (hr - (hr > 1)), c0"),
}

_PIN_SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, %(root)r)
import oracle
rng = np.random.default_rng(0)
def ints(r, c): return rng.integers(-3, 4, size=(r, c)).astype(float)
bad = 0
for L, dim in ((1, 2), (2, 4)):
    for a in range(dim * dim):
        for c in range(dim * dim):
            A = np.zeros((dim, dim)); A.flat[a] = 1
            B = np.zeros((dim, dim)); B.flat[c] = 1
            bad |= not np.array_equal(oracle.strassen(A, B, levels=L), A @ B)
for (m, n, k) in ((7, 5, 9), (33, 17, 65), (6, 6, 6)):
    A, B = ints(m, k), ints(k, n)
    for L in (1, 2):
        bad |= not np.array_equal(oracle.strassen(A, B, levels=L), A @ B)
sys.exit(1 if bad else 0)
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, "mutation anchor not found: " + name
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                    str(mut), "-o", str(lib)], check=True)
    env = dict(os.environ, STRASSEN_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-c", _PIN_SCRIPT % {"root": ROOT}], env=env,
                       capture_output=True, timeout=120)
    assert r.returncode != 0, "planted mistake %r passed every pin" % name
    # and the unmutated source passes the same script
    if name == sorted(MUTANTS)[0]:
        r0 = subprocess.run([sys.executable, "-c", _PIN_SCRIPT % {"root": ROOT}],
                            capture_output=True, timeout=120)
        assert r0.returncode == 0, r0.stderr.decode()[-2000:]
