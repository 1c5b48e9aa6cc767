"""CPU oracle for Strassen-fused GEMM -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and the two share no
code: this package has its own copy of the seven-product scheme, typed from
the paper, and its own arithmetic.

What it computes (paper: Introduction eq. "prime"; Method eq. "gpu_allops")

* ``gemm_f64``       C* = alpha*A*B + beta*C by the classical definition, in
                     fp64, from the exact input values (fp32/bf16/fp16 widen
                     exactly to fp64).
* ``strassen``       the seven-product scheme applied recursively ``levels``
                     times on ceil(dim/2) quadrants with zero padding, in
                     fp64 (``f32emu=False``) or with every sum and product
                     rounded to binary32 (``f32emu=True``).
* ``gemm_entries``   single entries C*_ij of the classical definition, for
                     sampled parity checks at sizes where a full oracle
                     product is too slow.

All functions take numpy arrays or CPU torch tensors and return numpy float64.
Pins (tests/test_oracle_pins.py) tie each function to facts fixed by the
paper and by mathematics: basis-matrix brute force (the bilinear identities of
the scheme), exact equality with the classical product on integer inputs,
a textbook library product for the classical definition, closed-form
special cases, and the f32 emulation against a serial binary32 accumulation.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# STRASSEN_ORACLE_LIB lets the planted-mistake tests load a mutated build.
_LIB_PATH = os.environ.get("STRASSEN_ORACLE_LIB") or os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build  # compiles oracle.c with gcc on first use
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_gemm_f64.argtypes = [_i64, _i64, _i64, _dp, _i64, _dp, _i64,
                                    _dp, _i64, ctypes.c_double, ctypes.c_double]
    lib.oracle_gemm_f64.restype = ctypes.c_int
    lib.oracle_strassen.argtypes = [_i64, _i64, _i64, _dp, _i64, _dp, _i64,
                                    _dp, _i64, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int]
    lib.oracle_strassen.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(x):
    """Exact widening to a C-contiguous float64 numpy array."""
    try:
        import torch
        if isinstance(x, torch.Tensor):
            x = x.detach().to("cpu", torch.float64).numpy()
    except ImportError:  # pragma: no cover
        pass
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _prep(A, B, C, beta):
    A = _f64(A)
    B = _f64(B)
    m, k = A.shape
    k2, n = B.shape
    if k2 != k:
        raise ValueError("inner dimensions differ: %d vs %d" % (k, k2))
    if C is None:
        if beta != 0.0:
            raise ValueError("C is required when beta != 0")
        Cout = np.zeros((m, n), dtype=np.float64)
    else:
        Cout = _f64(C).copy()
        if Cout.shape != (m, n):
            raise ValueError("C has shape %s, expected %s" % (Cout.shape, (m, n)))
    # zero-extent arrays still need a valid pointer
    if A.size == 0:
        A = np.zeros((max(m, 1), max(k, 1)))
    if B.size == 0:
        B = np.zeros((max(k, 1), max(n, 1)))
    return A, B, Cout, m, n, k


def gemm_f64(A, B, C=None, alpha=1.0, beta=0.0):
    """C* = alpha * A @ B + beta * C, classical definition in fp64."""
    A, B, Cout, m, n, k = _prep(A, B, C, beta)
    if m == 0 or n == 0:
        return Cout
    rc = _load().oracle_gemm_f64(m, n, k, _ptr(A), A.shape[1], _ptr(B), B.shape[1],
                                 _ptr(Cout), n, float(alpha), float(beta))
    if rc:
        raise MemoryError("oracle_gemm_f64 failed (%d)" % rc)
    return Cout


def strassen(A, B, C=None, alpha=1.0, beta=0.0, levels=1, f32emu=False):
    """alpha * (A @ B by `levels` levels of the seven-product scheme) + beta*C."""
    if levels < 0:
        raise ValueError("levels must be >= 0")
    A, B, Cout, m, n, k = _prep(A, B, C, beta)
    if m == 0 or n == 0:
        return Cout
    if f32emu:
        for X in (A, B, Cout):
            if not np.array_equal(X, X.astype(np.float32).astype(np.float64)):
                raise ValueError("f32emu needs inputs exactly representable in binary32")
    rc = _load().oracle_strassen(m, n, k, _ptr(A), A.shape[1], _ptr(B), B.shape[1],
                                 _ptr(Cout), n, float(alpha), float(beta),
                                 int(levels), 1 if f32emu else 0)
    if rc:
        raise RuntimeError("oracle_strassen failed (%d)" % rc)
    return Cout


def gemm_entries(A, B, C, rows, cols, alpha=1.0, beta=0.0):
    """Entries C*_ij = alpha * sum_l A[i,l] B[l,j] + beta*C[i,j] for the pairs
    (rows[s], cols[s]); fp64, classical definition.  C may be None when
    beta == 0.  Only the sampled rows of A and columns of B are widened."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    a = _f64(A[rows.tolist()] if not isinstance(A, np.ndarray) else A[rows])
    b = _f64(B[:, cols.tolist()] if not isinstance(B, np.ndarray) else B[:, cols])
    dot = (a * b.T).sum(axis=1) if a.shape[1] else np.zeros(len(rows))
    out = (alpha * dot) if alpha != 0.0 else np.zeros(len(rows))
    if beta != 0.0:
        if isinstance(C, np.ndarray):
            c = C[rows, cols]
        else:
            import torch
            c = C[torch.as_tensor(rows), torch.as_tensor(cols)]
        out = out + beta * _f64(c)
    return out
