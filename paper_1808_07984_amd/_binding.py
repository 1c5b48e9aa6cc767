"""ctypes binding of libstrassen.so: the C ABI of include/strassen.h with the
same names, argument marshalling only.

The library must have been built (``python paper_1808_07984_amd/build.py`` or
``__graft_entry__.build()``); importing this module without it raises, there
is no fallback path.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libstrassen.so")

# strassen_dtype_t / strassen_mode_t
STRASSEN_F32, STRASSEN_BF16, STRASSEN_F16 = 0, 1, 2
STRASSEN_MODE_PLAIN, STRASSEN_MODE_BF16X3 = 0, 1
STRASSEN_MAX_LEVELS = 2


class strassen_plan_info_t(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("blocks_per_dim", ctypes.c_int32),
        ("sub_m", ctypes.c_int64),
        ("sub_n", ctypes.c_int64),
        ("sub_k", ctypes.c_int64),
        ("n_instances", ctypes.c_int32),
        ("n_launches", ctypes.c_int32),
        ("tile_m", ctypes.c_int32),
        ("tile_n", ctypes.c_int32),
        ("tile_k", ctypes.c_int32),
        ("workgroups_per_instance", ctypes.c_int32),
        ("executed_flops", ctypes.c_double),
        ("classical_flops", ctypes.c_double),
    ]


class strassen_instance_t(ctypes.Structure):
    _fields_ = [
        ("launch", ctypes.c_int32),
        ("n_a", ctypes.c_int32),
        ("n_b", ctypes.c_int32),
        ("n_c", ctypes.c_int32),
        ("a_block", ctypes.c_int32 * 4),
        ("a_sign", ctypes.c_int32 * 4),
        ("b_block", ctypes.c_int32 * 4),
        ("b_sign", ctypes.c_int32 * 4),
        ("c_block", ctypes.c_int32 * 4),
        ("c_sign", ctypes.c_int32 * 4),
        ("c_first", ctypes.c_int32 * 4),
    ]


class strassen_launch_record_t(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_char * 64),
        ("launch", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("workgroups", ctypes.c_int32),
        ("ms", ctypes.c_float),
        ("flops", ctypes.c_double),
    ]


# Exported functions and their signatures, in header order.
_i64, _int, _f32, _vp = ctypes.c_int64, ctypes.c_int, ctypes.c_float, ctypes.c_void_p
SIGNATURES = {
    "strassen_gemm": (_int, [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _f32, _f32, _int]),
    "strassen_gemm_ex": (_int, [_i64, _i64, _i64, _vp, _i64, _int, _int, _vp, _i64, _int, _int,
                                _vp, _i64, _f32, _f32, _int, _int, _vp]),
    "strassen_gemm_hybrid": (_int, [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _f32, _f32,
                                    _vp, _i64, _vp]),
    "strassen_hybrid_workspace_size": (_i64, [_i64, _i64, _i64]),
    "strassen_gemm_formed": (_int, [_i64, _i64, _i64, _vp, _i64, _int, _vp, _i64, _int, _vp, _i64,
                                    _f32, _f32, _int, _vp, _i64, _vp]),
    "strassen_formed_workspace_size": (_i64, [_i64, _i64, _i64, _int, _int]),
    "strassen_gemm_formed_ex": (_int, [_i64, _i64, _i64, _vp, _i64, _int, _vp, _i64, _int, _vp, _i64,
                                       _f32, _f32, _int, _int, _vp, _i64, _vp]),
    "strassen_formed_workspace_size_ex": (_i64, [_i64, _i64, _i64, _int, _int, _int]),
    "strassen_gemm_formed_noalloc": (_int, [_i64, _i64, _i64, _vp, _i64, _int, _vp, _i64, _int, _vp,
                                            _i64, _f32, _f32, _int, _vp]),
    "strassen_set_stream": (_int, [_vp]),
    "strassen_set_tile": (_int, [_int]),
    "strassen_set_schedule": (_int, [_int]),
    "strassen_plan_info": (_int, [_i64, _i64, _i64, _int, _int, _int,
                                  ctypes.POINTER(strassen_plan_info_t)]),
    "strassen_plan_instances": (_int, [_int, ctypes.POINTER(strassen_instance_t), _int]),
    "strassen_error_string": (ctypes.c_char_p, [_int]),
    "strassen_build_id": (ctypes.c_char_p, []),
    "strassen_profile_start": (_int, []),
    "strassen_profile_stop": (_int, [ctypes.POINTER(strassen_launch_record_t), _int]),
    "strassen_probe_mfma": (_int, [_int, _int, _i64, ctypes.c_int32, _vp, _vp]),
}


def _hip_runtimes():
    """Distinct libamdhip64 files mapped into this process (Linux)."""
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln and "/" in ln})
    except OSError:
        return []


def check_single_hip_runtime():
    """A process must hold one HIP runtime: a second copy cannot open the GPU
    and reports "no ROCm-capable device".  Raises if two are mapped."""
    libs = _hip_runtimes()
    if len(libs) > 1:
        raise RuntimeError("two HIP runtimes are loaded (%s); import torch before this "
                           "package so libstrassen.so binds to torch's runtime" % ", ".join(libs))


def _load():
    # torch ships its own libamdhip64 (soname libamdhip64.so.7) and loads it by
    # the unversioned name.  Importing torch first makes the dynamic linker
    # resolve libstrassen.so's libamdhip64.so.7 to that same copy.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libstrassen.so is not built (%s); run `python paper_1808_07984_amd/build.py`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    check_single_hip_runtime()
    built = lib.strassen_build_id().decode()
    want = source_id()
    if want is not None and built != want:
        raise ImportError("libstrassen.so (%s) was built from other sources than those in %s (%s): "
                          "rebuild with `python paper_1808_07984_amd/build.py`"
                          % (built[:12], os.path.join(_HERE, "csrc"), want[:12]))
    return lib


def source_id():
    """The build id of the sources beside this file (same rule as
    build.source_id), or None when they are not shipped."""
    import hashlib
    csrc = os.path.join(_HERE, "csrc")
    include = os.path.join(os.path.dirname(_HERE), "include")
    if not (os.path.isdir(csrc) and os.path.isdir(include)):
        return None
    h = hashlib.sha256()
    for d in (csrc, include):
        for name in sorted(os.listdir(d)):
            if name.endswith((".hip", ".cpp", ".hpp", ".h")):
                h.update(name.encode())
                with open(os.path.join(d, name), "rb") as f:
                    h.update(f.read())
    return h.hexdigest()


lib = _load()


class StrassenError(RuntimeError):
    """A non-zero return code of the C ABI."""

    def __init__(self, code, where):
        self.code = code
        super().__init__("%s returned %d: %s" % (where, code, strassen_error_string(code)))


def strassen_gemm(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta, levels):
    return lib.strassen_gemm(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta, levels)


def strassen_gemm_ex(m, n, k, A, lda, a_type, trans_a, B, ldb, b_type, trans_b, C, ldc,
                     alpha, beta, levels, mode, hip_stream):
    return lib.strassen_gemm_ex(m, n, k, A, lda, a_type, trans_a, B, ldb, b_type, trans_b,
                                C, ldc, alpha, beta, levels, mode, hip_stream)


def strassen_gemm_hybrid(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta, workspace,
                         workspace_bytes, hip_stream):
    return lib.strassen_gemm_hybrid(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta, workspace,
                                    workspace_bytes, hip_stream)


def strassen_hybrid_workspace_size(m, n, k):
    return lib.strassen_hybrid_workspace_size(m, n, k)


def strassen_gemm_formed(m, n, k, A, lda, a_type, B, ldb, b_type, C, ldc, alpha, beta, mode,
                         workspace, workspace_bytes, hip_stream):
    return lib.strassen_gemm_formed(m, n, k, A, lda, a_type, B, ldb, b_type, C, ldc, alpha, beta,
                                    mode, workspace, workspace_bytes, hip_stream)


STRASSEN_NOALLOC_SCRATCH_BYTES = 256 << 20
STRASSEN_ERROR_SCRATCH_LIMIT = 0x5C00


def strassen_gemm_formed_noalloc(m, n, k, A, lda, a_type, B, ldb, b_type, C, ldc, alpha, beta, mode,
                                 hip_stream):
    return lib.strassen_gemm_formed_noalloc(m, n, k, A, lda, a_type, B, ldb, b_type, C, ldc, alpha,
                                            beta, mode, hip_stream)


def strassen_formed_workspace_size(m, n, k, dtype=STRASSEN_F32, mode=STRASSEN_MODE_PLAIN):
    return lib.strassen_formed_workspace_size(m, n, k, dtype, mode)


def strassen_gemm_formed_ex(m, n, k, A, lda, a_type, B, ldb, b_type, C, ldc, alpha, beta, levels, mode,
                            workspace, workspace_bytes, hip_stream):
    return lib.strassen_gemm_formed_ex(m, n, k, A, lda, a_type, B, ldb, b_type, C, ldc, alpha, beta,
                                       levels, mode, workspace, workspace_bytes, hip_stream)


def strassen_formed_workspace_size_ex(m, n, k, levels=1, dtype=STRASSEN_F32, mode=STRASSEN_MODE_PLAIN):
    return lib.strassen_formed_workspace_size_ex(m, n, k, levels, dtype, mode)


def strassen_set_stream(hip_stream):
    return lib.strassen_set_stream(hip_stream)


STRASSEN_TILE_AUTO, STRASSEN_TILE_128, STRASSEN_TILE_256 = 0, 1, 2


def strassen_set_tile(tile):
    return lib.strassen_set_tile(tile)


STRASSEN_SCHEDULE_BATCHED, STRASSEN_SCHEDULE_CONCURRENT, STRASSEN_SCHEDULE_STREAMS = 0, 1, 2


def strassen_set_schedule(schedule):
    return lib.strassen_set_schedule(schedule)


def strassen_plan_info(m, n, k, levels, dtype=STRASSEN_F32, mode=STRASSEN_MODE_PLAIN):
    """Returns (code, strassen_plan_info_t)."""
    out = strassen_plan_info_t()
    rc = lib.strassen_plan_info(m, n, k, levels, dtype, mode, ctypes.byref(out))
    return rc, out


def strassen_plan_instances(levels, capacity=None):
    """Returns (count_or_code, list of strassen_instance_t)."""
    if capacity is None:
        capacity = 7 ** max(0, min(int(levels), STRASSEN_MAX_LEVELS))
    buf = (strassen_instance_t * max(capacity, 1))()
    rc = lib.strassen_plan_instances(levels, buf, capacity)
    return rc, list(buf[:max(0, min(rc, capacity))])


def strassen_error_string(code):
    s = lib.strassen_error_string(code)
    return s.decode() if s else ""


def strassen_build_id():
    return lib.strassen_build_id().decode()


def strassen_profile_start():
    return lib.strassen_profile_start()


def strassen_profile_stop(capacity=4096):
    """Returns (count_or_code, list of strassen_launch_record_t)."""
    buf = (strassen_launch_record_t * max(capacity, 1))()
    rc = lib.strassen_profile_stop(buf, capacity)
    return rc, list(buf[:max(0, min(rc, capacity))])


def strassen_probe_mfma(op, random, iters, workgroups, out, hip_stream=None):
    return lib.strassen_probe_mfma(op, random, iters, workgroups, out, hip_stream)
