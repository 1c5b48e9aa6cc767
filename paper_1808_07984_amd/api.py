"""torch-facing convenience layer over the C ABI.

torch supplies device memory and the current stream only: ``gemm`` checks
shapes, dtypes, devices and strides, passes raw pointers and leading
dimensions to ``strassen_gemm_ex`` and raises on a non-zero code.  All
arithmetic happens in the HIP kernels of libstrassen.so.
"""
import torch

from . import _binding as B

_DTYPES = {torch.float32: B.STRASSEN_F32, torch.bfloat16: B.STRASSEN_BF16,
           torch.float16: B.STRASSEN_F16}
_MODES = {"plain": B.STRASSEN_MODE_PLAIN, "bf16x3": B.STRASSEN_MODE_BF16X3}


def _ld(t, name):
    if t.dim() != 2:
        raise ValueError("%s must be 2-D" % name)
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError("%s must have unit stride along its second dimension" % name)
    return max(t.stride(0), 1) if t.shape[0] > 1 else max(t.shape[1], 1)


def gemm(A, B_, C, alpha=1.0, beta=1.0, levels=1, mode="plain", trans_a=False, trans_b=False,
         stream=None):
    """C := alpha * op(A) @ op(B) + beta * C in place, with `levels` levels of
    Strassen (0 = plain blocked GEMM).  op(X) = X, or X.T when trans_x is set,
    in which case X is passed in its stored (untransposed) layout.
    A, B: fp32, bf16 or fp16 CUDA tensors of one dtype; C: fp32 CUDA tensor.
    Returns C."""
    if not (A.is_cuda and B_.is_cuda and C.is_cuda):
        raise ValueError("A, B and C must be GPU tensors")
    if not (A.device == B_.device == C.device):
        raise ValueError("A, B and C must be on one device")
    if A.dtype not in _DTYPES or B_.dtype != A.dtype:
        raise TypeError("A and B must share a dtype among float32, bfloat16, float16")
    if C.dtype != torch.float32:
        raise TypeError("C must be float32")
    if mode not in _MODES:
        raise ValueError("mode must be one of %s" % sorted(_MODES))
    m, k = (A.shape[1], A.shape[0]) if trans_a else (A.shape[0], A.shape[1])
    kb, n = (B_.shape[1], B_.shape[0]) if trans_b else (B_.shape[0], B_.shape[1])
    if kb != k or tuple(C.shape) != (m, n):
        raise ValueError("shape mismatch: op(A) %dx%d, op(B) %dx%d, C %s" % (m, k, kb, n, tuple(C.shape)))
    lda, ldb, ldc = _ld(A, "A"), _ld(B_, "B"), _ld(C, "C")
    with torch.cuda.device(C.device):
        s = stream if stream is not None else torch.cuda.current_stream(C.device)
        rc = B.strassen_gemm_ex(m, n, k, A.data_ptr(), lda, _DTYPES[A.dtype], int(bool(trans_a)),
                                B_.data_ptr(), ldb, _DTYPES[A.dtype], int(bool(trans_b)),
                                C.data_ptr(), ldc, float(alpha), float(beta), int(levels),
                                _MODES[mode], s.cuda_stream)
    if rc != 0:
        raise B.StrassenError(rc, "strassen_gemm_ex")
    return C


def plan_info(m, n, k, levels, dtype=torch.float32, mode="plain"):
    rc, info = B.strassen_plan_info(m, n, k, levels, _DTYPES[dtype], _MODES[mode])
    if rc != 0:
        raise B.StrassenError(rc, "strassen_plan_info")
    return info


def gemm_hybrid(A, B_, C, alpha=1.0, beta=1.0, workspace=None, stream=None):
    """Hybrid two-level Strassen: C := alpha * A @ B + beta * C in place, fp32.
    `workspace` is a GPU tensor of at least strassen_hybrid_workspace_size
    bytes (allocated by torch here when not given: the library itself
    allocates nothing).  Returns C."""
    for t, name in ((A, "A"), (B_, "B"), (C, "C")):
        if not t.is_cuda or t.dtype != torch.float32:
            raise TypeError("%s must be an fp32 GPU tensor" % name)
    m, k = A.shape
    kb, n = B_.shape
    if kb != k or tuple(C.shape) != (m, n):
        raise ValueError("shape mismatch")
    need = B.strassen_hybrid_workspace_size(m, n, k)
    if need < 0:
        raise B.StrassenError(int(need), "strassen_hybrid_workspace_size")
    if workspace is None:
        workspace = torch.empty(max(need, 16), dtype=torch.uint8, device=C.device)
    if workspace.numel() * workspace.element_size() < need:
        raise ValueError("workspace smaller than %d bytes" % need)
    with torch.cuda.device(C.device):
        s = stream if stream is not None else torch.cuda.current_stream(C.device)
        rc = B.strassen_gemm_hybrid(m, n, k, A.data_ptr(), _ld(A, "A"), B_.data_ptr(), _ld(B_, "B"),
                                    C.data_ptr(), _ld(C, "C"), float(alpha), float(beta),
                                    workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                    s.cuda_stream)
    if rc != 0:
        raise B.StrassenError(rc, "strassen_gemm_hybrid")
    return C


def formed_workspace_bytes(m, n, k, dtype=torch.float32, mode="plain", levels=1):
    """Bytes of workspace gemm_formed needs for this shape, dtype, mode and
    number of levels."""
    need = B.strassen_formed_workspace_size_ex(m, n, k, levels, _DTYPES[dtype], _MODES[mode])
    if need < 0:
        raise B.StrassenError(int(need), "strassen_formed_workspace_size_ex")
    return need


def gemm_formed(A, B_, C, alpha=1.0, beta=1.0, mode="plain", workspace=None, stream=None, levels=1):
    """One- or two-level Strassen with the multi-term operand sums formed
    first into workspace: C := alpha * A @ B + beta * C in place (levels=0:
    the plain product, on pre-split copies of A and B in the bf16x3 mode).
    Equal to gemm(..., levels=levels) bit for bit, except that at one level on the
    16-bit matrix cores with 256x256 tiles the products M5 and M6 are
    accumulated after M2 and M3 and added into C3 and C0 with them, so those
    two blocks can differ in the last bits.  A, B: fp32, bf16 or fp16 GPU tensors of one dtype,
    as stored (no transposes); C fp32.  `workspace` is a GPU tensor of at
    least formed_workspace_bytes(...) bytes (allocated by torch here when not
    given: the library itself allocates nothing).  Returns C."""
    if not (A.is_cuda and B_.is_cuda and C.is_cuda):
        raise ValueError("A, B and C must be GPU tensors")
    if A.dtype not in _DTYPES or B_.dtype != A.dtype:
        raise TypeError("A and B must share a dtype among float32, bfloat16, float16")
    if C.dtype != torch.float32:
        raise TypeError("C must be float32")
    if mode not in _MODES:
        raise ValueError("mode must be one of %s" % sorted(_MODES))
    m, k = A.shape
    kb, n = B_.shape
    if kb != k or tuple(C.shape) != (m, n):
        raise ValueError("shape mismatch: A %s, B %s, C %s" % (tuple(A.shape), tuple(B_.shape), tuple(C.shape)))
    need = formed_workspace_bytes(m, n, k, A.dtype, mode, levels)
    if workspace is None:
        workspace = torch.empty(max(need, 16), dtype=torch.uint8, device=C.device)
    wbytes = workspace.numel() * workspace.element_size()
    if wbytes < need:
        raise ValueError("workspace smaller than %d bytes" % need)
    with torch.cuda.device(C.device):
        s = stream if stream is not None else torch.cuda.current_stream(C.device)
        rc = B.strassen_gemm_formed_ex(m, n, k, A.data_ptr(), _ld(A, "A"), _DTYPES[A.dtype],
                                       B_.data_ptr(), _ld(B_, "B"), _DTYPES[A.dtype],
                                       C.data_ptr(), _ld(C, "C"), float(alpha), float(beta), int(levels),
                                       _MODES[mode], workspace.data_ptr(), wbytes, s.cuda_stream)
    if rc != 0:
        raise B.StrassenError(rc, "strassen_gemm_formed_ex")
    return C
