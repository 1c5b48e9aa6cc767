"""Differentiation: StrassenMatmul's backward (dA = dC B^T, dB = A^T dC,
through the transposed-operand kernels) against the classical gradient from
the fp64 oracle and a finite-difference check of the bilinear map (torch's
gradcheck is not used: in fp32 its finite differences are too coarse to pin
anything the oracle gradient does not).  Shapes: 64x48x80 (gradient checks) and the two
differentiation workloads (4096^3 and 8192x2048x6144, sampled entries)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1808_07984_amd as sg
from paper_1808_07984_amd import inputs
from parity import EPS, tau

pytestmark = pytest.mark.gpu


def _grads(m, n, k, levels, mode="plain"):
    A = inputs.uniform(m, k, inputs.SEED_A)
    B = inputs.uniform(k, n, inputs.SEED_B)
    dC = inputs.normal(m, n, inputs.SEED_DC)
    Ad = A.cuda().requires_grad_(True)
    Bd = B.cuda().requires_grad_(True)
    C = sg.strassen_matmul(Ad, Bd, levels, mode)
    C.backward(dC.cuda())
    torch.cuda.synchronize()
    return A, B, dC, C.detach(), Ad.grad, Bd.grad


def _check(got, want, k, xmax, ymax, levels, eps=EPS["f32"]):
    err = float(np.abs(got - want).max())
    en = err / (eps * k * xmax * ymax)
    print("e_norm %.4f (tau %g)" % (en, tau(levels)), flush=True)
    assert en <= tau(levels)


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_backward_matches_classical_gradient(levels):
    m, n, k = 64, 48, 80
    A, B, dC, C, dA, dB = _grads(m, n, k, levels)
    _check(C.cpu().double().numpy(), oracle.gemm_f64(A, B), k, 1, 1, levels)
    # dA = dC B^T (inner dim n), dB = A^T dC (inner dim m)
    _check(dA.cpu().double().numpy(), oracle.gemm_f64(dC, B.t()), n,
           float(dC.abs().max()), 1, levels)
    _check(dB.cpu().double().numpy(), oracle.gemm_f64(A.t(), dC), m, 1,
           float(dC.abs().max()), levels)


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_finite_difference_of_bilinear_map(levels):
    """C is bilinear, so (f(A+V, B) - f(A-V, B)) / 2 = V B exactly: the
    directional derivative <dC, V B> must equal <dA, V> (and likewise for B)."""
    m, n, k = 64, 48, 80
    A, B, dC, C, dA, dB = _grads(m, n, k, levels)
    V = inputs.uniform(m, k, 11).cuda()
    W = inputs.uniform(k, n, 12).cuda()
    Ad, Bd, dCd = A.cuda(), B.cuda(), dC.cuda()
    fd_a = (sg.strassen_matmul(Ad + V, Bd, levels) - sg.strassen_matmul(Ad - V, Bd, levels)) / 2
    fd_b = (sg.strassen_matmul(Ad, Bd + W, levels) - sg.strassen_matmul(Ad, Bd - W, levels)) / 2
    lhs_a = float((dCd.double() * fd_a.double()).sum())
    rhs_a = float((dA.double() * V.double()).sum())
    lhs_b = float((dCd.double() * fd_b.double()).sum())
    rhs_b = float((dB.double() * W.double()).sum())
    scale = float(dCd.abs().sum()) * k * 2 * EPS["f32"] * tau(levels)
    assert abs(lhs_a - rhs_a) <= scale, (lhs_a, rhs_a)
    assert abs(lhs_b - rhs_b) <= scale, (lhs_b, rhs_b)


@pytest.mark.parametrize("m,n,k", [(4096, 4096, 4096), (8192, 2048, 6144)])
@pytest.mark.parametrize("levels", [1, 2])
def test_differentiation_workloads_sampled(m, n, k, levels):
    A, B, dC, C, dA, dB = _grads(m, n, k, levels)
    rng = np.random.default_rng(levels)
    r, c = rng.integers(0, m, 200), rng.integers(0, k, 200)
    want = oracle.gemm_entries(dC, B.t(), None, r, c)
    got = dA[torch.as_tensor(r, device="cuda"), torch.as_tensor(c, device="cuda")].double().cpu().numpy()
    _check(got, want, n, float(dC.abs().max()), 1, levels)
    r, c = rng.integers(0, k, 200), rng.integers(0, n, 200)
    want = oracle.gemm_entries(A.t(), dC, None, r, c)
    got = dB[torch.as_tensor(r, device="cuda"), torch.as_tensor(c, device="cuda")].double().cpu().numpy()
    _check(got, want, m, 1, float(dC.abs().max()), levels)


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_backward_bf16x3_mode(levels):
    """The compensated mode differentiates through the same transposed
    kernels; gradients within the bf16x3 gate (eps 2^-16)."""
    m, n, k = 64, 48, 80
    A, B, dC, C, dA, dB = _grads(m, n, k, levels, mode="bf16x3")
    eps = 2.0 ** -16
    _check(C.cpu().double().numpy(), oracle.gemm_f64(A, B), k, 1, 1, levels, eps)
    _check(dA.cpu().double().numpy(), oracle.gemm_f64(dC, B.t()), n,
           float(dC.abs().max()), 1, levels, eps)
    _check(dB.cpu().double().numpy(), oracle.gemm_f64(A.t(), dC), m, 1,
           float(dC.abs().max()), levels, eps)
