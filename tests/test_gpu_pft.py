"""GPU parity of the partial transform (pft2d_forward / pft2d_adjoint)
against the FP64 oracle, through the C ABI.

Tolerance (FP32 path): relative L2 error <= 1e-5 over each call's output,
and every patch's own relative L2 error <= 3e-5.  Derivation: each output
is a sum of n^2 products of O(1) terms formed in two float stages; the
rounding error of a length-K float dot product with random signs grows like
sqrt(K) * 2^-24 relative to the output's own scale, i.e. ~1e-6 at K = 256
per stage, so 1e-5 leaves a margin of several times over two stages.
"""

import numpy as np
import pytest
import torch

import workloads
from oracle import pft as opft

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOL_PATCH = 3e-5
# split hi+lo operands: products hi*hi + hi*lo + lo*hi leave the lo*lo term
# and the 16-bit rounding of the lo parts, ~2^-16 (bf16, 8-bit significand)
# or ~2^-22 (fp16, 11-bit) relative per operand, times the growth over the
# two stages: bf16 lands near 5e-6, fp16 near 1e-7.
TOLS = {"fp32": (1e-5, 3e-5), "split_bf16": (1e-4, 3e-4), "split_fp16": (1e-5, 3e-5)}
PRECS = sorted(TOLS)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def per_patch_rel(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


@pytest.fixture(scope="module")
def pkg():
    import paper_2408_03532_amd as p
    p.lib()
    return p


SHAPES = [(32, 16, 5), (64, 16, 3), (40, 24, 4), (17, 5, 3), (128, 32, 4), (256, 64, 3),
          (128, 128, 2), (512, 128, 2), (48, 48, 2), (1, 1, 2), (33, 33, 2), (200, 70, 2),
          (96, 80, 2)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,m,batch", SHAPES)
def test_forward_matches_oracle(pkg, n, m, batch, prec):
    print(f"forward n={n} m={m} batch={batch} {prec}", flush=True)
    x = workloads.pft_patches(n, range(batch), seed=100 + n)
    y = pkg.pft2d_forward(torch.from_numpy(x).cuda(), m, prec)
    torch.cuda.synchronize()
    ref = opft.forward(x, m)
    got = y.cpu().numpy()
    assert got.shape == (batch, m, m)
    tol, tol_patch = TOLS[prec]
    assert rel(got, ref) <= tol
    assert per_patch_rel(got, ref).max() <= tol_patch


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,m,batch", SHAPES)
def test_adjoint_matches_oracle(pkg, n, m, batch, prec):
    print(f"adjoint n={n} m={m} batch={batch} {prec}", flush=True)
    y = workloads.pft_coeffs(m, range(batch), seed=200 + n)
    x = pkg.pft2d_adjoint(torch.from_numpy(y).cuda(), n, prec)
    torch.cuda.synchronize()
    ref = opft.adjoint(y, n)
    got = x.cpu().numpy()
    assert got.shape == (batch, n, n)
    tol, tol_patch = TOLS[prec]
    assert rel(got, ref) <= tol
    assert per_patch_rel(got, ref).max() <= tol_patch


def test_unaligned_input_takes_the_masked_path(pkg):
    n, m = 64, 32
    x = workloads.pft_patches(n, range(3), seed=7)
    buf = torch.zeros(3 * n * n + 1, dtype=torch.complex64, device="cuda")
    view = buf[1:].view(3, n, n)          # 8-byte but not 16-byte aligned
    view.copy_(torch.from_numpy(x).cuda())
    assert view.data_ptr() % 16 == 8
    got = pkg.pft2d_forward(view, m).cpu().numpy()
    assert rel(got, opft.forward(x, m)) <= TOL


def test_empty_batch_and_errors(pkg):
    plan = pkg.get_plan(32, 16)
    e = torch.empty(0, 32, 32, dtype=torch.complex64, device="cuda")
    assert plan.forward(e).shape == (0, 16, 16)
    with pytest.raises(ValueError):
        plan.forward(torch.zeros(2, 32, 31, dtype=torch.complex64, device="cuda"))
    with pytest.raises(TypeError):
        plan.forward(torch.zeros(2, 32, 32, dtype=torch.complex128, device="cuda"))
    x = torch.zeros(2, 32, 32, dtype=torch.complex64, device="cuda")
    with pytest.raises(pkg.PftpieError, match="overlap"):
        plan.forward(x, out=x.view(-1)[: 2 * 16 * 16].view(2, 16, 16))


def test_gpu_adjoint_identity_at_workload_shape(pkg):
    n, m, B = 256, 64, 8
    x = torch.from_numpy(workloads.pft_patches(n, range(B), seed=11)).cuda()
    y = torch.from_numpy(workloads.pft_coeffs(m, range(B), seed=12)).cuda()
    Fx = pkg.pft2d_forward(x, m)
    Fhy = pkg.pft2d_adjoint(y, n)
    lhs = torch.vdot(y.reshape(-1).to(torch.complex128), Fx.reshape(-1).to(torch.complex128))
    rhs = torch.vdot(Fhy.reshape(-1).to(torch.complex128), x.reshape(-1).to(torch.complex128))
    scale = n * x.abs().pow(2).sum().sqrt() * y.abs().pow(2).sum().sqrt()
    assert abs((lhs - rhs).item()) / scale.item() < 1e-6
    # F (F^H y) = n^2 y
    back = pkg.pft2d_forward(Fhy, m)
    assert ((back - n * n * y).abs().pow(2).sum().sqrt() / (n * n * y.abs().pow(2).sum().sqrt())).item() < 1e-5


def test_autograd_backward_is_the_adjoint(pkg):
    n, m = 64, 16
    x = torch.from_numpy(workloads.pft_patches(n, range(2), seed=13)).cuda().requires_grad_(True)
    g = torch.from_numpy(workloads.pft_coeffs(m, range(2), seed=14)).cuda()
    y = pkg.pft2d(x, m)
    y.backward(g)
    ref = opft.adjoint(g.cpu().numpy(), n)
    assert rel(x.grad.cpu().numpy(), ref) <= TOL


@pytest.mark.parametrize("prec", PRECS)
def test_standalone_batch_full_size_sampled(pkg, prec):
    """The 4096 x 256^2, m = 64 batch in the benchmark's launch
    configuration; 24 sampled patches checked against the oracle."""
    n, m, B = 256, 64, 4096
    TOL = TOLS[prec][0]
    idx = np.random.default_rng(0).choice(B, 24, replace=False)
    x = torch.empty(B, n, n, dtype=torch.complex64, device="cuda")
    for b0 in range(0, B, 512):
        x[b0:b0 + 512] = torch.from_numpy(workloads.pft_patches(n, range(b0, b0 + 512))).cuda()
    y = pkg.pft2d_forward(x, m, prec)
    yin = torch.empty(B, m, m, dtype=torch.complex64, device="cuda")
    yin.copy_(torch.from_numpy(workloads.pft_coeffs(m, range(B))).cuda())
    xa = pkg.pft2d_adjoint(yin, n, prec)
    torch.cuda.synchronize()
    xs = workloads.pft_patches(n, idx)
    assert rel(y[idx].cpu().numpy(), opft.forward(xs, m)) <= TOL
    ys = workloads.pft_coeffs(m, idx)
    assert rel(xa[idx].cpu().numpy(), opft.adjoint(ys, n)) <= TOL
    assert torch.isfinite(torch.view_as_real(y)).all() and torch.isfinite(torch.view_as_real(xa)).all()


def test_measured_peaks_are_plausible(pkg):
    """The matrix-core loops of the measurement aid report rates within a
    factor of the published dense peaks (FP32 157.3, BF16 / FP16 2516.6
    TFLOP/s) and above what the transforms reach."""
    import ctypes
    v = [ctypes.c_double() for _ in range(3)]
    assert pkg.lib().pftpie_measure_mfma_peaks(*[ctypes.byref(x) for x in v]) == 0
    fp32, bf16, fp16 = (x.value for x in v)
    print("measured peaks", fp32, bf16, fp16, flush=True)
    assert 60.0 < fp32 < 200.0
    assert 800.0 < bf16 < 3200.0 and 800.0 < fp16 < 3200.0
