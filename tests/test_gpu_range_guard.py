"""The FP16 range guard of the split-precision engines, against the FP64
oracle.  FP16 holds magnitudes up to 65504; operands or stage-1
intermediates beyond it would become inf when split.  The engines rescale
such a patch by a power of two and undo the scale on the result, so inputs
of any magnitude meet the split-FP16 tolerances (relative L2 <= 1e-5 for
the transforms and one sweep, <= 1e-4 for the loss gradient) instead of
returning inf or NaN.  BF16 keeps the FP32 exponent range and is checked on
the same inputs."""

import numpy as np
import pytest
import torch

import workloads
from oracle import loss as oloss
from oracle import pft as opft
from oracle import pie as opie

pytestmark = pytest.mark.gpu

TOL = {"split_fp16": 1e-5, "split_bf16": 1e-4}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def pk():
    import paper_2408_03532_amd as p
    p.lib()
    return p


@pytest.mark.parametrize("prec", sorted(TOL))
def test_adjoint_of_an_all_ones_patch_forward(pk, prec):
    """The forward of an all-ones 256^2 patch has its zero-frequency
    coefficient at n^2 = 65536, just above FP16's range: the adjoint of that
    output must come back finite and match the oracle."""
    print("guard all ones", prec, flush=True)
    x = np.ones((2, 256, 256), dtype=np.complex64)
    y = pk.pft2d_forward(torch.from_numpy(x).cuda(), 64, prec)
    yh = y.cpu().numpy()
    assert rel(yh, opft.forward(x, 64)) <= TOL[prec]
    xa = pk.pft2d_adjoint(y, 256, prec).cpu().numpy()
    assert np.isfinite(xa).all()
    assert rel(xa, opft.adjoint(yh, 256)) <= TOL[prec]


@pytest.mark.parametrize("prec", sorted(TOL))
@pytest.mark.parametrize("n,m", [(256, 64), (128, 32), (40, 24), (512, 128)])
def test_transforms_of_large_inputs(pk, n, m, prec):
    """Patches of magnitude ~1e5 (operands beyond FP16) and coefficients of
    magnitude ~1e6, one ordinary patch beside them: every patch matches."""
    print("guard large", n, m, prec, flush=True)
    x = workloads.pft_patches(n, range(3), seed=300 + n).astype(np.complex128)
    x[0] *= 1e5
    x[2] *= 3e3
    x = x.astype(np.complex64)
    y = pk.pft2d_forward(torch.from_numpy(x).cuda(), m, prec).cpu().numpy()
    ref = opft.forward(x, m)
    for b in range(3):
        assert rel(y[b], ref[b]) <= TOL[prec]
    c = workloads.pft_coeffs(m, range(3), seed=400 + m).astype(np.complex128)
    c[1] *= 1e6
    c = c.astype(np.complex64)
    xa = pk.pft2d_adjoint(torch.from_numpy(c).cuda(), n, prec).cpu().numpy()
    ra = opft.adjoint(c, n)
    for b in range(3):
        assert rel(xa[b], ra[b]) <= TOL[prec]


@pytest.mark.parametrize("prec", sorted(TOL))
@pytest.mark.parametrize("mode", [dict(batch=64, norm=1, beta=1.0, gamma=0.5, alpha=1e-3),
                                  dict(batch=1, norm=0, beta=1.0)], ids=["batched", "sequential"])
def test_pie_sweep_at_large_scale(pk, prec, mode):
    """The object step is equivariant under O -> k O, a -> k a, and so is the
    overlap-normalised probe step (the plain probe step is not: it grows as
    k^2): at k = 1e5 the exit waves exceed FP16's range; one sweep still
    matches the oracle."""
    print("guard pie", prec, mode, flush=True)
    tiny = workloads.tiny_pie()
    k = 1e5
    I = (tiny["intensity"].astype(np.float64) * k * k).astype(np.float32)
    init = (tiny["init"].astype(np.complex128) * k).astype(np.complex64)
    scan = pk.Scan(tiny["pos"], init.shape, 32, 16, precision=prec)
    A = pk.crop_amplitudes(torch.from_numpy(I).cuda(), 16)
    O = torch.from_numpy(init).cuda()
    P = torch.from_numpy(tiny["probe"]).cuda()
    st = pk.pie_sweep(O, P, scan, A, pk.PieParams(**mode)).cpu().numpy()
    Or, Pr, sr = opie.pie_sweep(init, tiny["probe"], tiny["pos"], opie.amplitudes(I, 16), 16, **mode)
    assert np.isfinite(O.cpu().numpy()).all() and st[3] == 0
    assert rel(O.cpu().numpy(), Or) <= TOL[prec]
    assert rel(P.cpu().numpy(), Pr) <= TOL[prec]
    assert abs(st[0] - sr[0]) <= TOL[prec] * sr[0]


@pytest.mark.parametrize("prec", sorted(TOL))
def test_loss_gradient_at_large_scale(pk, prec):
    """Loss and gradients with the object and amplitudes scaled by 1e5."""
    print("guard loss", prec, flush=True)
    case = workloads.amp_loss_case(seed=4, size=288, n=64, m=16, grid=4, step=64, offset=16,
                                   radius=20.0, sigma_f=8.0)
    k = 1e5
    obj = (case["obj"].astype(np.complex128) * k).astype(np.complex64)
    amp = (case["amp"].astype(np.float64) * k).astype(np.float32)
    scan = pk.Scan(case["pos"], obj.shape, 64, 16, precision=prec)
    O = torch.from_numpy(obj).cuda()
    P = torch.from_numpy(case["probe"]).cuda()
    A = torch.from_numpy(amp).cuda()
    L = pk.amp_loss(O, P, scan, A).item()
    gO, gP = pk.amp_loss_grad(O, P, scan, A)
    Lr, gOr, gPr = oloss.amp_loss_grad(obj, case["probe"], case["pos"], amp, 16)
    tol = TOL[prec] * 10
    assert abs(L - Lr) <= tol * Lr
    assert rel(gO.cpu().numpy(), gOr) <= tol
    assert rel(gP.cpu().numpy(), gPr) <= tol


@pytest.mark.parametrize("prec", sorted(TOL))
def test_uneven_batch_with_large_patches(pk, prec):
    """The persistent uneven-batch kernel uses the same engines: a mixed
    batch with some patches at 1e5 matches the oracle patch by patch."""
    print("guard group", prec, flush=True)
    d, tin, tout = workloads.grouped_descs(count=16, seed=9)
    x = workloads.grouped_inputs(d, tin, seed=9).astype(np.complex128)
    for i in (0, 5, 11):
        n, m, io, _ = (int(v) for v in d[i])
        x[io:io + n * n] *= 1e5
    x = x.astype(np.complex64)
    g = pk.Group(d, tin, tout, prec)
    y = g.run(torch.from_numpy(x).cuda()).cpu().numpy()
    for i in range(len(d)):
        n, m, io, oo = (int(v) for v in d[i])
        ref = opft.forward(x[io:io + n * n].reshape(n, n), m)
        assert rel(y[oo:oo + m * m].reshape(m, m), ref) <= TOL[prec]
