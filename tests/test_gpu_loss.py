"""GPU parity of the amplitude loss and its hand-written gradient against the
FP64 oracle (whose gradient is pinned by finite differences and torch
autograd on the CPU).

Tolerances (FP32 path, relative L2): loss <= 1e-5; dL/dO and dL/dP <= 1e-4.
The gradient is a difference of two nearly equal terms (u - a sgn u) near a
good fit, so it carries the transform's rounding amplified by |u| / |u - a|;
1e-4 leaves that margin.
"""

import numpy as np
import pytest
import torch

import workloads
from oracle import loss as oloss

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def pk():
    import paper_2408_03532_amd as p
    p.lib()
    return p


def to_dev(case):
    return (torch.from_numpy(case["obj"]).cuda(), torch.from_numpy(case["probe"]).cuda(),
            torch.from_numpy(case["amp"]).cuda())


SMALL = dict(seed=4, size=288, n=64, m=16, grid=4, step=64, offset=16, radius=20.0, sigma_f=8.0)


@pytest.mark.parametrize("store_u", [True, False])
def test_small_loss_and_gradient(pk, store_u):
    case = workloads.amp_loss_case(**SMALL)
    O, P, A = to_dev(case)
    n, m = 64, 16
    scan = pk.Scan(case["pos"], O.shape, n, m)
    Og = O.clone().requires_grad_(True)
    Pg = P.clone().requires_grad_(True)
    L = pk.amplitude_loss(Og, Pg, scan, A, store_u=store_u)
    L.backward()
    Lr, gOr, gPr = oloss.amp_loss_grad(case["obj"], case["probe"], case["pos"], case["amp"], m)
    assert abs(L.item() - Lr) <= 1e-5 * Lr
    assert rel(Og.grad.cpu().numpy(), gOr) <= 1e-4
    assert rel(Pg.grad.cpu().numpy(), gPr) <= 1e-4


def test_gradient_scale_and_object_only(pk):
    case = workloads.amp_loss_case(**SMALL)
    O, P, A = to_dev(case)
    scan = pk.Scan(case["pos"], O.shape, 64, 16)
    Og = O.clone().requires_grad_(True)
    L = pk.amplitude_loss(Og, P, scan, A)
    (2.5 * L).backward()
    _, gOr, _ = oloss.amp_loss_grad(case["obj"], case["probe"], case["pos"], case["amp"], 16)
    assert rel(Og.grad.cpu().numpy(), 2.5 * gOr) <= 1e-4


@pytest.fixture(scope="module")
def full_case():
    """The full loss workload (1024 positions, 256^2 patches, m = 64 on a
    2304^2 object) with its FP64 oracle loss and gradients, computed once."""
    case = workloads.amp_loss_case()
    Lr, gOr, gPr = oloss.amp_loss_grad(case["obj"], case["probe"], case["pos"], case["amp"], 64)
    return case, Lr, gOr, gPr


def test_full_workload_loss_and_gradient(pk, full_case):
    """1024 positions, 256^2 patches, m = 64 on a 2304^2 object."""
    print("loss full workload", flush=True)
    case, Lr, gOr, gPr = full_case
    O, P, A = to_dev(case)
    scan = pk.Scan(case["pos"], O.shape, 256, 64)
    u = torch.empty(1024, 64, 64, dtype=torch.complex64, device="cuda")
    L = pk.amp_loss(O, P, scan, A, saved_u=u)
    gO, gP = pk.amp_loss_grad(O, P, scan, A, saved_u=u)
    gO2, gP2 = pk.amp_loss_grad(O, P, scan, A)      # recompute path
    torch.cuda.synchronize()
    assert abs(L.item() - Lr) <= 1e-5 * Lr
    assert rel(gO.cpu().numpy(), gOr) <= 1e-4
    assert rel(gP.cpu().numpy(), gPr) <= 1e-4
    assert rel(gO2.cpu().numpy(), gOr) <= 1e-4
    assert rel(gP2.cpu().numpy(), gPr) <= 1e-4


def test_loss_gradient_at_truth_is_small(pk):
    case = workloads.amp_loss_case(**SMALL)
    O = torch.from_numpy(case["obj_true"]).cuda()
    P = torch.from_numpy(case["probe_true"]).cuda()
    A = torch.from_numpy(case["amp"]).cuda()
    scan = pk.Scan(case["pos"], O.shape, 64, 16)
    L = pk.amp_loss(O, P, scan, A).item()
    scale = float(np.sum(case["amp"].astype(np.float64) ** 2))
    assert L <= 1e-10 * scale


@pytest.mark.parametrize("precision,tol", [("split_bf16", 1e-3), ("split_fp16", 1e-4)])
def test_split_precision_loss_and_gradient(pk, precision, tol):
    case = workloads.amp_loss_case(**SMALL)
    O, P, A = to_dev(case)
    scan = pk.Scan(case["pos"], O.shape, 64, 16, precision=precision)
    L = pk.amp_loss(O, P, scan, A)
    gO, gP = pk.amp_loss_grad(O, P, scan, A)
    Lr, gOr, gPr = oloss.amp_loss_grad(case["obj"], case["probe"], case["pos"], case["amp"], 16)
    assert abs(L.item() - Lr) <= tol * Lr
    assert rel(gO.cpu().numpy(), gOr) <= tol
    assert rel(gP.cpu().numpy(), gPr) <= tol


@pytest.mark.parametrize("precision,tol_l,tol_g", [("split_bf16", 1e-4, 1e-3), ("split_fp16", 1e-5, 1e-4)])
def test_full_workload_split_precision(pk, full_case, precision, tol_l, tol_g):
    """The full loss workload in the split precisions, stored and recomputed
    spectra, against the FP64 oracle (loss and both gradients)."""
    print("loss full workload", precision, flush=True)
    case, Lr, gOr, gPr = full_case
    O, P, A = to_dev(case)
    scan = pk.Scan(case["pos"], O.shape, 256, 64, precision=precision)
    u = torch.empty(1024, 64, 64, dtype=torch.complex64, device="cuda")
    L = pk.amp_loss(O, P, scan, A, saved_u=u)
    gO, gP = pk.amp_loss_grad(O, P, scan, A, saved_u=u)
    gO2, gP2 = pk.amp_loss_grad(O, P, scan, A)
    torch.cuda.synchronize()
    assert abs(L.item() - Lr) <= tol_l * Lr
    for g, r in ((gO, gOr), (gP, gPr), (gO2, gOr), (gP2, gPr)):
        assert rel(g.cpu().numpy(), r) <= tol_g


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("split_bf16", 1e-3), ("split_fp16", 1e-4)])
def test_zero_exit_wave_has_zero_subgradient(pk, precision, tol):
    """A window of zero object gives u = 0 exactly: its residual term uses
    sgn(0) = 0, so R_j = 2 F^H u F = 0 there and the position adds a^2 to the
    loss and nothing to the gradients; the rest match the oracle."""
    print("loss zero window", precision, flush=True)
    case = workloads.amp_loss_case(**SMALL)
    obj = case["obj"].copy()
    r, c = case["pos"][5]
    obj[r:r + 64, c:c + 64] = 0      # windows of this scan do not overlap
    O = torch.from_numpy(obj).cuda()
    P = torch.from_numpy(case["probe"]).cuda()
    A = torch.from_numpy(case["amp"]).cuda()
    scan = pk.Scan(case["pos"], O.shape, 64, 16, precision=precision)
    L = pk.amp_loss(O, P, scan, A)
    gO, gP = pk.amp_loss_grad(O, P, scan, A)
    Lr, gOr, gPr = oloss.amp_loss_grad(obj, case["probe"], case["pos"], case["amp"], 16)
    assert abs(L.item() - Lr) <= tol * Lr
    assert rel(gO.cpu().numpy(), gOr) <= tol
    assert rel(gP.cpu().numpy(), gPr) <= tol
    assert np.all(np.isfinite(gO.cpu().numpy())) and np.all(np.isfinite(gP.cpu().numpy()))


@pytest.mark.parametrize("n,m", [(40, 12), (64, 20)])
def test_ragged_sizes_loss_and_gradient(pk, n, m):
    """Windows that are not whole 16-pixel tiles (n = 40) or kept blocks that
    are not (m = 12, 20): the kernels that hold the twiddle table in LDS and
    whole windows per wave step aside for the general ones; same results."""
    print("loss ragged", n, m, flush=True)
    case = workloads.amp_loss_case(seed=6, size=200, n=n, m=m, grid=4, step=40, offset=8, radius=n / 3.0,
                                   sigma_f=8.0)
    O, P, A = to_dev(case)
    scan = pk.Scan(case["pos"], O.shape, n, m)
    Og = O.clone().requires_grad_(True)
    Pg = P.clone().requires_grad_(True)
    L = pk.amplitude_loss(Og, Pg, scan, A)
    L.backward()
    Lr, gOr, gPr = oloss.amp_loss_grad(case["obj"], case["probe"], case["pos"], case["amp"], m)
    assert abs(L.item() - Lr) <= 1e-5 * Lr
    assert rel(Og.grad.cpu().numpy(), gOr) <= 1e-4
    assert rel(Pg.grad.cpu().numpy(), gPr) <= 1e-4
