"""GPU parity of the full-window fast transform (plan method "fft", m = n):
the plain forward / adjoint and the fused PIE position step against the FP64
oracle, and against the dense contraction on the same inputs.

With m = n the kept window is the whole spectrum and the partial transform
is the 2-D DFT in centred order, so the fast transform computes the same
quantity as the dense contraction (the oracle's F_m psi F_m^T) in
~5 n^2 log2 n instead of 8 n^3 flops.  Tolerances are the FP32 ones of the
dense path: relative L2 <= 1e-5 per transform and per sweep from a common
state, Phi per sweep <= 1e-5 relative.
"""

import numpy as np
import pytest
import torch

import workloads
from oracle import pft as opft
from oracle import pie as opie

pytestmark = pytest.mark.gpu

SIZES = [16, 32, 64, 128]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def amps(pk, intensity, m):
    """Each side crops the data itself (Algorithm 3): the library's crop
    kernel on the device, the oracle's crop in float64 on the host."""
    return pk.crop_amplitudes(torch.from_numpy(intensity).cuda(), m), opie.amplitudes(intensity, m)


@pytest.fixture(scope="module")
def pk():
    import paper_2408_03532_amd as p
    p.lib()
    return p


@pytest.mark.parametrize("n", SIZES)
def test_method_resolution(pk, n):
    print("fft method resolution", n, flush=True)
    assert pk.Plan(n, n).method == "fft"
    assert pk.Plan(n, n, method="dense").method == "dense"
    assert pk.Plan(n, n // 2).method == "dense"
    with pytest.raises(pk.PftpieError):
        pk.Plan(n, n // 2, method="fft")


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_forward_adjoint_match_oracle(pk, n, precision):
    # the fast transform computes in FP32 whatever the plan's precision
    print("fft transform", n, precision, flush=True)
    plan = pk.Plan(n, n, precision, method="fft")
    x = workloads.pft_patches(n, range(5), seed=31)
    y = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel(y, opft.forward(x, n)) <= 1e-5
    c = workloads.pft_coeffs(n, range(5), seed=32)
    xa = plan.adjoint(torch.from_numpy(c).cuda()).cpu().numpy()
    assert rel(xa, opft.adjoint(c, n)) <= 1e-5


@pytest.mark.parametrize("n", SIZES)
def test_fft_and_dense_agree(pk, n):
    print("fft vs dense", n, flush=True)
    x = torch.from_numpy(workloads.pft_patches(n, range(3, 9), seed=33)).cuda()
    yf = pk.Plan(n, n, method="fft").forward(x).cpu().numpy()
    yd = pk.Plan(n, n, method="dense").forward(x).cpu().numpy()
    assert rel(yf, yd) <= 5e-6
    c = torch.from_numpy(workloads.pft_coeffs(n, range(2), seed=34)).cuda()
    af = pk.Plan(n, n, method="fft").adjoint(c).cpu().numpy()
    ad = pk.Plan(n, n, method="dense").adjoint(c).cpu().numpy()
    assert rel(af, ad) <= 5e-6


def test_empty_batch_and_large_batch_tail(pk):
    print("fft empty batch and grid tail", flush=True)
    plan = pk.Plan(32, 32, method="fft")
    out = plan.forward(torch.empty(0, 32, 32, dtype=torch.complex64, device="cuda"))
    assert out.shape == (0, 32, 32)
    # more patches than the persistent grid: every patch is reached once
    idx = np.arange(0, 4100, 257)
    x = workloads.pft_patches(32, np.arange(4100), seed=35)
    y = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel(y[idx], opft.forward(x[idx], 32)) <= 1e-5


@pytest.fixture(scope="module")
def tiny():
    return workloads.tiny_pie()


# Sequential overlap-normalised steps use alpha = 0.1: each step divides by
# |P|^2 + alpha max |P|^2, and with alpha = 1e-3 the 64 chained steps amplify
# float rounding in the probe's tails until any FP32 path (the dense
# contraction as much as the fast transform) ends ~25 % of |dO| away from the
# FP64 oracle, while one or two steps still agree to 1e-6.
MODES = [dict(batch=1, norm=0, beta=1.0, gamma=0.0),
         dict(batch=1, norm=1, beta=1.0, gamma=0.0, alpha=0.1),
         dict(batch=1, norm=1, beta=0.9, gamma=0.3, alpha=0.1),
         dict(batch=64, norm=1, beta=1.0, gamma=0.0, alpha=1e-3),
         dict(batch=7, norm=1, beta=0.8, gamma=0.5, alpha=1e-3),
         dict(batch=10, norm=0, beta=0.05, gamma=0.02)]


@pytest.mark.parametrize("mode", MODES, ids=lambda d: "-".join(f"{k}{v}" for k, v in d.items()))
def test_pie_sweep_full_window_matches_oracle(pk, tiny, mode):
    print("fft pie sweep", mode, flush=True)
    n = tiny["probe"].shape[0]
    A, amp = amps(pk, tiny["intensity"], n)
    init = tiny["init"]
    P0 = tiny["probe"] * (1.0 + 0.05j) if mode.get("gamma", 0) else tiny["probe"]
    scan = pk.Scan(tiny["pos"], init.shape, n, n, method="fft")
    assert scan.plan.method == "fft"
    O = torch.from_numpy(init.astype(np.complex64)).cuda()
    P = torch.from_numpy(P0.astype(np.complex64)).cuda()
    st = pk.pie_sweep(O, P, scan, A, pk.PieParams(**mode)).cpu().numpy()
    Or, Pr, sr = opie.pie_sweep(init, P0, tiny["pos"], amp, n, **mode)
    assert rel(O.cpu().numpy(), Or) <= 1e-5
    if mode.get("gamma", 0):
        assert rel(P.cpu().numpy(), Pr) <= 1e-5
    assert abs(st[0] - sr[0]) <= 1e-5 * sr[0]
    assert st[3] == 0


def test_pie_sweep_order_and_invalid_entries(pk, tiny):
    # a permuted order with an out-of-range entry: that entry contributes
    # nothing, the rest follow the permutation
    print("fft pie order", flush=True)
    n = tiny["probe"].shape[0]
    A0, amp = amps(pk, tiny["intensity"], n)
    J = len(tiny["pos"])
    order = np.random.default_rng(7).permutation(J).astype(np.int32)
    order_bad = order.copy()
    order_bad[5] = J + 3
    scan = pk.Scan(tiny["pos"], tiny["init"].shape, n, n, method="fft")
    for ordr in (order, order_bad):
        O = torch.from_numpy(tiny["init"]).cuda()
        P = torch.from_numpy(tiny["probe"]).cuda()
        A = A0
        prm = pk.PieParams(batch=1, norm=1, beta=1.0, alpha=0.1)
        pk.pie_sweep(O, P, scan, A, prm, order=torch.from_numpy(ordr).cuda())
        # the oracle takes the valid entries, in order, as a scan of their own
        keep = ordr[(ordr >= 0) & (ordr < J)]
        Or, _, _ = opie.pie_sweep(tiny["init"], tiny["probe"], tiny["pos"][keep], amp[keep], n,
                                  batch=1, norm=1, beta=1.0, alpha=0.1)
        assert rel(O.cpu().numpy(), Or) <= 1e-5


def test_noise_free_fixed_point(pk, tiny):
    # the true object and probe are a fixed point of the full-window step
    print("fft pie fixed point", flush=True)
    n = tiny["probe"].shape[0]
    A, amp = amps(pk, tiny["intensity"], n)
    scan = pk.Scan(tiny["pos"], tiny["obj"].shape, n, n, method="fft")
    O = torch.from_numpy(tiny["obj"].astype(np.complex64)).cuda()
    P = torch.from_numpy(tiny["probe"].astype(np.complex64)).cuda()
    O0 = O.clone()
    pk.pie_sweep(O, P, scan, A, pk.PieParams(batch=64, norm=1, beta=1.0, alpha=1e-3))
    assert rel(O.cpu().numpy(), O0.cpu().numpy()) <= 1e-6


def test_phase2_at_scale_fft_matches_dense_and_oracle(pk):
    # one full-resolution sweep of the warm-started workload (1024^2 object,
    # 128^2 probe, 900 positions, m = n = 128, fully batched, normalised)
    print("fft pie at scale", flush=True)
    case = workloads.pie_at_scale()
    A, amp = amps(pk, case["intensity"], 128)
    prm = dict(batch=900, norm=1, beta=1.0, alpha=1e-3)
    outs = {}
    for method in ("fft", "dense"):
        scan = pk.Scan(case["pos"], (1024, 1024), 128, 128, method=method)
        O = torch.from_numpy(case["init"]).cuda()
        P = torch.from_numpy(case["probe"]).cuda()
        st = pk.pie_sweep(O, P, scan, A, pk.PieParams(**prm)).cpu().numpy()
        outs[method] = (O.cpu().numpy(), st)
    assert rel(outs["fft"][0], outs["dense"][0]) <= 5e-6
    Or, _, sr = opie.pie_sweep(case["init"], case["probe"], case["pos"], amp, 128, **prm)
    assert rel(outs["fft"][0], Or) <= 1e-5
    assert abs(outs["fft"][1][0] - sr[0]) <= 1e-5 * sr[0]
