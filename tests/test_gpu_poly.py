"""GPU parity of the paper's polynomial PFT (Algorithms 1-2, 4-5) against
the FP64 oracle of the same algorithm and against the exact transform.

Tolerances: every coefficient within the algorithm's bound (2 eps + eps^2)
||psi||_1 of the exact transform, plus FP32 rounding of 2e-5 of the
largest exact coefficient; the device and the oracle choose the same number
of polynomial terms r.
"""

import numpy as np
import pytest
import torch

import workloads
from oracle import pft as opft
from oracle import polypft

pytestmark = pytest.mark.gpu

CONFIGS = [(256, 128, 64, 1e-7), (128, 32, 16, 1e-4), (64, 16, 16, 1e-2), (512, 64, 32, 1e-5),
           (96, 40, 32, 1e-3)]


@pytest.fixture(scope="module")
def pk():
    import paper_2408_03532_amd as p
    p.lib()
    return p


@pytest.mark.parametrize("n,m,p,eps", CONFIGS)
def test_poly_matches_exact_within_the_bound(pk, n, m, p, eps):
    print("poly pft", n, m, p, eps, flush=True)
    plan = pk.PolyPlan(n, m, p, eps)
    cfg = polypft.configure(n, m, p, eps)
    assert plan.r == cfg["r"]
    x = workloads.pft_patches(n, range(5), seed=71)
    y = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    exact = opft.forward(x, m)
    bound = polypft.error_bound_2d(x, eps)[:, None, None] + 2e-5 * np.max(np.abs(exact), axis=(-2, -1),
                                                                          keepdims=True)
    assert np.all(np.abs(y - exact) <= bound)
    # and the same algorithm in FP64 agrees to twice that
    ref = polypft.online_2d(x, cfg)
    assert np.all(np.abs(y - ref) <= 2 * bound)


def test_poly_empty_and_long_batches(pk):
    print("poly batches", flush=True)
    plan = pk.PolyPlan(64, 16, 16, 1e-3)
    assert plan.forward(torch.empty(0, 64, 64, dtype=torch.complex64, device="cuda")).shape == (0, 16, 16)
    x = workloads.pft_patches(64, np.arange(700), seed=72)
    y = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    idx = np.arange(0, 700, 97)
    exact = opft.forward(x[idx], 16)
    bound = polypft.error_bound_2d(x[idx], 1e-3)[:, None, None] + 2e-5 * np.max(np.abs(exact))
    assert np.all(np.abs(y[idx] - exact) <= bound)


def test_poly_loose_tolerance_error_is_visible_and_bounded(pk):
    # at eps = 1e-2 the approximation error dominates float rounding: it is
    # well above FP32 noise and inside the bound
    plan = pk.PolyPlan(128, 64, 32, 1e-2)
    x = workloads.pft_patches(128, range(3), seed=73)
    y = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    exact = opft.forward(x, 64)
    err = np.max(np.abs(y - exact), axis=(-2, -1))
    assert np.all(err <= polypft.error_bound_2d(x, 1e-2))
    assert np.all(err > 1e-4 * np.max(np.abs(exact), axis=(-2, -1)))
