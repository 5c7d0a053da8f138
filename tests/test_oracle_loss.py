"""Pins of the FP64 amplitude-loss gradient: central finite differences and an
independent autograd route through torch.fft on the CPU."""

import numpy as np
import pytest
import torch

import workloads
from oracle import loss


def tiny(seed=0, H=36, n=16, m=8, grid=3, step=8, offset=2):
    rs = np.random.default_rng(seed)
    obj = rs.standard_normal((H, H)) + 1j * rs.standard_normal((H, H))
    probe = workloads.gaussian_probe(n, 5.0, 0.04).astype(np.complex128) * (1 + 0.2j)
    pos = workloads.raster(grid, grid, step, offset)
    amp = np.abs(rs.standard_normal((len(pos), m, m))) * n
    return obj, probe, pos, amp, m


def test_directional_finite_differences():
    obj, probe, pos, amp, m = tiny(1)
    L, gO, gP = loss.amp_loss_grad(obj, probe, pos, amp, m)
    assert abs(L - loss.amp_loss(obj, probe, pos, amp, m)) < 1e-12 * L
    rs = np.random.default_rng(2)
    h = 1e-6
    for _ in range(8):
        VO = rs.standard_normal(obj.shape) + 1j * rs.standard_normal(obj.shape)
        VP = rs.standard_normal(probe.shape) + 1j * rs.standard_normal(probe.shape)
        fd = (loss.amp_loss(obj + h * VO, probe + h * VP, pos, amp, m)
              - loss.amp_loss(obj - h * VO, probe - h * VP, pos, amp, m)) / (2 * h)
        an = np.real(np.vdot(gO, VO) + np.vdot(gP, VP))
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_coordinate_finite_differences_exhaustive_tiny():
    obj, probe, pos, amp, m = tiny(3, H=12, n=8, m=4, grid=2, step=3, offset=0)
    _, gO, gP = loss.amp_loss_grad(obj, probe, pos, amp, m)
    h = 1e-6
    for arr, g, which in ((obj, gO, 0), (probe, gP, 1)):
        for idx in np.ndindex(arr.shape):
            for unit in (1.0, 1j):
                e = np.zeros_like(arr)
                e[idx] = unit
                args_p = (obj + h * e, probe) if which == 0 else (obj, probe + h * e)
                args_m = (obj - h * e, probe) if which == 0 else (obj, probe - h * e)
                fd = (loss.amp_loss(*args_p, pos, amp, m) - loss.amp_loss(*args_m, pos, amp, m)) / (2 * h)
                an = (g[idx].real if unit == 1.0 else g[idx].imag)
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_matches_torch_autograd_through_full_fft():
    obj, probe, pos, amp, m = tiny(4)
    L, gO, gP = loss.amp_loss_grad(obj, probe, pos, amp, m)
    O = torch.tensor(obj, dtype=torch.complex128, requires_grad=True)
    P = torch.tensor(probe, dtype=torch.complex128, requires_grad=True)
    n = probe.shape[0]
    s = n // 2 - m // 2
    tot = 0
    for j, (r, c) in enumerate(pos):
        spec = torch.fft.fftshift(torch.fft.fft2(P * O[r:r + n, c:c + n]))
        u = spec[s:s + m, s:s + m]
        tot = tot + ((u.abs() - torch.tensor(amp[j])) ** 2).sum()
    tot.backward()
    assert abs(tot.item() - L) < 1e-12 * L
    assert np.linalg.norm(O.grad.numpy() - gO) / np.linalg.norm(gO) < 1e-13
    assert np.linalg.norm(P.grad.numpy() - gP) / np.linalg.norm(gP) < 1e-13


def test_gradient_is_zero_at_the_truth_and_sgn0_is_zero():
    case = workloads.amp_loss_case(seed=4, size=96, n=32, m=8, grid=3, step=24, offset=8,
                                   radius=10.0, sigma_f=6.0)
    L, gO, gP = loss.amp_loss_grad(case["obj_true"], case["probe_true"], case["pos"], case["amp"], 8)
    # zero up to the float32 rounding of the stored amplitudes
    scale = float(np.sum(case["amp"].astype(np.float64) ** 2))
    assert L < 1e-12 * scale
    assert np.max(np.abs(gO)) < 1e-6 * np.sqrt(scale) and np.max(np.abs(gP)) < 1e-6 * np.sqrt(scale)
    # all-zero exit wave with zero data: u = 0 everywhere, sgn(0) = 0 gives 0
    z = np.zeros((16, 16), complex)
    L0, g0, _ = loss.amp_loss_grad(z, np.ones((8, 8)), np.array([[0, 0]]), np.zeros((1, 4, 4)), 4)
    assert L0 == 0.0 and np.all(g0 == 0)


@pytest.mark.parametrize("bad", ["no_conj", "half"])
def test_plausible_mistakes_fail_finite_differences(bad):
    obj, probe, pos, amp, m = tiny(5)
    _, gO, _ = loss.amp_loss_grad(obj, probe, pos, amp, m)
    if bad == "no_conj":
        # the gradient with respect to O carries conj(P); without it FD fails
        probe_phase = probe / np.conj(probe)
        wrong = gO.copy()
        n = probe.shape[0]
        r, c = pos[4]
        wrong[r:r + n, c:c + n] *= np.where(np.abs(probe) > 0, probe_phase, 1)
    else:
        wrong = 0.5 * gO
    V = np.random.default_rng(7).standard_normal(obj.shape) + 0j
    h = 1e-6
    fd = (loss.amp_loss(obj + h * V, probe, pos, amp, m) - loss.amp_loss(obj - h * V, probe, pos, amp, m)) / (2 * h)
    assert abs(fd - np.real(np.vdot(wrong, V))) > 1e-4 * abs(fd)
