"""Pins of the polynomial PFT oracle (Algorithms 1, 2, 4, 5) against the
library FFT, the paper's printed constant and its error bound."""

import numpy as np
import pytest

from oracle import polypft


def crop_fft(z, m):
    n = z.shape[-1]
    lo = n // 2 - m // 2
    return np.fft.fftshift(np.fft.fft(z))[lo:lo + m]


def crop_fft2(Z, m):
    n = Z.shape[-1]
    lo = n // 2 - m // 2
    return np.fft.fftshift(np.fft.fft2(Z), axes=(-2, -1))[..., lo:lo + m, lo:lo + m]


def test_paper_constant_r13_at_eps_1e7():
    # Sec. 4: m~ = p = 64 (m~/p = 1) and eps = 1e-7 give r = 13
    assert polypft.choose_r(1e-7, 1.0) == 13
    assert polypft.xi_of(1e-7, 12) < 1.0 <= polypft.xi_of(1e-7, 13)


@pytest.mark.parametrize("eps,r", [(1e-7, 13), (1e-4, 8), (1e-2, 5)])
def test_xi_is_the_largest_scope_within_eps(eps, r):
    xi = polypft.xi_of(eps, r)
    assert polypft.poly_error(polypft.chebyshev_poly(xi, r), xi) <= eps
    assert polypft.poly_error(polypft.chebyshev_poly(1.01 * xi, r), 1.01 * xi) > eps


@pytest.mark.parametrize("n,m,p,eps", [(256, 128, 64, 1e-7), (512, 64, 32, 1e-5), (240, 40, 20, 1e-3)])
def test_online_1d_within_bound_of_exact(n, m, p, eps):
    rng = np.random.default_rng(61)
    z = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    cfg = polypft.configure(n, m, p, eps)
    got = polypft.online_1d(z, cfg)
    assert np.max(np.abs(got - crop_fft(z, m))) <= eps * np.sum(np.abs(z))


@pytest.mark.parametrize("n,m,p,eps", [(256, 128, 64, 1e-7), (128, 32, 16, 1e-4), (64, 16, 16, 1e-2)])
def test_online_2d_within_bound_of_exact(n, m, p, eps):
    rng = np.random.default_rng(62)
    Z = rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))
    cfg = polypft.configure(n, m, p, eps)
    got = polypft.online_2d(Z, cfg)
    err = np.max(np.abs(got - crop_fft2(Z, m)), axis=(-2, -1))
    assert np.all(err <= polypft.error_bound_2d(Z, eps))
    # and not trivially: the error is above float rounding for loose eps
    if eps >= 1e-4:
        assert np.max(err) > 1e-3 * eps * np.max(np.sum(np.abs(Z), axis=(-2, -1))) / n


def test_tight_tolerance_reaches_the_exact_transform():
    rng = np.random.default_rng(63)
    Z = rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64))
    cfg = polypft.configure(64, 32, 16, 1e-13)
    ref = crop_fft2(Z, 32)
    assert np.max(np.abs(polypft.online_2d(Z, cfg) - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_plausible_mistakes_break_the_bound():
    rng = np.random.default_rng(64)
    Z = rng.standard_normal((128, 128)) + 1j * rng.standard_normal((128, 128))
    ref = crop_fft2(Z, 32)
    bound = polypft.error_bound_2d(Z, 1e-6)
    cfg = polypft.configure(128, 32, 16, 1e-6)
    for bad in ("sign", "transpose", "shift"):
        c = dict(cfg)
        if bad == "sign":      # e^{+pi i t/p} instead of e^{-pi i t/p}
            c["W"] = cfg["W"] * np.exp(2j * np.pi * (np.arange(32) - 16) / 16)[:, None]
        elif bad == "transpose":  # 1 + 2j/q instead of 1 - 2j/q
            c["B"] = cfg["B"][::-1, :]
        else:                  # frequency index t instead of t mod p picked off by one
            c["W"] = np.roll(cfg["W"], 1, axis=0)
        assert np.max(np.abs(polypft.online_2d(Z, c) - ref)) > 10 * bound
