"""Pins of the FP64 partial-DFT oracle against things other than itself:
the DFT definition written as loops, NumPy's FFT, closed forms and the
algebraic identities of the DFT (Sec. 3.1.1, eq. (7); Appendix A, eq. (16);
Fig. 2)."""

import json
import os

import numpy as np
import pytest

from oracle import pft

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def rnd(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def fft_crop(psi, m):
    """Independent route: full FFT, shift the zero frequency to floor(n/2),
    cut the centred m x m window."""
    n = psi.shape[-1]
    s = n // 2 - m // 2
    spec = np.fft.fftshift(np.fft.fft2(psi), axes=(-2, -1))
    return spec[..., s:s + m, s:s + m]


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("m", [1, 2, 5, 16, 17, 64])
def test_window_is_centred(m):
    t = pft.window(m)
    assert len(t) == m
    assert t[0] == -(m // 2) and t[-1] == (m + 1) // 2 - 1
    assert np.all(np.diff(t) == 1)
    assert (t == 0).sum() == 1 and t[m // 2] == 0


def test_twiddle_rows_orthogonal_and_unimodular():
    for n, m in [(8, 8), (32, 16), (33, 7), (256, 64)]:
        F = pft.twiddles(n, m)
        assert F.shape == (m, n)
        assert np.allclose(np.abs(F), 1.0, atol=1e-15)
        assert np.allclose(F[:, 0], 1.0)
        # rows of the partial DFT are orthogonal with norm^2 n
        assert np.allclose(F @ F.conj().T, n * np.eye(m), atol=1e-11 * n)


def test_twiddle_integer_reduction_keeps_large_phases_exact():
    # t*k reaches 64*255; the table must equal the n-th roots of unity looked
    # up at (t*k mod n), to within one rounding of each root.
    n, m = 256, 128
    F = pft.twiddles(n, m)
    t = pft.window(m)
    roots = np.exp(-2j * np.pi * np.arange(n) / n)
    ref = roots[np.mod(np.outer(t, np.arange(n)), n)]
    assert np.max(np.abs(F - ref)) < 1e-15
    # an unreduced angle would already be off by more than that
    bad = np.exp(-2j * np.pi * np.outer(t, np.arange(n)).astype(np.float32) / np.float32(n))
    assert np.max(np.abs(bad - ref)) > 1e-9


@pytest.mark.parametrize("n,m", [(4, 4), (5, 3), (8, 4), (9, 9), (12, 5), (16, 8)])
def test_forward_equals_direct_quadruple_sum(n, m):
    psi = rnd((n, n), n * 100 + m)
    assert rel(pft.forward(psi, m), pft.forward_direct(psi, m)) < 1e-13


@pytest.mark.parametrize("n,m", [(32, 16), (64, 16), (128, 32), (128, 128), (256, 64),
                                 (33, 8), (31, 31), (40, 1), (512, 128)])
def test_forward_equals_fft_centre_crop(n, m):
    psi = rnd((2, n, n), n + m)
    assert rel(pft.forward(psi, m), fft_crop(psi, m)) < 1e-13


def test_fig2_crop_matches_paper_sizes():
    g = json.load(open(GOLDEN))
    full = g["fig2_full_side"]["value"]
    crop = g["fig2_crop_side"]["value"]
    # the 128 x 128 window of Fig. 2 has half-width m~ = 64 (Sec. 3.1.2)
    assert crop == g["crop_side_from_half_width"]["value"] == 2 * g["crop_half_width"]["value"]
    psi = rnd((full, full), 7)
    Y = pft.forward(psi, crop)
    spec = np.fft.fftshift(np.fft.fft2(psi))
    lo = full // 2 - crop // 2
    assert lo == 192
    assert rel(Y, spec[lo:lo + crop, lo:lo + crop]) < 1e-12


def test_closed_forms():
    n, m = 24, 10
    t = pft.window(m)
    # delta at (k1, k2)
    for k1, k2 in [(0, 0), (3, 17), (23, 1)]:
        psi = np.zeros((n, n))
        psi[k1, k2] = 1.0
        ref = np.exp(-2j * np.pi * (t[:, None] * k1 + t[None, :] * k2) / n)
        assert np.max(np.abs(pft.forward(psi, m) - ref)) < 1e-13
    # constant one: n^2 at t = (0, 0), zero elsewhere
    Y = pft.forward(np.ones((n, n)), m)
    ref = np.zeros((m, m), complex)
    ref[m // 2, m // 2] = n * n
    assert np.max(np.abs(Y - ref)) < 1e-10
    # plane waves: n^2 delta at t = f when f is kept, else zero
    for f1, f2 in [(2, -3), (-5, 4), (9, 0), (-11, 2)]:
        k = np.arange(n)
        psi = np.exp(2j * np.pi * (f1 * k[:, None] + f2 * k[None, :]) / n)
        Y = pft.forward(psi, m)
        ref = np.zeros((m, m), complex)
        if t[0] <= f1 <= t[-1] and t[0] <= f2 <= t[-1]:
            ref[f1 + m // 2, f2 + m // 2] = n * n
        assert np.max(np.abs(Y - ref)) < 1e-10


def test_linearity_and_shift_theorem():
    n, m = 32, 12
    a, b = rnd((n, n), 1), rnd((n, n), 2)
    al, be = 0.3 - 1.2j, -2.0 + 0.5j
    assert rel(pft.forward(al * a + be * b, m), al * pft.forward(a, m) + be * pft.forward(b, m)) < 1e-13
    t = pft.window(m)
    for s1, s2 in [(1, 0), (0, 5), (7, -3)]:
        shifted = np.roll(a, (s1, s2), axis=(0, 1))
        ramp = np.exp(-2j * np.pi * (t[:, None] * s1 + t[None, :] * s2) / n)
        assert rel(pft.forward(shifted, m), ramp * pft.forward(a, m)) < 1e-13


def test_real_input_hermitian_symmetry_and_energy_bound():
    n, m = 30, 11  # odd m: the window is symmetric about 0
    x = np.random.default_rng(3).standard_normal((n, n))
    Y = pft.forward(x, m)
    # Y[-t] = conj(Y[t]); for odd m index c <-> m-1-c
    assert np.max(np.abs(Y[::-1, ::-1] - np.conj(Y))) < 1e-11
    # ||Y||^2 <= n^2 ||psi||^2, equality for band-limited input
    psi = rnd((n, n), 4)
    assert np.linalg.norm(pft.forward(psi, m)) ** 2 <= n * n * np.linalg.norm(psi) ** 2
    band = pft.adjoint(rnd((m, m), 5), n)
    assert abs(np.linalg.norm(pft.forward(band, m)) ** 2 / (n * n * np.linalg.norm(band) ** 2) - 1) < 1e-12


@pytest.mark.parametrize("n,m", [(16, 16), (32, 8), (33, 10), (128, 32), (256, 64)])
def test_adjoint_identity_and_pseudo_inverse(n, m):
    x = rnd((n, n), n)
    y = rnd((m, m), m)
    lhs = np.vdot(y, pft.forward(x, m))            # <F x, y> with conj on y
    rhs = np.vdot(pft.adjoint(y, n), x)            # <x, F^H y>
    assert abs(lhs - rhs) / (np.linalg.norm(x) * np.linalg.norm(y) * n) < 1e-13
    # F_m (F_m^H y) = n^2 y
    assert rel(pft.forward(pft.adjoint(y, n), m), n * n * y) < 1e-13


@pytest.mark.parametrize("n,m", [(16, 6), (32, 32), (64, 16), (31, 9)])
def test_adjoint_equals_scaled_ifft_of_zero_padded_window(n, m):
    y = rnd((m, m), 11)
    pad = np.zeros((n, n), complex)
    s = n // 2 - m // 2
    pad[s:s + m, s:s + m] = y
    ref = n * n * np.fft.ifft2(np.fft.ifftshift(pad))
    assert rel(pft.adjoint(y, n), ref) < 1e-13


def test_grouped_equals_per_patch_fft():
    descs, off_in, off_out = [], 0, 0
    rng = np.random.default_rng(9)
    shapes = [(16, 4), (32, 8), (8, 2), (32, 8), (64, 16)]
    for n, m in shapes:
        descs.append((n, m, off_in, off_out))
        off_in += n * n
        off_out += m * m
    flat = rng.standard_normal(off_in) + 1j * rng.standard_normal(off_in)
    out = pft.grouped_forward(descs, flat, off_out)
    for n, m, io, oo in descs:
        ref = fft_crop(flat[io:io + n * n].reshape(n, n), m)
        assert rel(out[oo:oo + m * m].reshape(m, m), ref) < 1e-13
    adj_descs = [(n, m, oo, io) for n, m, io, oo in descs]
    back = pft.grouped_adjoint(adj_descs, out, off_in)
    for n, m, io, oo in descs:
        assert rel(back[io:io + n * n], pft.adjoint(out[oo:oo + m * m].reshape(m, m), n).ravel()) < 1e-14


def test_plausible_mistakes_are_caught():
    """A transposed operand or a flipped sign in the oracle would fail the
    FFT-crop pin; check that the pin can tell them apart."""
    n, m = 32, 12
    psi = rnd((n, n), 21)
    F = pft.twiddles(n, m)
    ref = fft_crop(psi, m)
    assert rel(F @ psi.T @ F.T, ref) > 0.5          # transposed patch
    assert rel(F.conj() @ psi @ F.conj().T, ref) > 0.5  # wrong sign
    Fo = np.exp(-2j * np.pi * np.outer(np.arange(m) - m // 2 + 1, np.arange(n)) / n)
    assert rel(Fo @ psi @ Fo.T, ref) > 0.5          # window off by one


# --- masked full field: DFT period larger than the window (Sec. 4.1.3) -------

@pytest.mark.parametrize("n,N,m,shift", [(8, 24, 10, (5, 11)), (6, 16, 7, (0, 9)), (12, 12, 5, (0, 0))])
def test_period_forward_equals_crop_of_zero_padded_field_fft(n, N, m, shift):
    # the window sits at `shift` in an N x N field of zeros; the kept
    # coefficients are the centred m x m crop of the field's fftshift-ed DFT
    rng = np.random.default_rng(41)
    psi = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    field = np.zeros((N, N), dtype=np.complex128)
    s1, s2 = shift
    field[s1:s1 + n, s2:s2 + n] = psi
    spec = np.fft.fftshift(np.fft.fft2(field))
    lo = N // 2 - m // 2
    ref = spec[lo:lo + m, lo:lo + m]
    got = pft.forward(psi, m, period=N, shift=shift)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_period_equal_to_window_and_no_shift_is_the_plain_transform():
    rng = np.random.default_rng(42)
    psi = rng.standard_normal((3, 16, 16)) + 1j * rng.standard_normal((3, 16, 16))
    assert np.array_equal(pft.forward(psi, 6, period=16), pft.forward(psi, 6))
    y = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    assert np.array_equal(pft.adjoint(y, 16, period=16), pft.adjoint(y, 16))


def test_period_adjoint_identity_with_shift():
    rng = np.random.default_rng(43)
    n, N, m, shift = 10, 32, 9, (7, 20)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    y = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    lhs = np.vdot(pft.forward(x, m, N, shift), y)
    rhs = np.vdot(x, pft.adjoint(y, n, N, shift))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_period_twiddles_reject_a_window_larger_than_the_period():
    with pytest.raises(ValueError):
        pft.twiddles(16, 4, period=8)
