"""Pins of the FP64 PIE oracle: projection properties (Sec. 2.1, eq. (3)),
the PIE iterate of eq. (5) evaluated with NumPy's full FFT at m = n, the
objective of eq. (4), the fixed point of noise-free data, the band-replacement
closed form, the tie between the PIE step and the loss gradient, and batching
invariances."""

import json
import os

import numpy as np
import pytest

import workloads
from oracle import loss, pft, pie

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def rnd(shape, seed, scale=1.0):
    r = np.random.default_rng(seed)
    return scale * (r.standard_normal(shape) + 1j * r.standard_normal(shape))


def small_case(seed=0, H=40, n=16, grid=3, step=8, offset=2):
    rs = np.random.default_rng(seed)
    obj = (rs.uniform(0.5, 1.0, (H, H)) * np.exp(1j * rs.uniform(-1, 1, (H, H))))
    probe = workloads.gaussian_probe(n, 4.0, 0.05).astype(np.complex128)
    pos = workloads.raster(grid, grid, step, offset)
    # fp64 intensities (the float32 ones of the generators would limit the
    # fixed-point pin to float32 rounding)
    inten = np.stack([np.abs(np.fft.fftshift(np.fft.fft2(probe * obj[r:r + n, c:c + n]))) ** 2
                      for r, c in pos])
    return obj, probe, pos, inten


def test_projection_properties():
    u = rnd((9, 9), 1)
    u[3, 4] = 0.0
    a = np.abs(rnd((9, 9), 2))
    pu = pie.project(u, a)
    assert np.allclose(np.abs(pu), a, atol=1e-14)
    nz = np.abs(u) > 0
    assert np.allclose(np.angle(pu[nz]), np.angle(u[nz]), atol=1e-12)
    assert pu[3, 4] == a[3, 4]                       # theta(0) = 0
    assert np.allclose(pie.project(pu, a), pu, atol=1e-14)   # idempotent
    v = a * np.exp(1j * np.angle(u))
    assert np.allclose(pie.project(v, a), v, atol=1e-14)     # fixed on the set


def test_crop_centre_matches_window():
    n, m = 20, 7
    psi = rnd((n, n), 5)
    spec = np.fft.fftshift(np.fft.fft2(psi))
    assert np.allclose(pie.crop_centre(spec, m), pft.forward(psi, m), atol=1e-11)


def paper_pie_step_fft(z, w, pos, d, beta):
    """Sec. 2.1, eq. (5) for one position with the full DFT: an independent
    route through numpy.fft (d is the fftshift-layout amplitude)."""
    n = w.shape[0]
    r, c = pos
    zj = z[r:r + n, c:c + n]
    ex = w * zj
    spec = np.fft.fftshift(np.fft.fft2(ex))
    pm = np.fft.ifft2(np.fft.ifftshift(d * np.exp(1j * np.angle(spec))))
    out = z.copy()
    out[r:r + n, c:c + n] = zj - beta * np.conj(w) * (ex - pm)
    return out


@pytest.mark.parametrize("beta", [1.0, 0.4])
def test_sequential_full_window_equals_paper_iterate(beta):
    obj, probe, pos, inten = small_case(1)
    d = np.sqrt(inten)
    z0 = obj * np.exp(1j * 0.3 * rnd(obj.shape, 3).real) * 0.9
    n = probe.shape[0]
    got, _, st = pie.pie_sweep(z0, probe, pos, d, n, batch=1, norm=0, beta=beta)
    ref = z0.copy()
    phi_ref = 0.0
    for j in range(len(pos)):
        r, c = pos[j]
        ex = probe * ref[r:r + n, c:c + n]
        spec = np.fft.fftshift(np.fft.fft2(ex))
        pm = np.fft.ifft2(np.fft.ifftshift(d[j] * np.exp(1j * np.angle(spec))))
        phi_ref += np.linalg.norm(ex - pm) ** 2          # eq. (4) summand
        ref = paper_pie_step_fft(ref, probe, pos[j], d[j], beta)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13
    assert abs(st[0] - phi_ref / len(pos)) / (phi_ref / len(pos)) < 1e-12


def test_sequential_full_window_probe_step_equals_paper_simultaneous_form():
    """eq. (6) with the pre-update object patch and the same residual."""
    obj, probe, pos, inten = small_case(2, grid=2)
    d = np.sqrt(inten)
    z0 = obj * 0.8
    w0 = probe * (1 + 0.1 * rnd(probe.shape, 4))
    n = probe.shape[0]
    beta, gamma = 0.7, 0.3
    gz, gw, _ = pie.pie_sweep(z0, w0, pos, d, n, batch=1, norm=0, beta=beta, gamma=gamma)
    z, w = z0.copy(), w0.copy()
    for j in range(len(pos)):
        r, c = pos[j]
        zj = z[r:r + n, c:c + n].copy()
        ex = w * zj
        spec = np.fft.fftshift(np.fft.fft2(ex))
        res = ex - np.fft.ifft2(np.fft.ifftshift(d[j] * np.exp(1j * np.angle(spec))))
        z[r:r + n, c:c + n] = zj - beta * np.conj(w) * res
        w = w - gamma * np.conj(zj) * res
    assert np.linalg.norm(gz - z) / np.linalg.norm(z) < 1e-13
    assert np.linalg.norm(gw - w) / np.linalg.norm(w) < 1e-13


def test_sequential_full_window_probe_step_equals_paper_literal_form():
    """eq. (6) as printed: the probe step at the updated object z_j^{k+1}
    with a recomputed projection (library FFT on the full window)."""
    obj, probe, pos, inten = small_case(2, grid=2)
    d = np.sqrt(inten)
    z0 = obj * 0.8
    w0 = probe * (1 + 0.1 * rnd(probe.shape, 4))
    n = probe.shape[0]
    beta, gamma = 0.7, 0.3
    order = np.array([3, 0, 2, 1])
    gz, gw, _ = pie.pie_sweep(z0, w0, pos, d, n, order=order, batch=1, norm=0, beta=beta, gamma=gamma,
                              probe_update="literal")

    def residual(ex, dj):
        spec = np.fft.fftshift(np.fft.fft2(ex))
        return ex - np.fft.ifft2(np.fft.ifftshift(dj * np.exp(1j * np.angle(spec))))

    z, w = z0.copy(), w0.copy()
    for j in order:
        r, c = pos[j]
        zj = z[r:r + n, c:c + n]
        z[r:r + n, c:c + n] = zj - beta * np.conj(w) * residual(w * zj, d[j])      # eq. (5)
        zj1 = z[r:r + n, c:c + n]
        w = w - gamma * np.conj(zj1) * residual(w * zj1, d[j])                     # eq. (6)
    assert np.linalg.norm(gz - z) / np.linalg.norm(z) < 1e-13
    assert np.linalg.norm(gw - w) / np.linalg.norm(w) < 1e-13
    # and it differs from the simultaneous reading
    _, gs, _ = pie.pie_sweep(z0, w0, pos, d, n, order=order, batch=1, norm=0, beta=beta, gamma=gamma)
    assert np.linalg.norm(gs - w) / np.linalg.norm(w) > 1e-6


def test_literal_probe_update_only_for_sequential_plain_steps():
    obj, probe, pos, inten = small_case(1)
    d = np.sqrt(inten)
    with pytest.raises(ValueError):
        pie.pie_sweep(obj, probe, pos, d, 8, batch=2, gamma=0.5, probe_update="literal")
    with pytest.raises(ValueError):
        pie.pie_sweep(obj, probe, pos, d, 8, norm=1, gamma=0.5, probe_update="literal")


@pytest.mark.parametrize("m,batch,norm,gamma", [(16, 1, 0, 0.0), (8, 9, 1, 0.0), (6, 4, 1, 0.5),
                                                (5, 1, 0, 1.0), (16, 9, 0, 0.2)])
def test_fixed_point_of_noise_free_data(m, batch, norm, gamma):
    obj, probe, pos, inten = small_case(3)
    amp = pie.amplitudes(inten, m)
    O, P, st = pie.pie_sweep(obj, probe, pos, amp, m, batch=batch, norm=norm, beta=0.9,
                             gamma=gamma, alpha=1e-3)
    assert np.linalg.norm(O - obj) / np.linalg.norm(obj) < 1e-12
    assert np.linalg.norm(P - probe) / np.linalg.norm(probe) < 1e-12
    assert st[0] < 1e-20 and st[3] == 0


def test_band_replacement_closed_form():
    """Unit probe, disjoint windows, beta = 1, plain step: the spectrum of the
    updated patch is the old spectrum with its kept window replaced by
    a * exp(i theta) (and, at m = n, the error-reduction modulus step)."""
    n, m = 16, 6
    rs = np.random.default_rng(8)
    obj = rnd((32, 48), 9)
    probe = np.ones((n, n), complex)
    pos = np.array([[0, 0], [16, 0], [0, 16], [16, 32]], dtype=np.int32)
    a_full = np.abs(rnd((len(pos), n, n), 10))
    for mm in (m, n):
        amp = pie.crop_centre(a_full, mm)
        O, _, _ = pie.pie_sweep(obj, probe, pos, amp, mm, batch=1, norm=0, beta=1.0)
        s = n // 2 - mm // 2
        for j, (r, c) in enumerate(pos):
            old = np.fft.fftshift(np.fft.fft2(obj[r:r + n, c:c + n]))
            new = np.fft.fftshift(np.fft.fft2(O[r:r + n, c:c + n]))
            ref = old.copy()
            blk = old[s:s + mm, s:s + mm]
            ref[s:s + mm, s:s + mm] = amp[j] * np.exp(1j * np.angle(blk))
            assert np.linalg.norm(new - ref) / np.linalg.norm(ref) < 1e-13
    assert rs is not None


def test_pie_step_is_scaled_loss_gradient():
    """One position, plain step: O_new - O = -beta / (2 n^2) dL/dO."""
    obj, probe, pos, inten = small_case(4, grid=1)
    m = 7
    amp = pie.amplitudes(inten, m) * 1.3
    z0 = obj * np.exp(0.2j)
    beta = 0.6
    n = probe.shape[0]
    O, _, _ = pie.pie_sweep(z0, probe, pos, amp, m, batch=1, norm=0, beta=beta)
    _, gO, _ = loss.amp_loss_grad(z0, probe, pos, amp, m)
    assert np.linalg.norm((O - z0) + beta / (2 * n * n) * gO) / np.linalg.norm(O - z0) < 1e-12


def test_batched_chunk_is_order_invariant_and_single_position_batches_agree():
    obj, probe, pos, inten = small_case(5)
    amp = pie.amplitudes(inten, 8) * 1.1
    z0 = obj * 0.7
    J = len(pos)
    perm = np.random.default_rng(1).permutation(J)
    a, _, sa = pie.pie_sweep(z0, probe, pos, amp, 8, batch=J, norm=1)
    b, _, sb = pie.pie_sweep(z0, probe, pos, amp, 8, order=perm, batch=J, norm=1)
    assert np.linalg.norm(a - b) / np.linalg.norm(a) < 1e-14
    assert abs(sa[0] - sb[0]) < 1e-12 * sa[0]
    one = pos[:1]
    c, _, _ = pie.pie_sweep(z0, probe, one, amp[:1], 8, batch=1, norm=1)
    d, _, _ = pie.pie_sweep(z0, probe, one, amp[:1], 8, batch=5, norm=1)
    assert np.array_equal(c, d)


def test_overlap_normalised_update_leaves_unlit_pixels():
    obj, probe, pos, inten = small_case(6)
    amp = pie.amplitudes(inten, 8) * 0.5
    z0 = obj.copy()
    O, _, st = pie.pie_sweep(z0, probe, pos, amp, 8, batch=len(pos), norm=1)
    lit = np.zeros(obj.shape, bool)
    n = probe.shape[0]
    for r, c in pos:
        lit[r:r + n, c:c + n] = True
    assert np.array_equal(O[~lit], z0[~lit])
    assert np.linalg.norm(O[lit] - z0[lit]) > 0
    assert abs(pie.rel_change(st) - np.linalg.norm(O - z0) / np.linalg.norm(z0)) < 1e-14


def _doubled_amplitudes(obj, probe, pos):
    """Full-window amplitudes twice the current model's, |fft2(P O_j)| in
    centred order via NumPy's FFT: at m = n the projection then doubles
    every coefficient, so the correction of eq. (3) is the exit wave itself
    (the pseudo-inverse of the whole spectrum is the inverse DFT)."""
    n = probe.shape[0]
    return np.stack([2.0 * np.abs(np.fft.fftshift(np.fft.fft2(probe * obj[r:r + n, c:c + n])))
                     for r, c in pos])


@pytest.mark.parametrize("alpha", [1e-3, 0.25])
def test_batched_overlap_normalised_step_closed_form(alpha):
    """One chunk of overlapping positions, overlap-normalised, with a probe
    step.  With amplitudes twice the model's at m = n the correction of
    position j is psi_j = P O_j, so numO = sum_j |P|^2 O = D O pixel by
    pixel and numP = P E: the step must be
        O' = O (1 + beta D / (D + alpha max D)),
        P' = P (1 + gamma E / (E + alpha max E)),
    with D, E the summed |P|^2 and |O_j|^2.  A denominator of sum |P| (or
    |P| sums squared), a missing conjugate, or a regulariser without the
    maximum each break it."""
    rs = np.random.default_rng(21)
    H, n = 20, 8
    obj = rs.uniform(0.3, 1.2, (H, H)) * np.exp(1j * rs.uniform(-2, 2, (H, H)))
    probe = rs.uniform(0.1, 1.5, (n, n)) * np.exp(1j * rs.uniform(-2, 2, (n, n)))
    # two windows sharing a 5 x 5 corner, a third overlapping both, one apart
    pos = np.array([[0, 0], [3, 3], [6, 1], [12, 12]])
    amp = _doubled_amplitudes(obj, probe, pos)
    beta, gamma = 0.7, 0.4
    O, P, _ = pie.pie_sweep(obj, probe, pos, amp, n, batch=len(pos), norm=1,
                            beta=beta, gamma=gamma, alpha=alpha)
    D = np.zeros((H, H))
    E = np.zeros((n, n))
    for r, c in pos:
        D[r:r + n, c:c + n] += np.abs(probe) ** 2
        E += np.abs(obj[r:r + n, c:c + n]) ** 2
    O_ref = obj * (1.0 + beta * D / (D + alpha * D.max()))
    P_ref = probe * (1.0 + gamma * E / (E + alpha * E.max()))
    assert np.max(np.abs(O - O_ref)) <= 1e-12 * np.max(np.abs(obj))
    assert np.max(np.abs(P - P_ref)) <= 1e-12 * np.max(np.abs(probe))
    # the overlap is real: some pixel is lit by three windows
    cover = np.zeros((H, H), int)
    for r, c in pos:
        cover[r:r + n, c:c + n] += 1
    assert cover.max() == 3
    # plausible mistakes are far from the oracle's answer: sum |P| as the
    # denominator, the regulariser without max D, and conj dropped (the
    # numerator then sums P^2 O instead of |P|^2 O)
    Dabs = np.zeros((H, H))
    S2 = np.zeros((H, H), complex)
    for r, c in pos:
        Dabs[r:r + n, c:c + n] += np.abs(probe)
        S2[r:r + n, c:c + n] += probe ** 2
    for wrong in (obj * (1.0 + beta * D / (Dabs + alpha * Dabs.max())),
                  obj * (1.0 + beta * D / (D + alpha)),
                  obj * (1.0 + beta * S2 / (D + alpha * D.max()))):
        assert np.linalg.norm(wrong - O) > 1e-3 * np.linalg.norm(O)


def test_order_entries_outside_the_scan_contribute_nothing():
    """An order entry outside range(J) keeps its place in its chunk and adds
    nothing: chunks of (a, bad, b) equal chunks of (a, b) when the chunk
    boundaries fall the same way."""
    obj, probe, pos, inten = small_case(14)
    amp = pie.amplitudes(inten, 8)
    J = len(pos)
    perm = np.random.default_rng(4).permutation(J)
    bad = perm.copy()
    bad[2] = J + 5
    z0 = obj * 0.9
    got, _, _ = pie.pie_sweep(z0, probe, pos, amp, 8, order=bad, batch=3, norm=1)
    # the same chunks, the bad entry's position left out of its chunk
    keep = [j for j in bad if j < J]
    ref = z0.astype(np.complex128)
    chunks = [bad[k:k + 3] for k in range(0, J, 3)]
    for ch in chunks:
        ch = [j for j in ch if j < J]
        ref, _, _ = pie.pie_sweep(ref, probe, pos[ch], amp[ch], 8, batch=len(ch), norm=1)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)
    # and the left-out position is not the same as a full permutation's result
    full, _, _ = pie.pie_sweep(z0, probe, pos, amp, 8, order=perm, batch=3, norm=1)
    assert np.linalg.norm(full - got) > 1e-6 * np.linalg.norm(full)
    assert len(keep) == J - 1


def test_rel_error_ignores_global_phase():
    z = rnd((10, 10), 11)
    assert pie.rel_error(z * np.exp(1.234j), z) < 1e-15
    assert abs(pie.rel_error(z * 1.1, z) - 0.1) < 1e-14


def test_hybrid_driver_defaults_and_two_phases():
    g = json.load(open(GOLDEN))
    import inspect
    sig = inspect.signature(pie.hybrid_pie).parameters
    assert sig["iters_pft"].default == g["hybrid_pft_max_iters"]["value"]
    assert sig["tol_pft"].default == g["hybrid_pft_tol"]["value"]
    assert sig["iters_full"].default == g["hybrid_fft_max_iters"]["value"]
    assert sig["tol_full"].default == g["hybrid_fft_tol"]["value"]
    obj, probe, pos, inten = small_case(7)
    z0 = workloads.random_init(np.random.default_rng(3), *obj.shape)
    O, _, hist = pie.hybrid_pie(z0, probe, pos, inten, 8, iters_pft=4, iters_full=3,
                                tol_pft=0.0, tol_full=0.0)
    assert [h[0] for h in hist] == [0] * 4 + [1] * 3
    assert all(np.isfinite(h[2]) for h in hist)
    # the full-resolution objective decreases over phase 2 (Sec. 3.2)
    assert hist[-1][2] <= hist[4][2]


def test_plausible_mistakes_in_the_update_are_caught():
    """A dropped conjugate on the probe or a wrong scale in the pseudo-inverse
    would break the eq. (5) pin: check the pin distinguishes them."""
    obj, probe, pos, inten = small_case(12, grid=1)
    d = np.sqrt(inten)
    n = probe.shape[0]
    z0 = obj * 0.8
    ref = paper_pie_step_fft(z0, probe, pos[0], d[0], 1.0)
    r, c = pos[0]
    u = pft.forward(probe * z0[r:r + n, c:c + n], n)
    corr = pft.adjoint(pie.project(u, d[0]) - u, n)
    for bad in (probe * corr / n ** 2, np.conj(probe) * corr / n):
        z = z0.copy()
        z[r:r + n, c:c + n] += bad
        assert np.linalg.norm(z - ref) / np.linalg.norm(ref) > 1e-3


# --- masked full field (Sec. 4.1.3): the sweep with a DFT period ------------

def _full_field_sweep(obj, probe, pos, amp, m, N, beta, alpha, norm):
    """The masked-field PIE iterate computed on the whole N x N field with
    the library FFT: exit wave = probe on the window, zero elsewhere; only
    the centred m x m band of the field's DFT is projected; the correction
    is the inverse DFT of the band change (1/N^2 included by ifft2),
    restricted to the window.  Sequential single-position chunks."""
    O = obj.astype(np.complex128).copy()
    P = probe.astype(np.complex128)
    n = P.shape[0]
    lo = N // 2 - m // 2
    for j, (r, c) in enumerate(pos):
        field = np.zeros((N, N), dtype=np.complex128)
        field[r:r + n, c:c + n] = P * O[r:r + n, c:c + n]
        spec = np.fft.fftshift(np.fft.fft2(field))
        u = spec[lo:lo + m, lo:lo + m]
        du = np.zeros_like(spec)
        du[lo:lo + m, lo:lo + m] = pie.project(u, amp[j]) - u
        corr = np.fft.ifft2(np.fft.ifftshift(du))[r:r + n, c:c + n]
        num = np.conj(P) * corr
        if norm:
            D = np.abs(P) ** 2
            num = num / (D + alpha * D.max())
        O[r:r + n, c:c + n] += beta * num
    return O


@pytest.mark.parametrize("norm", [0, 1])
def test_masked_field_sweep_equals_full_field_computation(norm):
    rng = np.random.default_rng(44)
    N, n, m = 32, 16, 12
    obj = np.exp(1j * rng.uniform(-1, 1, (N, N)))
    probe = np.exp(-((np.arange(n) - 7.5) ** 2)[:, None] / 40 - ((np.arange(n) - 7.5) ** 2)[None, :] / 40) + 0j
    pos = np.array([[0, 0], [0, 8], [8, 0], [8, 8], [16, 16], [4, 12]])
    true = obj * np.exp(0.3j * rng.standard_normal((N, N)))
    amp = np.empty((len(pos), m, m))
    lo = N // 2 - m // 2
    for j, (r, c) in enumerate(pos):
        field = np.zeros((N, N), dtype=np.complex128)
        field[r:r + n, c:c + n] = probe * true[r:r + n, c:c + n]
        amp[j] = np.abs(np.fft.fftshift(np.fft.fft2(field))[lo:lo + m, lo:lo + m])
    ref = _full_field_sweep(obj, probe, pos, amp, m, N, beta=0.9, alpha=0.05, norm=norm)
    got, _, st = pie.pie_sweep(obj, probe, pos, amp, m, batch=1, norm=norm, beta=0.9, alpha=0.05, period=N)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # phi: mean over positions of the field-space residual energy (Parseval, 1/N^2)
    assert st[0] > 0.0


def test_masked_field_shift_ramp_cancels_in_the_sweep():
    # the update depends on the window's position only through which object
    # pixels it covers: the same sweep with the ramp dropped (all windows
    # treated as unshifted) gives the same object
    rng = np.random.default_rng(45)
    N, n, m = 24, 12, 9
    obj = np.exp(1j * rng.uniform(-1, 1, (N, N)))
    probe = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    pos = np.array([[0, 3], [7, 5], [12, 12]])
    amp = np.abs(rng.standard_normal((3, m, m)))
    a, _, _ = pie.pie_sweep(obj, probe, pos, amp, m, batch=1, norm=1, alpha=0.1, period=N)
    # same arithmetic without the ramp: extraction form with twiddles of period N
    O = obj.astype(np.complex128).copy()
    for j, (r, c) in enumerate(pos):
        psi = probe * O[r:r + n, c:c + n]
        u = pft.forward(psi, m, N)
        d = pft.adjoint(pie.project(u, amp[j]) - u, n, N) / float(N * N)
        D = np.abs(probe) ** 2
        O[r:r + n, c:c + n] += np.conj(probe) * d / (D + 0.1 * D.max())
    assert np.max(np.abs(a - O)) <= 1e-12 * np.max(np.abs(O))
