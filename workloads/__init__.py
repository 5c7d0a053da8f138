"""Seeded synthetic inputs shaped like the paper's ptychography workloads.

This module holds input recipes only: objects, probes, scan positions,
simulated measurements and random initial guesses.  It contains none of the
partial-transform or PIE arithmetic.  It is the one module that both the
checked path (the HIP library through its binding) and the FP64 oracle read
their inputs from.

The measured intensities are simulated with NumPy's full FFT of the true exit
waves (the measurement model of Sec. 2, eq. (1)); the transform under test is
never used to make its own inputs.

All arrays come out as complex64 / float32 / int32 (what the library takes);
the oracle upcasts the same values.

Stand-ins: the paper's test images (a baboon magnitude and a cameraman phase,
Sec. 4) are not available; the smooth synthetic amplitude / phase objects
below stand in for them with the same kind of content and value ranges.
"""

import numpy as np

# ----------------------------------------------------------------------------
# basic pieces


def streams(k):
    """Six independent generators for configuration k, in the order
    [object, probe, scan, noise, init, perturb]."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(k).spawn(6)]


def _radius2(n):
    c = (n - 1) / 2.0
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    return (y - c) ** 2 + (x - c) ** 2


def gaussian_probe(n, sigma, kappa):
    """Gaussian amplitude exp(-r^2 / 2 sigma^2) (the probe form of Sec. 4.2.1)
    with quadratic phase kappa r^2; peak amplitude 1."""
    r2 = _radius2(n)
    return (np.exp(-r2 / (2.0 * sigma * sigma)) * np.exp(1j * kappa * r2)).astype(np.complex64)


def aperture_probe(n, radius, kappa):
    """Circular aperture (1 inside radius, 0 outside; the circular windows of
    Sec. 4.2.1) with quadratic phase kappa r^2."""
    r2 = _radius2(n)
    amp = (r2 <= radius * radius).astype(np.float64)
    return (amp * np.exp(1j * kappa * r2)).astype(np.complex64)


def blob_object(rng, h, w, nblobs=5):
    """Amplitude iid U[0.8, 1]; phase a sum of ``nblobs`` Gaussian blobs with
    centres U[0, size), widths U[6, 20] px and heights U[-1, 1], rescaled so
    that max |phase| = pi/2."""
    amp = rng.uniform(0.8, 1.0, size=(h, w))
    cy = rng.uniform(0, h, size=nblobs)
    cx = rng.uniform(0, w, size=nblobs)
    s = rng.uniform(6.0, 20.0, size=nblobs)
    A = rng.uniform(-1.0, 1.0, size=nblobs)
    y, x = np.mgrid[0:h, 0:w].astype(np.float64)
    ph = np.zeros((h, w))
    for b in range(nblobs):
        ph += A[b] * np.exp(-((y - cy[b]) ** 2 + (x - cx[b]) ** 2) / (2.0 * s[b] ** 2))
    ph *= (np.pi / 2.0) / np.max(np.abs(ph))
    return (amp * np.exp(1j * ph)).astype(np.complex64)


def smooth_phase_object(rng, h, w, sigma_f):
    """Pure phase object |O| = 1: iid N(0,1) field low-passed by a periodic
    Gaussian of width ``sigma_f`` px (applied in Fourier space), rescaled so
    that max |phase| = pi/2."""
    f = rng.standard_normal((h, w))
    fy = np.fft.fftfreq(h)[:, None]
    fx = np.fft.fftfreq(w)[None, :]
    filt = np.exp(-2.0 * np.pi ** 2 * sigma_f ** 2 * (fy ** 2 + fx ** 2))
    ph = np.real(np.fft.ifft2(np.fft.fft2(f) * filt))
    ph *= (np.pi / 2.0) / np.max(np.abs(ph))
    return np.exp(1j * ph).astype(np.complex64)


def raster(ny, nx, step, offset, rng=None, jitter=0):
    """Row-major raster of top-left (row, col) offsets, j = nx*iy + ix, with
    optional integer jitter U{-jitter..jitter} per axis per position."""
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([offset + step * iy.ravel(), offset + step * ix.ravel()], axis=1)
    if jitter:
        pos = pos + rng.integers(-jitter, jitter + 1, size=pos.shape)
    return pos.astype(np.int32)


def intensities(obj, probe, pos):
    """Simulated far-field intensities |FFT2(P * O_j)|^2 in fftshift layout
    (zero frequency at index floor(n/2)), float32 [J][n][n]."""
    n = probe.shape[0]
    P = probe.astype(np.complex128)
    out = np.empty((len(pos), n, n), dtype=np.float32)
    for j, (r, c) in enumerate(pos):
        ex = P * obj[r:r + n, c:c + n].astype(np.complex128)
        out[j] = np.abs(np.fft.fftshift(np.fft.fft2(ex))) ** 2
    return out


def poisson(rng, intensity, photons):
    """Poisson counts with one global scale so that the mean total count per
    pattern equals ``photons``; returned rescaled to the input's units."""
    s = photons / float(np.mean(np.sum(intensity.astype(np.float64), axis=(1, 2))))
    return (rng.poisson(s * intensity.astype(np.float64)) / s).astype(np.float32)


def random_init(rng, h, w):
    """Initial guess of Sec. 4.1.2: magnitude U[0,1], phase U[0, pi/2]."""
    amp = rng.uniform(0.0, 1.0, size=(h, w))
    ph = rng.uniform(0.0, np.pi / 2.0, size=(h, w))
    return (amp * np.exp(1j * ph)).astype(np.complex64)


def complex_normal(rng, shape):
    """Re / Im iid N(0,1), drawn in float32 directly, as complex64."""
    z = rng.standard_normal(tuple(shape) + (2,), dtype=np.float32)
    return z.view(np.complex64).reshape(shape)


# ----------------------------------------------------------------------------
# the five workloads


def tiny_pie(seed=1):
    """Plain PIE, tiny: 128^2 blob object, 32^2 Gaussian probe (sigma 6 px,
    kappa = pi/144), 8 x 8 raster step 8 from offset 20, noise-free data,
    window m = 16.  The amplitudes are cropped by each side itself (the data
    cropping of Algorithm 3 is a step of the method, not an input)."""
    rs = streams(seed)
    obj = blob_object(rs[0], 128, 128)
    probe = gaussian_probe(32, 6.0, np.pi / 144.0)
    pos = raster(8, 8, 8, 20)
    inten = intensities(obj, probe, pos)
    init = random_init(rs[4], 128, 128)
    return dict(obj=obj, probe=probe, pos=pos, intensity=inten, m=16, init=init)


PFT_BLOCK = 64   # patches per seeded block of the standalone-transform batch


def pft_patches(n, idx, seed=2):
    """Patches ``idx`` of the standalone batch, complex64 [len(idx)][n][n].
    Patch b is row b % 64 of block b // 64, drawn from SeedSequence([seed, 0,
    block]); any subset can be regenerated without the rest."""
    idx = np.asarray(idx, dtype=np.int64)
    out = np.empty((len(idx), n, n), dtype=np.complex64)
    for blk in np.unique(idx // PFT_BLOCK):
        rng = np.random.default_rng(np.random.SeedSequence([seed, 0, int(blk)]))
        block = complex_normal(rng, (PFT_BLOCK, n, n))
        sel = np.nonzero(idx // PFT_BLOCK == blk)[0]
        out[sel] = block[idx[sel] % PFT_BLOCK]
    return out


def pft_coeffs(m, idx, seed=2):
    """Adjoint inputs: independent iid blocks [len(idx)][m][m], from
    SeedSequence([seed, 1, block])."""
    idx = np.asarray(idx, dtype=np.int64)
    out = np.empty((len(idx), m, m), dtype=np.complex64)
    for blk in np.unique(idx // PFT_BLOCK):
        rng = np.random.default_rng(np.random.SeedSequence([seed, 1, int(blk)]))
        block = complex_normal(rng, (PFT_BLOCK, m, m))
        sel = np.nonzero(idx // PFT_BLOCK == blk)[0]
        out[sel] = block[idx[sel] % PFT_BLOCK]
    return out


def pie_at_scale(seed=3, photons=1e4):
    """Warm-started PIE at scale: 1024^2 smooth phase object (sigma_f 24 px),
    128^2 circular aperture probe (radius 40, kappa = pi/1600), 30 x 30 raster
    step 24 from offset 100 with +-2 px jitter, Poisson data at ``photons``
    per pattern (None: noise-free), phase-1 window m = 32."""
    rs = streams(seed)
    obj = smooth_phase_object(rs[0], 1024, 1024, 24.0)
    probe = aperture_probe(128, 40.0, np.pi / 1600.0)
    pos = raster(30, 30, 24, 100, rng=rs[2], jitter=2)
    inten = intensities(obj, probe, pos)
    if photons is not None:
        inten = poisson(rs[3], inten, photons)
    init = random_init(rs[4], 1024, 1024)
    return dict(obj=obj, probe=probe, pos=pos, intensity=inten, m=32, init=init)


def amp_loss_case(seed=4, size=2304, n=256, m=64, grid=32, step=64, offset=32,
                  radius=80.0, sigma_f=48.0):
    """Differentiable amplitude loss: phase object (sigma_f 48 px) on a 2304^2
    grid, 256^2 aperture probe (radius 80, kappa = pi/6400), 32 x 32 raster
    step 64 from offset 32 (J = 1024), noise-free 64 x 64 amplitudes; the
    evaluation point perturbs object (0.1 N(0,1) complex) and probe (0.05,
    on the aperture).  Smaller instances reuse the recipe with other sizes."""
    rs = streams(seed)
    obj_t = smooth_phase_object(rs[0], size, size, sigma_f)
    kappa = np.pi / (radius * radius)
    probe_t = aperture_probe(n, radius, kappa)
    pos = raster(grid, grid, step, offset)
    amp = np.empty((len(pos), m, m), dtype=np.float32)
    s = n // 2 - m // 2
    P = probe_t.astype(np.complex128)
    for j, (r, c) in enumerate(pos):
        spec = np.fft.fftshift(np.fft.fft2(P * obj_t[r:r + n, c:c + n].astype(np.complex128)))
        amp[j] = np.abs(spec[s:s + m, s:s + m])
    w = rs[5].standard_normal((2, size, size))
    obj = (obj_t.astype(np.complex128) + 0.1 * (w[0] + 1j * w[1])).astype(np.complex64)
    v = rs[5].standard_normal((2, n, n))
    on = np.abs(probe_t) > 0
    probe = (probe_t.astype(np.complex128) + 0.05 * on * (v[0] + 1j * v[1])).astype(np.complex64)
    return dict(obj=obj, probe=probe, pos=pos, amp=amp, m=m,
                obj_true=obj_t, probe_true=probe_t)


GROUP_SIZES = (64, 128, 256, 512)


def grouped_descs(count=8192, seed=5, sizes=GROUP_SIZES):
    """Uneven batch: ``count`` descriptors, sizes a seeded permutation of
    equal shares of ``sizes``, m = n/4, packed in descriptor order.
    Returns int64 [count][4] rows (n, m, in_offset, out_offset) for the
    forward direction, plus the total input / output lengths (complex
    elements).  Every offset is a multiple of 32 elements (256 bytes)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0]))
    share = count // len(sizes)
    ns = rng.permutation(np.repeat(np.asarray(sizes, dtype=np.int64), share))
    ms = ns // 4
    in_sz = ns * ns
    out_sz = ms * ms
    in_off = np.concatenate([[0], np.cumsum(in_sz)[:-1]])
    out_off = np.concatenate([[0], np.cumsum(out_sz)[:-1]])
    desc = np.stack([ns, ms, in_off, out_off], axis=1).astype(np.int64)
    return desc, int(in_sz.sum()), int(out_sz.sum())


def grouped_inputs(desc, total, idx=None, seed=5, adjoint=False):
    """Packed complex64 inputs of the uneven batch: patch i (or coefficient
    block i when ``adjoint``) is iid complex normal from SeedSequence([seed,
    1 or 2, i]).  With ``idx`` only those entries are filled (others zero)."""
    out = np.zeros(total, dtype=np.complex64)
    idx = range(len(desc)) if idx is None else idx
    for i in idx:
        n, m, io, _ = (int(v) for v in desc[i])
        side = m if adjoint else n
        rng = np.random.default_rng(np.random.SeedSequence([seed, 2 if adjoint else 1, int(i)]))
        out[io:io + side * side] = complex_normal(rng, (side * side,))
    return out


def adjoint_descs(desc):
    """The same uneven batch for the adjoint direction: input blocks are the
    m x m coefficient blocks, outputs the n x n patches."""
    d = np.asarray(desc, dtype=np.int64)
    return np.stack([d[:, 0], d[:, 1], d[:, 3], d[:, 2]], axis=1)


def serpentine(k, step, by_rows=False):
    """k x k window corners, column by column: down the first column, up the
    second, down the third, ... (the scan of the non-blind experiments,
    Sec. 4.1.1); by_rows: along the first row to the right, back along the
    second, ... (the blind experiments), as (row, col) offsets [k*k][2]."""
    pos = []
    for a in range(k):
        seq = range(k) if a % 2 == 0 else range(k - 1, -1, -1)
        pos += [(step * a, step * b) if by_rows else (step * b, step * a) for b in seq]
    return np.asarray(pos, dtype=np.int32)


def masked_field_amplitudes(field_img, probe, pos, m, period, workers=-1):
    """|kept m x m coefficients| of the period-point 2-D DFT of each masked
    field (probe on the window at pos[j], zero elsewhere), float32 [J][m][m].
    The window's position only multiplies the coefficients by a phase, so
    each window is transformed at the origin: zero-padded row transforms of
    length `period` keep the m centred columns, then zero-padded column
    transforms keep the m centred rows (library FFT, complex64)."""
    import scipy.fft as sfft
    n = probe.shape[0]
    keep = (np.arange(m) - m // 2) % period
    out = np.empty((len(pos), m, m), dtype=np.float32)
    for j, (r, c) in enumerate(pos):
        rows = np.empty((n, m), dtype=np.complex64)
        for r0 in range(0, n, 512):
            blk = probe[r0:r0 + 512] * field_img[r + r0:r + r0 + min(512, n - r0), c:c + n]
            rows[r0:r0 + 512] = sfft.fft(blk, n=period, axis=1, workers=workers)[:, keep]
        out[j] = np.abs(sfft.fft(rows, n=period, axis=0, workers=workers)[keep, :])
    return out


def masked_field(seed=6, field=16384, m=128, coarse=1024, sigma_f=24.0, amp_positions=None, with_init=True):
    """Non-blind masked-field workload (the large experiment of Sec. 4.1.3):
    a field x field pure-phase object (smooth random phase made on a
    coarse x coarse grid with sigma_f px and interpolated bilinearly),
    identity probe on field/2 x field/2 windows, 3 x 3 serpentine scan with
    shift field/4 (9 positions, 50 % overlap), noise-free amplitudes of the
    centred m x m coefficients of each masked field's field-point DFT, and a
    random initial object.  amp_positions (indices into pos) limits the
    amplitudes to those windows; with_init=False skips the initial object."""
    from scipy.ndimage import zoom
    rs = streams(seed)
    n = field // 2
    ph = np.angle(smooth_phase_object(rs[0], coarse, coarse, sigma_f)).astype(np.float32)
    ph = zoom(ph, field / coarse, order=1, mode="grid-wrap", grid_mode=True)
    obj = np.exp(1j * ph).astype(np.complex64)
    del ph
    probe = np.ones((n, n), dtype=np.complex64)
    pos = serpentine(3, field // 4)
    sel = pos if amp_positions is None else pos[np.asarray(amp_positions)]
    amp = masked_field_amplitudes(obj, probe, sel, m, field)
    init = random_init(rs[4], field, field) if with_init else None
    return dict(obj=obj, probe=probe, pos=pos, amp=amp, m=m, period=field, init=init)


def circular_probe(n, radius, sigma=1e6):
    """Circular illumination window of the blind experiments (Sec. 4.2.1, Appendix B): the
    Gaussian exp(-r^2 / 2 sigma^2) inside a circle of `radius` px (sigma =
    1e6: flat), zero outside."""
    r2 = _radius2(n)
    return ((r2 <= radius * radius) * np.exp(-r2 / (2.0 * sigma * sigma))).astype(np.complex64)


def blind_circular(seed=7, n=128, radius=58.0, shift=50, grid=4, m=32):
    """Blind ePIE with circular windows (Sec. 4.2.3), scaled so the full
    window fits the full-resolution phase: 4 x 4 windows of n = 128 with a
    flat circular probe of radius 58 shifted by 50 px (about the paper's
    radius / shift ratio 175 / 150 and 50 % overlap), row-wise serpentine
    scan, object padded to cover every window (3 * 50 + 128 = 278 px),
    amplitude U[0.8, 1] with phase blobs in [-pi/2, pi/2], noise-free data;
    initial object as Sec. 4.1.2, initial probe a flat circle of 0.8 times
    the radius.  PFT window m."""
    rs = streams(seed)
    size = shift * (grid - 1) + n
    obj = blob_object(rs[0], size, size)
    probe = circular_probe(n, radius)
    pos = serpentine(grid, shift, by_rows=True)
    inten = intensities(obj, probe, pos)
    init = random_init(rs[4], size, size)
    probe0 = circular_probe(n, 0.8 * radius)
    return dict(obj=obj, probe=probe, pos=pos, intensity=inten, m=m, init=init, probe_init=probe0)

