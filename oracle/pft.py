"""FP64 oracle of the 2-D partial DFT and its adjoint.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the partial transform computes
-----------------------------------
The paper's PFT (Sec. 3.1; Appendix A) returns the Fourier coefficients of the
low-frequency window that the full 2-D DFT (Appendix A, eq. (16); 1-D form
Sec. 3.1.1, eq. (7)) would give, without forming the full DFT (Fig. 2).  Its
polynomial scheme only approximates those coefficients to a tolerance; the
exact target is the plain DFT sum restricted to the kept frequencies, and that
sum is what this module evaluates.

Window convention (the paper writes the window as [-m~, m~] yet counts 128
coefficients for m~ = 64, Sec. 3.1.2; we read ``m`` as the number of kept
coefficients per axis):

    t_c = c - floor(m/2),   c = 0 .. m-1

which is exactly the centred crop of an fftshift-ed spectrum.  The output is
stored in that centred order, row-major ``[c1][c2]``, axis 0 = rows.  The
spatial index k runs over 0 .. n-1 from the patch's top-left corner, as in the
paper's sums.
"""

import numpy as np


def window(m):
    """Kept frequencies t_c = c - floor(m/2) for c = 0..m-1 (centred order)."""
    if m < 1:
        raise ValueError("m must be >= 1")
    return np.arange(m, dtype=np.int64) - (m // 2)


def twiddles(n, m, period=None):
    """Partial DFT matrix F_m[c, k] = exp(-2 pi i t_c k / N), shape [m][n],
    with DFT length N = ``period`` (default n).

    The DFT kernel of Sec. 3.1.1, eq. (7), restricted to the kept rows t_c.
    A period N > n is the masked full field of the paper's experiments
    (Sec. 4.1.3: an n x n illuminated window inside an N x N field, every
    other pixel zero): the field's DFT at frequency t only sums the window's
    pixels, k = 0..n-1 counted from the window's corner.  The phase t_c*k is
    reduced modulo N in integer arithmetic before the trigonometric call, so
    the argument stays in [0, 2 pi).
    """
    N = n if period is None else int(period)
    if not (1 <= n <= N and 1 <= m <= N):
        raise ValueError("need 1 <= n <= period and 1 <= m <= period")
    t = window(m)
    k = np.arange(n, dtype=np.int64)
    phase_int = np.mod(np.outer(t, k), N)          # exact integer reduction
    return np.exp(-2j * np.pi * phase_int.astype(np.float64) / N)


def shift_ramp(m, shift, period):
    """Phase of the window's position in the field: R[c1, c2] =
    exp(-2 pi i (t_c1 s1 + t_c2 s2) / N) for a window whose corner sits at
    field pixel (s1, s2) (the DFT shift theorem), reduced modulo N."""
    t = window(m)
    s1, s2 = (int(v) for v in shift)
    r1 = np.exp(-2j * np.pi * np.mod(t * s1, period).astype(np.float64) / period)
    r2 = np.exp(-2j * np.pi * np.mod(t * s2, period).astype(np.float64) / period)
    return np.outer(r1, r2)


def forward(psi, m, period=None, shift=None):
    """Y = F_m psi F_m^T for each trailing [n][n] slice (Appendix A, eq. (16)).

    psi: array [..., n, n] (any complex/real dtype; upcast to complex128).
    Returns complex128 [..., m, m]:
        Y[c1, c2] = sum_{k1,k2} psi[k1,k2] exp(-2 pi i (t_c1 k1 + t_c2 k2)/N).
    The 2-D sum factorises into one DFT per axis, so it is two matrix
    products with the same partial DFT matrix.  With a period N > n and the
    window's corner ``shift`` = (s1, s2) in the N x N field, Y is further
    multiplied by ``shift_ramp``: the kept coefficients of the whole masked
    field.
    """
    psi = np.asarray(psi).astype(np.complex128)
    n = psi.shape[-1]
    if psi.shape[-2] != n:
        raise ValueError("patches must be square")
    N = n if period is None else int(period)
    F = twiddles(n, m, N)
    y = F @ psi @ F.T
    if shift is not None:
        y = y * shift_ramp(m, shift, N)
    return y


def adjoint(y, n, period=None, shift=None):
    """X = F_m^H Y conj(F_m): the adjoint of ``forward`` (no normalisation).

    y: array [..., m, m].  Returns complex128 [..., n, n]:
        X[k1, k2] = sum_{c1,c2} Y[c1,c2] exp(+2 pi i (t_c1 k1 + t_c2 k2)/N),
    after multiplying Y by the conjugate ``shift_ramp`` when a shift is given.
    """
    y = np.asarray(y).astype(np.complex128)
    m = y.shape[-1]
    if y.shape[-2] != m:
        raise ValueError("coefficient blocks must be square")
    N = n if period is None else int(period)
    if shift is not None:
        y = y * np.conj(shift_ramp(m, shift, N))
    F = twiddles(n, m, N)
    return F.conj().T @ y @ F.conj()


def forward_direct(psi, m):
    """The 2-D DFT sum of Appendix A, eq. (16), as four nested loops.

    Only for tiny patches (n <= 16): it is the definition written out term by
    term, used to pin ``forward``.
    """
    psi = np.asarray(psi).astype(np.complex128)
    n = psi.shape[-1]
    t = window(m)
    out = np.zeros((m, m), dtype=np.complex128)
    for c1 in range(m):
        for c2 in range(m):
            acc = 0j
            for k1 in range(n):
                for k2 in range(n):
                    ang = -2.0 * np.pi * (t[c1] * k1 + t[c2] * k2) / n
                    acc += psi[k1, k2] * complex(np.cos(ang), np.sin(ang))
            out[c1, c2] = acc
    return out


def grouped_forward(descs, flat_in, flat_out_size):
    """Forward transform of a packed list of patches of differing sizes.

    descs: iterable of (n, m, in_offset, out_offset), offsets in complex
    elements of the flat input / output arrays.  Each descriptor is one
    independent ``forward`` call; returns the packed complex128 output.
    """
    flat_in = np.asarray(flat_in)
    out = np.zeros(flat_out_size, dtype=np.complex128)
    for n, m, io, oo in descs:
        patch = flat_in[io:io + n * n].reshape(n, n)
        out[oo:oo + m * m] = forward(patch, m).reshape(-1)
    return out


def grouped_adjoint(descs, flat_in, flat_out_size):
    """Adjoint counterpart of ``grouped_forward``: input blocks are [m][m]."""
    flat_in = np.asarray(flat_in)
    out = np.zeros(flat_out_size, dtype=np.complex128)
    for n, m, io, oo in descs:
        blk = flat_in[io:io + m * m].reshape(m, m)
        out[oo:oo + n * n] = adjoint(blk, n).reshape(-1)
    return out
