"""FP64 oracle of the paper's polynomial partial Fourier transform
(Sec. 3.1: offline Algorithm 1 and online Algorithm 2 in 1-D; Appendix A:
Algorithms 4 and 5 in 2-D).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What it computes
----------------
With n = p q and the window's corner split as k = q k' + j, the DFT
coefficient at frequency t is

    z^_t = sum_{k'<p} sum_{j<q} z_{qk'+j} e^{-2 pi i t (j - q/2)/n} e^{-2 pi i t k'/p} e^{-pi i t/p}.

The first factor equals e^{pi i x} with x = (t/p)(1 - 2j/q), |x| <= |t|/p.
Replacing e^{pi i x} by a polynomial P(x) = sum_l w_l x^l that is within eps
of it on |x| <= xi, with xi >= m~/p, gives for |t| <= m~

    z^_t ~= sum_l W[t, l] C^[t mod p, l],   C[k', l] = sum_j z_{qk'+j} B[j, l],

B[j, l] = w_l (1 - 2j/q)^l, W[t, l] = (t/p)^l e^{-pi i t/p}, C^ = the p-point
DFT of each column of C.  In 2-D the same substitution is made per axis.
Each coefficient is then within eps * ||z||_1 (1-D) or (2 eps + eps^2) *
||z||_1 (2-D) of the exact DFT.

Readings
--------
* The coefficients w of the best (minimax) approximation come from Park et
  al.'s database in the paper; that database is not available.  Here P is
  the interpolant of e^{pi i x} at the r Chebyshev points of [-xi, xi], a
  near-minimax polynomial, and xi(eps, r) is the largest xi (bisection)
  whose interpolant stays within eps on a dense grid of [-xi, xi].  The
  paper's constant r = 13 at eps = 1e-7, m~/p = 1 holds for it (pinned).
* Window: the outputs are the m coefficients t_c = c - floor(m/2) of the
  exact transform (``pft.window``), so m~ = floor(m/2) = max |t|.
"""

import numpy as np

from . import pft

_GRID = 4001


def chebyshev_poly(xi, r):
    """Monomial coefficients w[0..r-1] (complex) of the degree r-1
    interpolant of e^{pi i x} at the Chebyshev points of [-xi, xi]."""
    nodes = xi * np.cos(np.pi * (np.arange(r) + 0.5) / r)
    V = np.vander(nodes, r, increasing=True)
    return np.linalg.solve(V, np.exp(1j * np.pi * nodes))


def poly_error(w, xi):
    """max |P(x) - e^{pi i x}| over a dense grid of [-xi, xi]."""
    x = np.linspace(-xi, xi, _GRID)
    return float(np.max(np.abs(np.polynomial.polynomial.polyval(x, w) - np.exp(1j * np.pi * x))))


def xi_of(eps, r):
    """xi(eps, r): largest xi whose r-point interpolant is within eps."""
    lo, hi = 0.0, 64.0
    if poly_error(chebyshev_poly(hi, r), hi) <= eps:
        return hi
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if poly_error(chebyshev_poly(mid, r), mid) <= eps:
            lo = mid
        else:
            hi = mid
    return lo


def choose_r(eps, ratio, rmax=25):
    """Algorithm 1, line 2: the least r with xi(eps, r) >= m~/p."""
    for r in range(1, rmax + 1):
        if xi_of(eps, r) >= ratio:
            return r
    raise ValueError("no r <= %d reaches the tolerance" % rmax)


def configure(n, m, p, eps):
    """Algorithm 1 for one axis: (B [q][r], W [m][r], p, q, r, w, xi) for the
    window t_c = c - floor(m/2) of an n-point DFT."""
    if n % p:
        raise ValueError("p must divide n")
    q = n // p
    mt = m // 2
    r = choose_r(eps, mt / p)
    xi = xi_of(eps, r)
    w = chebyshev_poly(xi, r)
    x = 1.0 - 2.0 * np.arange(q) / q
    B = w[None, :] * x[:, None] ** np.arange(r)[None, :]
    t = pft.window(m).astype(np.float64)
    W = (t[:, None] / p) ** np.arange(r)[None, :] * np.exp(-1j * np.pi * t / p)[:, None]
    return dict(B=B, W=W, p=p, q=q, r=r, w=w, xi=xi, m=m, n=n)


def online_1d(z, cfg):
    """Algorithm 2: coefficients t_c of the n-point DFT of z (complex [m])."""
    z = np.asarray(z).astype(np.complex128)
    p, q = cfg["p"], cfg["q"]
    C = z.reshape(p, q) @ cfg["B"]                  # [p][r]
    Ch = np.fft.fft(C, axis=0)                       # p-point DFT of each column
    t = pft.window(cfg["m"])
    return np.sum(Ch[np.mod(t, p), :] * cfg["W"], axis=1)


def online_2d(Z, cfg):
    """Algorithm 5 with the same configuration on both axes: the m x m
    window of the 2-D DFT of each trailing [n][n] slice of Z."""
    Z = np.asarray(Z).astype(np.complex128)
    p, q, r = cfg["p"], cfg["q"], cfg["r"]
    lead = Z.shape[:-2]
    blocks = Z.reshape(lead + (p, q, p, q))                       # [k1][j1][k2][j2]
    C = np.einsum("...ajbk,jl,ks->...abls", blocks, cfg["B"], cfg["B"])   # [k1][k2][l1][l2]
    Ch = np.fft.fft2(C, axes=(-4, -3))                            # 2-D DFT over (k1, k2)
    t = np.mod(pft.window(cfg["m"]), p)
    Cs = Ch[..., t, :, :, :][..., :, t, :, :]                     # [c1][c2][l1][l2]
    return np.einsum("...abls,al,bs->...ab", Cs, cfg["W"], cfg["W"])


def error_bound_2d(Z, eps):
    """Bound on |online_2d - exact| per coefficient: (2 eps + eps^2) ||z||_1."""
    return (2 * eps + eps * eps) * np.sum(np.abs(Z), axis=(-2, -1))
