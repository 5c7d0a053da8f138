"""FP64 oracle of the amplitude loss and its gradient.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper needs derivatives through the partial transform (Sec. 1.1) and views
the PIE iterates as gradient steps on its objective (Sec. 2.1, remark after
eq. (6)).  The loss differentiated here is

    L(O, P) = sum_j || |F_m (P * O_j) F_m^T| - a_j ||^2,

with O_j the n x n window of the object at position j.  Gradients follow the
convention grad = dL/dRe + i dL/dIm (= 2 dL/d conj(z)), so that the
directional derivative along V is Re <grad, V>.  The subgradient of |u| at
u = 0 is taken as 0 (sgn(0) = 0).

Closed form (chain rule through the linear map u = F_m psi F_m^T):
    G_u = 2 (u - a * sgn(u)),  R_j = F_m^H G_u conj(F_m),
    dL/dO[window j] += conj(P) * R_j,   dL/dP += conj(O_j) * R_j.
"""

import numpy as np

from . import pft


def _sgn(u):
    mag = np.abs(u)
    return np.where(mag > 0.0, u / np.where(mag > 0.0, mag, 1.0), 0.0)


def amp_loss(obj, probe, pos, amp, m):
    """L = sum_j || |u_j| - a_j ||^2 with u_j = F_m (P * O_j) F_m^T."""
    O = np.asarray(obj).astype(np.complex128)
    P = np.asarray(probe).astype(np.complex128)
    amp = np.asarray(amp).astype(np.float64)
    n = P.shape[0]
    L = 0.0
    for j, (r, c) in enumerate(np.asarray(pos, dtype=np.int64)):
        u = pft.forward(P * O[r:r + n, c:c + n], m)
        L += float(np.sum((np.abs(u) - amp[j]) ** 2))
    return L


def amp_loss_grad(obj, probe, pos, amp, m):
    """Returns (L, dL/dO [H][W], dL/dP [n][n]) in the convention above."""
    O = np.asarray(obj).astype(np.complex128)
    P = np.asarray(probe).astype(np.complex128)
    amp = np.asarray(amp).astype(np.float64)
    n = P.shape[0]
    gO = np.zeros_like(O)
    gP = np.zeros_like(P)
    L = 0.0
    for j, (r, c) in enumerate(np.asarray(pos, dtype=np.int64)):
        Oj = O[r:r + n, c:c + n]
        u = pft.forward(P * Oj, m)
        L += float(np.sum((np.abs(u) - amp[j]) ** 2))
        R = pft.adjoint(2.0 * (u - amp[j] * _sgn(u)), n)
        gO[r:r + n, c:c + n] += np.conj(P) * R
        gP += np.conj(Oj) * R
    return L, gO, gP
