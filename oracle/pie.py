"""FP64 oracle of the Fourier-magnitude projection, the PIE / ePIE sweep and the
hybrid driver.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings of the paper that this module fixes (each is listed with its reason
in the design notes):

* Projection (Sec. 2.1, eq. (3)): with the partial transform the inverse of a
  cropped spectrum is not defined, so the correction is applied through the
  pseudo-inverse F_m^+ = F_m^H / n^2 and only the kept band is corrected:
      psi' = psi + F_m^H (P(u) - u) conj(F_m) / n^2,   u = F_m psi F_m^T.
  At m = n this is exactly the projection of eq. (3) with the full inverse DFT.
* theta(0) = 0, so the projection of a zero coefficient is the measured
  amplitude itself.
* The probe iterate (eq. (6)) is taken in its simultaneous form: it uses the
  object patch from before the object step and the same residual.
* Batching: positions are processed in consecutive chunks of ``batch``
  positions of the scan order.  Every position of a chunk sees the object and
  probe as they were at the chunk start; their corrections are summed and then
  applied.  ``batch = 1`` with ``norm = 0`` is eq. (5) exactly.
* ``norm = 1`` divides the summed object correction by the summed probe
  intensity (denominator regularised by ``alpha * max``), the usual overlap
  normalisation; ``norm = 0`` is the plain step of eq. (5).
* One iteration is one pass over all positions; the stopping quantity is
  ||z^{k+1} - z^k|| / ||z^k|| over that pass (Sec. 4).
"""

import numpy as np

from . import pft


def project(u, a):
    """Fourier-magnitude projection of Sec. 2.1, eq. (3), on the kept band.

    Returns a * exp(i theta(u)) with theta(0) = 0 (so a zero coefficient maps
    to the real value a).
    """
    u = np.asarray(u).astype(np.complex128)
    a = np.asarray(a).astype(np.float64)
    mag = np.abs(u)
    safe = np.where(mag > 0.0, mag, 1.0)
    return np.where(mag > 0.0, a * (u / safe), a + 0j)


def crop_centre(intensity, m):
    """Centre crop of an fftshift-layout [..., n, n] array to [..., m, m].

    This is the data cropping of Algorithm 3 (Sec. 3.2): rows and columns
    floor(n/2) - floor(m/2) .. + m, i.e. frequencies t = -floor(m/2) ..
    ceil(m/2) - 1 around the zero frequency at index floor(n/2).
    """
    n = intensity.shape[-1]
    s = n // 2 - m // 2
    return intensity[..., s:s + m, s:s + m]


def amplitudes(intensity, m):
    """Cropped amplitudes a_j = sqrt(I_j) on the kept window (Sec. 3.2)."""
    return np.sqrt(np.asarray(crop_centre(intensity, m)).astype(np.float64))


def pie_sweep(obj, probe, pos, amp, m, order=None, batch=1, norm=0,
              beta=1.0, gamma=0.0, alpha=1e-3, period=None, probe_update="simultaneous"):
    """One PIE / ePIE iteration (Sec. 2.1, eqs. (5)-(6)) over all positions.

    obj   [H][W] complex, probe [n][n] complex, pos [J][2] integer top-left
    (row, col) offsets, amp [J][m][m] real cropped amplitudes, order a
    permutation of range(J) or None for scan order.  An order entry outside
    range(J) names no position: it takes its place in its chunk and
    contributes nothing (the chunks stay those of the order as given).

    Returns (obj_new, probe_new, stats) with stats =
    (phi, ||dO||^2, ||O||^2, n_nonfinite):
      phi   = (1/J) sum_j ||psi_j - P_M(psi_j)||^2 (eq. (4)), which with the
              pseudo-inverse equals sum_j ||(|u_j| - a_j)||^2 / (J n^2);
      dO    = object after minus object before the sweep;
      n_nonfinite counts non-finite entries of the new object (and probe).

    period: the masked-field form of the experiments (Sec. 4.1.3): the object
    is the whole N x N field (N = period), exit wave j is the field masked
    to the n x n window at pos[j] (times the probe), its data are the kept
    coefficients of the field's N-point DFT (``pft.forward`` with period N
    and the window's shift ramp), and the correction is the inverse N-point
    DFT of the coefficient change restricted to the window, i.e.
    F_m^H (...) conj(F_m) / N^2 with the conjugate ramp; phi is normalised
    by J N^2.  The ramp is applied literally here even though it cancels
    (the projection keeps it, the adjoint removes it).

    probe_update: "simultaneous" (default) evaluates the probe step of
    eq. (6) with the object and residual of the object step; "literal"
    takes eq. (6) as printed: after the object step of position j, the exit
    wave is formed again from the updated object, projected again, and the
    probe moves along conj(z_j^{k+1}) times that new residual.  The literal
    form is defined for single-position chunks without normalisation
    (batch = 1, norm = 0), which is what eqs. (5)-(6) describe.
    """
    if probe_update not in ("simultaneous", "literal"):
        raise ValueError("probe_update must be 'simultaneous' or 'literal'")
    literal = probe_update == "literal" and gamma > 0.0
    if literal and (batch != 1 or norm != 0):
        raise ValueError("the literal probe update is defined for batch = 1, norm = 0")
    O = np.asarray(obj).astype(np.complex128).copy()
    P = np.asarray(probe).astype(np.complex128).copy()
    pos = np.asarray(pos, dtype=np.int64)
    amp = np.asarray(amp).astype(np.float64)
    n = P.shape[0]
    J = pos.shape[0]
    N = n if period is None else int(period)
    order = np.arange(J) if order is None else np.asarray(order, dtype=np.int64)
    O_start = O.copy()
    phi_acc = 0.0
    for c0 in range(0, J, batch):
        chunk = order[c0:c0 + batch]
        numO = np.zeros_like(O)
        D = np.zeros(O.shape, dtype=np.float64)
        numP = np.zeros_like(P)
        E = np.zeros(P.shape, dtype=np.float64)
        for j in chunk:
            if not 0 <= j < J:
                continue
            r, c = pos[j]
            Oj = O[r:r + n, c:c + n]
            psi = P * Oj                                   # exit wave, eq. (1)
            shift = None if period is None else (r, c)
            u = pft.forward(psi, m, N, shift)
            up = project(u, amp[j])
            phi_acc += float(np.sum((np.abs(u) - amp[j]) ** 2))
            delta = pft.adjoint(up - u, n, N, shift) / float(N * N)  # P_M(psi) - psi
            numO[r:r + n, c:c + n] += np.conj(P) * delta
            D[r:r + n, c:c + n] += np.abs(P) ** 2
            if gamma > 0.0 and not literal:
                numP += np.conj(Oj) * delta
                E += np.abs(Oj) ** 2
        if norm == 0:
            O = O + beta * numO
            if literal:
                # eq. (6) at the updated object: new exit wave, new projection
                (j,) = chunk
                if not 0 <= j < J:
                    continue
                r, c = pos[j]
                Oj = O[r:r + n, c:c + n]
                shift = None if period is None else (r, c)
                u = pft.forward(P * Oj, m, N, shift)
                delta = pft.adjoint(project(u, amp[j]) - u, n, N, shift) / float(N * N)
                P = P + gamma * np.conj(Oj) * delta
            elif gamma > 0.0:
                P = P + gamma * numP
        else:
            # unlit pixels (D = 0) have numO = 0 and stay as they are; a chunk
            # that lights nothing changes nothing
            if D.max() > 0.0:
                O = O + beta * numO / (D + alpha * D.max())
            if gamma > 0.0 and E.max() > 0.0:
                P = P + gamma * numP / (E + alpha * E.max())
    phi = phi_acc / (J * N * N)
    dO2 = float(np.sum(np.abs(O - O_start) ** 2))
    O2 = float(np.sum(np.abs(O_start) ** 2))
    nonfinite = int(np.count_nonzero(~np.isfinite(O)))
    if gamma > 0.0:
        nonfinite += int(np.count_nonzero(~np.isfinite(P)))
    return O, P, (phi, dO2, O2, nonfinite)


def rel_change(stats):
    """Stopping quantity ||z^{k+1} - z^k|| / ||z^k|| of Sec. 4."""
    _, dO2, O2, _ = stats
    return float(np.sqrt(dO2 / O2)) if O2 > 0 else float("inf")


def rel_error(obj, obj_true, mask=None):
    """Relative error ||z - z_true|| / ||z_true|| (Sec. 4.1.2), after removing
    the global phase that the measurements cannot fix.  ``mask`` restricts
    the comparison to illuminated pixels."""
    z = np.asarray(obj).astype(np.complex128)
    zt = np.asarray(obj_true).astype(np.complex128)
    if mask is not None:
        z = z[mask]
        zt = zt[mask]
    ip = np.vdot(z, zt)                     # sum conj(z) * z_true
    ph = ip / abs(ip) if abs(ip) > 0 else 1.0
    return float(np.linalg.norm(z * ph - zt) / np.linalg.norm(zt))


def hybrid_pie(obj0, probe, pos, intensity, m, iters_pft=50, tol_pft=1e-2,
               iters_full=100, tol_full=5e-4, batch=None, norm=1, beta=1.0,
               gamma=0.0, alpha=1e-3, order=None, callback=None):
    """Hybrid PIE of Algorithm 3 (Sec. 3.2).

    Phase 1 crops the data to the central m x m window and runs partial-
    transform sweeps until the relative change drops below ``tol_pft`` or
    ``iters_pft`` sweeps have run; phase 2 starts from that object and runs
    full-resolution sweeps (m = n) on the full data until ``tol_full`` or
    ``iters_full``.  ``intensity`` is [J][n][n] in fftshift layout.
    Returns (obj, probe, history) where history holds one
    (phase, sweep, phi, rel_change) tuple per sweep.
    """
    O = np.asarray(obj0).astype(np.complex128)
    P = np.asarray(probe).astype(np.complex128)
    n = P.shape[0]
    J = len(pos)
    batch = J if batch is None else batch
    history = []
    for phase, (mm, iters, tol) in enumerate(((m, iters_pft, tol_pft),
                                               (n, iters_full, tol_full))):
        amp = amplitudes(intensity, mm)
        for it in range(iters):
            O, P, st = pie_sweep(O, P, pos, amp, mm, order=order, batch=batch,
                                 norm=norm, beta=beta, gamma=gamma, alpha=alpha)
            rc = rel_change(st)
            history.append((phase, it, st[0], rc))
            if callback is not None:
                callback(phase, it, O, P, st)
            if rc < tol:
                break
    return O, P, history
