"""Python binding of the PIE / ePIE sweep and the hybrid driver.

The sweep (Sec. 2.1 of the paper: projection eq. (3), objective eq. (4),
iterates eqs. (5)-(6)) runs entirely in the HIP library; this module builds
scans, sizes workspaces and reads back the three per-sweep statistics the
stopping rule of Sec. 4 needs.
"""

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from .pft import _require, _stream_ptr, get_plan


@dataclass
class PieParams:
    """batch: positions per chunk (1 = sequential eq. (5), J = fully batched);
    norm: 0 plain step, 1 overlap-normalised; beta / gamma: object / probe
    steps (gamma = 0: probe fixed); alpha: denominator regulariser;
    probe_update: "simultaneous" (eq. (6) with the object and residual of
    the object step) or "literal" (eq. (6) as printed, at the updated object;
    batch 1, norm 0)."""
    batch: int = 1
    norm: int = 0
    beta: float = 1.0
    gamma: float = 0.0
    alpha: float = 1e-3
    probe_update: str = "simultaneous"

    def c(self):
        modes = {"simultaneous": 0, "literal": 1}
        if self.probe_update not in modes:
            raise ValueError("probe_update must be 'simultaneous' or 'literal'")
        return _lib.PieParams(int(self.batch), int(self.norm), float(self.beta), float(self.gamma),
                              float(self.alpha), modes[self.probe_update])


class Scan:
    """Scan positions (top-left (row, col) of each n x n window) inside an
    H x W object, bound to the plan of (n, m, precision, method, period); see
    ``pft.Plan`` for the method and the masked-field period."""

    def __init__(self, pos, obj_shape, n, m, precision="fp32", device=None, method="auto", period=None):
        pos = np.ascontiguousarray(np.asarray(pos, dtype=np.int32))
        if pos.ndim != 2 or pos.shape[1] != 2:
            raise ValueError("pos must be [J][2]")
        self.pos = pos
        self.J = pos.shape[0]
        self.H, self.W = (int(v) for v in obj_shape)
        self.plan = get_plan(n, m, precision, device, method, period)
        self.n, self.m, self.precision = self.plan.n, self.plan.m, precision
        h = _lib.c_scan()
        with torch.cuda.device(self.plan.device):
            _lib.call("pie_scan_create", self.plan.handle,
                      pos.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), self.J, self.H, self.W,
                      ctypes.byref(h))
        self.handle = h
        self._ws = {}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.lib().pie_scan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, params):
        nb = ctypes.c_size_t()
        cp = params.c()
        _lib.call("pie_workspace_size", self.handle, ctypes.byref(cp), ctypes.byref(nb))
        return nb.value

    def workspace(self, params):
        """A cached device workspace big enough for ``params``."""
        need = self.workspace_bytes(params)
        ws = self._ws.get("pie")
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.plan.device)
            self._ws["pie"] = ws
        return ws


def crop_amplitudes(intensity, m):
    """sqrt of the centred m x m crop of fftshift-layout intensities
    [J][n][n] -> [J][m][m] (the data cropping of Algorithm 3)."""
    _require(intensity, "intensity", torch.float32)
    J, n = intensity.shape[0], intensity.shape[-1]
    out = torch.empty(J, m, m, dtype=torch.float32, device=intensity.device)
    _lib.call("pie_crop_amplitudes", ctypes.c_void_p(intensity.data_ptr()), J, n, m,
              ctypes.c_void_p(out.data_ptr()), _stream_ptr(intensity))
    return out


def pie_sweep(obj, probe, scan, amp, params, order=None, stats=None, workspace=None):
    """One sweep over every position, updating obj (and probe when
    params.gamma > 0) in place.  Returns the device float64 stats tensor
    {Phi, ||dO||^2, ||O||^2, n_nonfinite}."""
    _require(obj, "obj")
    _require(probe, "probe")
    _require(amp, "amp", torch.float32)
    if tuple(obj.shape) != (scan.H, scan.W):
        raise ValueError(f"obj must be ({scan.H}, {scan.W})")
    if tuple(probe.shape) != (scan.n, scan.n):
        raise ValueError(f"probe must be ({scan.n}, {scan.n})")
    if tuple(amp.shape) != (scan.J, scan.m, scan.m):
        raise ValueError(f"amp must be ({scan.J}, {scan.m}, {scan.m})")
    if order is not None:
        _require(order, "order", torch.int32)
        if order.numel() != scan.J:
            raise ValueError("order must hold J entries")
    if stats is None:
        stats = torch.zeros(4, dtype=torch.float64, device=obj.device)
    ws = scan.workspace(params) if workspace is None else workspace
    cp = params.c()
    _lib.call("pie_sweep", scan.handle, ctypes.c_void_p(obj.data_ptr()), ctypes.c_void_p(probe.data_ptr()),
              ctypes.c_void_p(amp.data_ptr()),
              ctypes.c_void_p(order.data_ptr() if order is not None else 0),
              ctypes.byref(cp), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
              ctypes.c_void_p(stats.data_ptr()), _stream_ptr(obj))
    return stats


def rel_change(stats_host):
    """Stopping quantity ||z^{k+1} - z^k|| / ||z^k|| (Sec. 4)."""
    _, d2, o2, _ = stats_host
    return float(np.sqrt(d2 / o2)) if o2 > 0 else float("inf")


def hybrid_pie(obj, probe, pos, intensity, m, iters_pft=50, tol_pft=1e-2, iters_full=100,
               tol_full=5e-4, params=None, full_params=None, order=None, callback=None,
               precision="fp32", full_method="auto", order_seed=0):
    """Hybrid PIE of Algorithm 3 (Sec. 3.2), on the device.

    Phase 1 runs partial-transform sweeps on the central m x m window of the
    data until the relative change falls below tol_pft or iters_pft sweeps;
    phase 2 starts from that object and runs full-window sweeps (m = n) on
    the full data until tol_full or iters_full.  obj / probe are updated in
    place; intensity is a device float32 [J][n][n] fftshift-layout tensor.
    Phase 2 uses the fast full-window transform where it applies
    (full_method "auto"; "dense" forces the contraction at m = n).
    order: None (scan order), a device int32 permutation, or "random" for
    a fresh permutation of the positions in every sweep (uniformly at
    random without replacement, Sec. 4.2.1; numpy generator seeded with
    order_seed).
    Returns the history [(phase, sweep, Phi, rel_change)].  The only host
    synchronisation is the read-back of the 4 statistics per sweep.
    """
    n = probe.shape[-1]
    params = params or PieParams(batch=len(pos), norm=1)
    full_params = full_params or params
    history = []
    rng = np.random.default_rng(order_seed)
    raise_nonfinite = True
    for phase, (mm, iters, tol, prm) in enumerate(((m, iters_pft, tol_pft, params),
                                                    (n, iters_full, tol_full, full_params))):
        scan = Scan(pos, obj.shape, n, mm, precision=precision, device=obj.device,
                    method=full_method if phase == 1 else "auto")
        amp = crop_amplitudes(intensity, mm)
        stats = torch.zeros(4, dtype=torch.float64, device=obj.device)
        for it in range(iters):
            ordr = order
            if isinstance(order, str):
                if order != "random":
                    raise ValueError("order must be None, a permutation tensor or 'random'")
                ordr = torch.from_numpy(rng.permutation(len(pos)).astype(np.int32)).to(obj.device)
            pie_sweep(obj, probe, scan, amp, prm, order=ordr, stats=stats)
            st = stats.cpu().numpy()
            if raise_nonfinite and st[3] > 0:
                raise FloatingPointError(f"phase {phase} sweep {it}: {int(st[3])} non-finite values")
            rc = rel_change(st)
            history.append((phase, it, float(st[0]), rc))
            if callback is not None:
                callback(phase, it, obj, probe, st)
            if rc < tol:
                break
        scan.close()
    return history
