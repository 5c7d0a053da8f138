"""Amplitude loss L = sum_j || |F_m (P * O_j) F_m^T| - a_j ||^2 with its
hand-written backward as a torch.autograd.Function.

Both directions run in the HIP library (amp_loss_forward /
amp_loss_backward).  The forward keeps the m x m spectra u_j (1/16 of the
exit waves at n = 4m) for the backward, or, with store_u=False, the backward
recomputes them; the exit waves themselves are never stored.
"""

import ctypes

import torch

from . import _lib
from .pft import _require, _stream_ptr


def _loss_workspace(scan):
    ws = scan._ws.get("loss")
    nb = ctypes.c_size_t()
    _lib.call("amp_loss_workspace_size", scan.handle, ctypes.byref(nb))
    if ws is None or ws.numel() < nb.value:
        ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=scan.plan.device)
        scan._ws["loss"] = ws
    return ws


def _check(obj, probe, scan, amp):
    _require(obj, "obj")
    _require(probe, "probe")
    _require(amp, "amp", torch.float32)
    if tuple(obj.shape) != (scan.H, scan.W) or tuple(probe.shape) != (scan.n, scan.n):
        raise ValueError("object / probe shapes do not match the scan")
    if tuple(amp.shape) != (scan.J, scan.m, scan.m):
        raise ValueError("amp must be [J][m][m]")


def amp_loss(obj, probe, scan, amp, saved_u=None):
    """Loss value as a device float64 0-d tensor (no autograd)."""
    _check(obj, probe, scan, amp)
    loss = torch.zeros(1, dtype=torch.float64, device=obj.device)
    ws = _loss_workspace(scan)
    _lib.call("amp_loss_forward", scan.handle, ctypes.c_void_p(obj.data_ptr()), ctypes.c_void_p(probe.data_ptr()),
              ctypes.c_void_p(amp.data_ptr()), ctypes.c_void_p(loss.data_ptr()),
              ctypes.c_void_p(saved_u.data_ptr() if saved_u is not None else 0),
              ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(obj))
    return loss[0]


def amp_loss_grad(obj, probe, scan, amp, saved_u=None, scale=None, want_probe=True):
    """(dL/dO, dL/dP) scaled by the device scalar ``scale`` (default 1)."""
    _check(obj, probe, scan, amp)
    gO = torch.empty_like(obj)
    gP = torch.empty_like(probe) if want_probe else None
    ws = _loss_workspace(scan)
    sc = None
    if scale is not None:
        sc = scale.to(device=obj.device, dtype=torch.float64).reshape(1).contiguous()
    _lib.call("amp_loss_backward", scan.handle, ctypes.c_void_p(obj.data_ptr()),
              ctypes.c_void_p(probe.data_ptr()), ctypes.c_void_p(amp.data_ptr()),
              ctypes.c_void_p(saved_u.data_ptr() if saved_u is not None else 0),
              ctypes.c_void_p(sc.data_ptr() if sc is not None else 0),
              ctypes.c_void_p(gO.data_ptr()), ctypes.c_void_p(gP.data_ptr() if gP is not None else 0),
              ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(obj))
    return gO, gP


class AmplitudeLoss(torch.autograd.Function):
    """L(O, P); backward gives grad = dL/dRe + i dL/dIm for O and P."""

    @staticmethod
    def forward(ctx, obj, probe, scan, amp, store_u=True):
        u = None
        if store_u:
            u = torch.empty(scan.J, scan.m, scan.m, dtype=torch.complex64, device=obj.device)
        loss = amp_loss(obj, probe, scan, amp, saved_u=u)
        ctx.scan = scan
        ctx.save_for_backward(obj, probe, amp, u if u is not None else torch.empty(0, device=obj.device))
        ctx.store_u = store_u
        return loss

    @staticmethod
    def backward(ctx, g):
        obj, probe, amp, u = ctx.saved_tensors
        gO, gP = amp_loss_grad(obj, probe, ctx.scan, amp, saved_u=u if ctx.store_u else None, scale=g,
                               want_probe=ctx.needs_input_grad[1])
        return (gO if ctx.needs_input_grad[0] else None), gP, None, None, None


def amplitude_loss(obj, probe, scan, amp, store_u=True):
    return AmplitudeLoss.apply(obj, probe, scan, amp, store_u)
