"""Python binding of the partial transform: plans, forward / adjoint calls on
torch tensors, and the autograd operator.

The partial transform keeps the centred m x m window of the 2-D DFT of each
n x n patch (Appendix A; Fig. 2 of the paper): y = F_m psi F_m^T with
F_m[c, k] = exp(-2 pi i (c - floor(m/2)) k / n).  The adjoint is
F_m^H y conj(F_m) without normalisation.
"""

import ctypes
import threading

import torch

from . import _lib

_plans = {}
_plans_lock = threading.Lock()


def _stream_ptr(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _require(t, name, dtype=torch.complex64):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """Twiddle tables of one (n, m, precision) on one device.

    method: "auto" (the fast full-window transform when m = n in
    {16, 32, 64, 128}, else the dense contraction), "dense" or "fft"; the
    resolved choice is in ``self.method``.  period: DFT length of a masked
    larger field (default n; see pftpie_plan_create_period)."""

    def __init__(self, n, m, precision="fp32", device=None, method="auto", period=None):
        if precision not in _lib.PRECISION:
            raise ValueError(f"precision must be one of {sorted(_lib.PRECISION)}")
        if method not in _lib.METHOD:
            raise ValueError(f"method must be one of {sorted(_lib.METHOD)}")
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else
                           torch.device(device).index or 0)
        self.n, self.m, self.precision, self.device = int(n), int(m), precision, dev
        self.period = int(n) if period is None else int(period)
        h = _lib.c_plan()
        with torch.cuda.device(dev):
            _lib.call("pftpie_plan_create_period", n, m, self.period, _lib.PRECISION[precision],
                      _lib.METHOD[method], ctypes.byref(h))
        self.handle = h
        resolved = ctypes.c_int32()
        _lib.call("pftpie_plan_method", self.handle, ctypes.byref(resolved))
        self.method = {v: k for k, v in _lib.METHOD.items()}[resolved.value]

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.lib().pftpie_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, psi, out=None):
        """psi: complex64 [..., n, n] on this plan's device -> [..., m, m]."""
        _require(psi, "psi")
        if psi.shape[-2:] != (self.n, self.n):
            raise ValueError(f"psi must end in ({self.n}, {self.n}), got {tuple(psi.shape)}")
        lead = psi.shape[:-2]
        if out is None:
            out = torch.empty(lead + (self.m, self.m), dtype=torch.complex64, device=psi.device)
        _require(out, "out")
        if out.shape != lead + (self.m, self.m):
            raise ValueError("out has the wrong shape")
        batch = psi.numel() // (self.n * self.n)
        _lib.call("pft2d_forward", self.handle, ctypes.c_void_p(psi.data_ptr()),
                  ctypes.c_void_p(out.data_ptr()), batch, _stream_ptr(psi))
        return out

    def adjoint(self, y, out=None):
        """y: complex64 [..., m, m] -> F_m^H y conj(F_m), [..., n, n]."""
        _require(y, "y")
        if y.shape[-2:] != (self.m, self.m):
            raise ValueError(f"y must end in ({self.m}, {self.m}), got {tuple(y.shape)}")
        lead = y.shape[:-2]
        if out is None:
            out = torch.empty(lead + (self.n, self.n), dtype=torch.complex64, device=y.device)
        _require(out, "out")
        if out.shape != lead + (self.n, self.n):
            raise ValueError("out has the wrong shape")
        batch = y.numel() // (self.m * self.m)
        _lib.call("pft2d_adjoint", self.handle, ctypes.c_void_p(y.data_ptr()),
                  ctypes.c_void_p(out.data_ptr()), batch, _stream_ptr(y))
        return out


def get_plan(n, m, precision="fp32", device=None, method="auto", period=None):
    """Cached plan for (device, n, m, precision, method, period)."""
    dev = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    period = int(n) if period is None else int(period)
    key = (dev, int(n), int(m), precision, method, period)
    with _plans_lock:
        p = _plans.get(key)
        if p is None:
            p = Plan(n, m, precision, device=torch.device("cuda", dev), method=method, period=period)
            _plans[key] = p
        return p


def pft2d_forward(psi, m, precision="fp32", out=None, method="auto"):
    """Centred m x m partial DFT of every trailing n x n patch of psi."""
    return get_plan(psi.shape[-1], m, precision, psi.device, method).forward(psi.contiguous(), out)


def pft2d_adjoint(y, n, precision="fp32", out=None, method="auto"):
    """Adjoint F_m^H y conj(F_m) of every trailing m x m block of y."""
    return get_plan(n, y.shape[-1], precision, y.device, method).adjoint(y.contiguous(), out)


class _PFT2D(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi, m, precision):
        ctx.n, ctx.precision = psi.shape[-1], precision
        return pft2d_forward(psi, m, precision)

    @staticmethod
    def backward(ctx, gy):
        # y = A psi is complex-linear: the gradient is A^H applied to gy
        return pft2d_adjoint(gy.contiguous(), ctx.n, ctx.precision), None, None


class _PFT2DAdjoint(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, n, precision):
        ctx.m, ctx.precision = y.shape[-1], precision
        return pft2d_adjoint(y, n, precision)

    @staticmethod
    def backward(ctx, gx):
        return pft2d_forward(gx.contiguous(), ctx.m, ctx.precision), None, None


def pft2d(psi, m, precision="fp32"):
    """Differentiable partial transform (backward = adjoint)."""
    return _PFT2D.apply(psi, m, precision)


def pft2d_adj(y, n, precision="fp32"):
    """Differentiable adjoint (backward = forward)."""
    return _PFT2DAdjoint.apply(y, n, precision)


def autotune(plan, sample=256):
    """Time the plan's candidate tile splits on a scratch batch and keep the
    fastest (see pftpie_plan_autotune).  Returns the best forward + adjoint
    milliseconds per call of `sample` patches."""
    ms = ctypes.c_double()
    with torch.cuda.device(plan.device):
        _lib.call("pftpie_plan_autotune", plan.handle, int(sample), ctypes.byref(ms))
    return ms.value


class Group:
    """An uneven batch: descriptors (n, m, in_offset, out_offset) over packed
    complex64 arrays, run as one persistent launch (replayed as a hipGraph).

    descs: int array [count][4]; offsets in complex elements.  For the
    forward, input blocks hold n*n and output blocks m*m elements; with
    adjoint=True the reverse.  All descriptors' (n, m) pairs get a plan of
    the given precision."""

    def __init__(self, descs, in_len, out_len, precision="fp32", adjoint=False, device=None):
        import numpy as np
        d = np.asarray(descs, dtype=np.int64).reshape(-1, 4)
        self.count, self.in_len, self.out_len = len(d), int(in_len), int(out_len)
        self.adjoint, self.precision = bool(adjoint), precision
        pairs = sorted({(int(n), int(m)) for n, m in d[:, :2]}) if len(d) else []
        self.plans = [get_plan(n, m, precision, device) for n, m in pairs]
        self.device = self.plans[0].device if self.plans else torch.device("cuda", torch.cuda.current_device())
        arr = (_lib.c_plan * max(1, len(self.plans)))(*[p.handle for p in self.plans])
        darr = (_lib.Desc * max(1, self.count))()
        for i, (n, m, io, oo) in enumerate(d):
            darr[i] = _lib.Desc(int(n), int(m), int(io), int(oo))
        h = _lib.c_group()
        with torch.cuda.device(self.device):
            _lib.call("pftpie_group_create", arr, len(self.plans), darr, self.count, self.in_len, self.out_len,
                      int(self.adjoint), ctypes.byref(h))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.lib().pftpie_group_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune(self):
        """Tune the group's launch choices on its descriptor mix (random
        inputs); returns the best batch time in milliseconds."""
        ms = ctypes.c_double()
        with torch.cuda.device(self.device):
            _lib.call("pftpie_group_autotune", self.handle, ctypes.byref(ms))
        return ms.value

    def run(self, inp, out=None):
        _require(inp, "inp")
        if inp.numel() != self.in_len:
            raise ValueError(f"inp must hold {self.in_len} complex elements")
        if out is None:
            out = torch.zeros(self.out_len, dtype=torch.complex64, device=inp.device)
        _require(out, "out")
        if out.numel() != self.out_len:
            raise ValueError(f"out must hold {self.out_len} complex elements")
        _lib.call("pft2d_group_run", self.handle, ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                  _stream_ptr(inp))
        return out


def _descs(descs):
    import numpy as np
    d = np.asarray(descs, dtype=np.int64).reshape(-1, 4)
    arr = (_lib.Desc * max(1, len(d)))()
    for i, (n, m, io, oo) in enumerate(d):
        arr[i] = _lib.Desc(int(n), int(m), int(io), int(oo))
    return d, arr


def grouped_workspace_bytes(descs, adjoint=False):
    d, arr = _descs(descs)
    nb = ctypes.c_size_t()
    _lib.call("pft2d_grouped_workspace_size", arr, len(d), int(bool(adjoint)), ctypes.byref(nb))
    return nb.value


def pft2d_grouped(descs, inp, out, precision="fp32", adjoint=False, workspace=None):
    """Per-call uneven batch (pft2d_forward_grouped / pft2d_adjoint_grouped):
    descriptors (n, m, in_offset, out_offset) over packed complex64 arrays;
    the plans of every (n, m) are created (and cached) first, since the call
    takes the twiddle tables of live plans.  Returns out."""
    d, arr = _descs(descs)
    _require(inp, "inp")
    _require(out, "out")
    for n, m in sorted({(int(a), int(b)) for a, b in d[:, :2]}):
        get_plan(n, m, precision, inp.device)
    need = grouped_workspace_bytes(d, adjoint)
    ws = workspace if workspace is not None else torch.empty(need, dtype=torch.uint8, device=inp.device)
    name = "pft2d_adjoint_grouped" if adjoint else "pft2d_forward_grouped"
    with torch.cuda.device(inp.device):
        _lib.call(name, arr, len(d), ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                  _lib.PRECISION[precision], ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(inp))
    return out


class PolyPlan:
    """The paper's polynomial partial Fourier transform (Sec. 3.1,
    Algorithms 1-2; Appendix A, Algorithms 4-5) for n x n patches, crop m,
    divisor p and tolerance eps, beside the exact transform for comparison.
    ``r`` and ``xi`` are the chosen number of polynomial terms and scope."""

    def __init__(self, n, m, p, eps, device=None):
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else
                           torch.device(device).index or 0)
        self.n, self.m, self.p, self.eps, self.device = int(n), int(m), int(p), float(eps), dev
        h = _lib.c_plan()
        with torch.cuda.device(dev):
            _lib.call("pftpie_poly_create", self.n, self.m, self.p, self.eps, ctypes.byref(h))
        self.handle = h
        r, xi = ctypes.c_int32(), ctypes.c_double()
        _lib.call("pftpie_poly_info", self.handle, ctypes.byref(r), ctypes.byref(xi))
        self.r, self.xi = r.value, xi.value
        self._ws = None

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.lib().pftpie_poly_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, batch):
        nb = ctypes.c_size_t()
        _lib.call("pftpie_poly_workspace_size", self.handle, int(batch), ctypes.byref(nb))
        if self._ws is None or self._ws.numel() < nb.value:
            self._ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=self.device)
        return self._ws

    def forward(self, psi, out=None):
        """psi: complex64 [..., n, n] -> approximate centred [..., m, m]."""
        _require(psi, "psi")
        if psi.shape[-2:] != (self.n, self.n):
            raise ValueError(f"psi must end in ({self.n}, {self.n})")
        lead = psi.shape[:-2]
        if out is None:
            out = torch.empty(lead + (self.m, self.m), dtype=torch.complex64, device=psi.device)
        _require(out, "out")
        batch = psi.numel() // (self.n * self.n)
        ws = self.workspace(batch)
        _lib.call("pft2d_poly_forward", self.handle, ctypes.c_void_p(psi.data_ptr()),
                  ctypes.c_void_p(out.data_ptr()), batch, ctypes.c_void_p(ws.data_ptr()),
                  ctypes.c_size_t(ws.numel()), _stream_ptr(psi))
        return out

