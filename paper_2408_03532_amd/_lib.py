"""ctypes loader of libpftpie.so (the C ABI declared in include/pftpie.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Importing works without a GPU (the library links the HIP runtime,
which loads without a device); a missing library raises at first use.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpftpie.so")

c_plan = ctypes.c_void_p
c_scan = ctypes.c_void_p
c_group = ctypes.c_void_p
vp = ctypes.c_void_p
i32 = ctypes.c_int32
i64 = ctypes.c_int64
f32 = ctypes.c_float
sz = ctypes.c_size_t

STATUS = {0: "PFTPIE_OK", 1: "PFTPIE_E_INVALID", 2: "PFTPIE_E_UNSUPPORTED",
          3: "PFTPIE_E_NOMEM", 4: "PFTPIE_E_DEVICE"}
PRECISION = {"fp32": 0, "split_bf16": 1, "split_fp16": 2}
METHOD = {"auto": 0, "dense": 1, "fft": 2}


class PieParams(ctypes.Structure):
    _fields_ = [("batch", i32), ("norm", i32), ("beta", f32), ("gamma", f32), ("alpha", f32),
                ("probe_update", i32)]


class Desc(ctypes.Structure):
    _fields_ = [("n", i32), ("m", i32), ("in_offset", i64), ("out_offset", i64)]


# name -> (restype, argtypes); every symbol include/pftpie.h declares
SIGNATURES = {
    "pftpie_status_string": (ctypes.c_char_p, [i32]),
    "pftpie_last_error": (ctypes.c_char_p, []),
    "pftpie_plan_create": (i32, [i32, i32, i32, ctypes.POINTER(c_plan)]),
    "pftpie_plan_create_method": (i32, [i32, i32, i32, i32, ctypes.POINTER(c_plan)]),
    "pftpie_plan_method": (i32, [c_plan, ctypes.POINTER(i32)]),
    "pftpie_plan_create_period": (i32, [i32, i32, i32, i32, i32, ctypes.POINTER(c_plan)]),
    "pftpie_plan_period": (i32, [c_plan, ctypes.POINTER(i32)]),
    "pftpie_poly_create": (i32, [i32, i32, i32, ctypes.c_double, ctypes.POINTER(c_plan)]),
    "pftpie_poly_destroy": (i32, [c_plan]),
    "pftpie_poly_info": (i32, [c_plan, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]),
    "pftpie_poly_workspace_size": (i32, [c_plan, i64, ctypes.POINTER(ctypes.c_size_t)]),
    "pft2d_poly_forward": (i32, [c_plan, vp, vp, i64, vp, ctypes.c_size_t, vp]),
    "pftpie_plan_destroy": (i32, [c_plan]),
    "pftpie_plan_info": (i32, [c_plan, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
    "pftpie_plan_autotune": (i32, [c_plan, i64, ctypes.POINTER(ctypes.c_double)]),
    "pft2d_forward": (i32, [c_plan, vp, vp, i64, vp]),
    "pft2d_adjoint": (i32, [c_plan, vp, vp, i64, vp]),
    "pftpie_group_create": (i32, [ctypes.POINTER(c_plan), i32, ctypes.POINTER(Desc), i64, i64, i64, i32,
                                  ctypes.POINTER(c_group)]),
    "pftpie_group_destroy": (i32, [c_group]),
    "pft2d_group_run": (i32, [c_group, vp, vp, vp]),
    "pftpie_group_autotune": (i32, [c_group, ctypes.POINTER(ctypes.c_double)]),
    "pftpie_measure_mfma_peaks": (i32, [ctypes.POINTER(ctypes.c_double)] * 3),
    "pft2d_grouped_workspace_size": (i32, [ctypes.POINTER(Desc), i64, i32, ctypes.POINTER(sz)]),
    "pft2d_forward_grouped": (i32, [ctypes.POINTER(Desc), i64, vp, vp, i32, vp, sz, vp]),
    "pft2d_adjoint_grouped": (i32, [ctypes.POINTER(Desc), i64, vp, vp, i32, vp, sz, vp]),
    "pie_scan_create": (i32, [c_plan, ctypes.POINTER(i32), i32, i32, i32, ctypes.POINTER(c_scan)]),
    "pie_scan_destroy": (i32, [c_scan]),
    "pie_workspace_size": (i32, [c_scan, ctypes.POINTER(PieParams), ctypes.POINTER(sz)]),
    "pie_sweep": (i32, [c_scan, vp, vp, vp, vp, ctypes.POINTER(PieParams), vp, sz, vp, vp]),
    "pie_sweep_noalloc": (i32, [c_scan, vp, vp, vp, vp, ctypes.POINTER(PieParams), vp, vp]),
    "pie_crop_amplitudes": (i32, [vp, i32, i32, i32, vp, vp]),
    "amp_loss_workspace_size": (i32, [c_scan, ctypes.POINTER(sz)]),
    "amp_loss_forward": (i32, [c_scan, vp, vp, vp, vp, vp, vp, sz, vp]),
    "amp_loss_backward": (i32, [c_scan, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2408_03532_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class PftpieError(RuntimeError):
    def __init__(self, fn, status):
        L = lib()
        detail = L.pftpie_last_error().decode()
        self.status = status
        super().__init__(f"{fn}: {STATUS.get(status, status)}: {detail}")


def check(fn, status):
    if status != 0:
        raise PftpieError(fn, status)


def call(name, *args):
    check(name, getattr(lib(), name)(*args))
