"""The C ABI without a GPU: the library loads, exports every function the
header declares, and rejects invalid arguments on the host before touching
the device."""

import ctypes
import os
import re

import pytest

import paper_2408_03532_amd as pk
from paper_2408_03532_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "pftpie.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^(?:const\s+char\s*\*|pftpie_status)\s+(\w+)\s*\(", txt, flags=re.M)))


def test_every_declared_symbol_is_exported_and_bound():
    names = declared()
    assert len(names) >= 15
    L = pk.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_status_strings():
    L = pk.lib()
    assert L.pftpie_status_string(0) == b"ok"
    assert L.pftpie_status_string(1) == b"invalid argument"
    assert L.pftpie_status_string(99) == b"unknown status"


@pytest.mark.parametrize("n,m,prec,msg", [(0, 1, 0, b"n <= 8192"), (8, 9, 0, b"m <= n"), (8, 0, 0, b"m <= n"),
                                          (9000, 4, 0, b"n <= 8192"), (8, 4, 7, b"unknown precision")])
def test_plan_create_rejects_bad_sizes_before_the_device(n, m, prec, msg):
    L = pk.lib()
    h = ctypes.c_void_p(123)
    assert L.pftpie_plan_create(n, m, prec, ctypes.byref(h)) == 1
    assert h.value is None
    assert msg in L.pftpie_last_error()


def test_plan_create_large_window_is_unsupported():
    L = pk.lib()
    h = ctypes.c_void_p()
    assert L.pftpie_plan_create(512, 256, 0, ctypes.byref(h)) == 2


@pytest.mark.parametrize("n,m,method,status,msg", [
    (32, 32, 7, 1, b"unknown method"),
    (64, 32, 2, 2, b"in {16, 32, 64, 128}"),   # the fast transform needs the full window
    (256, 256, 2, 2, b"m > 128"),                    # windows above 128 are not built
    (48, 48, 2, 2, b"in {16, 32, 64, 128}"),   # not a supported length
])
def test_plan_method_rejected_on_the_host(n, m, method, status, msg):
    L = pk.lib()
    h = ctypes.c_void_p(123)
    assert L.pftpie_plan_create_method(n, m, 0, method, ctypes.byref(h)) == status
    assert h.value is None
    assert msg in L.pftpie_last_error()


@pytest.mark.parametrize("n,m,period,method,status,msg", [
    (32, 16, 31, 0, 1, b"n <= period"),          # the field cannot be smaller than the window
    (32, 16, (1 << 20) + 1, 0, 1, b"period <= 2^20"),
    (32, 32, 64, 2, 2, b"m = n = period"),       # the fast transform is for the window's own period
])
def test_plan_period_rejected_on_the_host(n, m, period, method, status, msg):
    L = pk.lib()
    h = ctypes.c_void_p(123)
    assert L.pftpie_plan_create_period(n, m, period, 0, method, ctypes.byref(h)) == status
    assert h.value is None
    assert msg in L.pftpie_last_error()


def test_plan_method_query_needs_a_plan():
    L = pk.lib()
    out = ctypes.c_int32(-1)
    assert L.pftpie_plan_method(None, ctypes.byref(out)) == 1
    assert out.value == -1


def test_null_handles_are_invalid_not_fatal():
    L = pk.lib()
    assert L.pft2d_forward(None, None, None, 1, None) == 1
    assert L.pft2d_adjoint(None, None, None, 1, None) == 1
    assert L.pftpie_plan_destroy(None) == 0
    assert L.pftpie_plan_create(8, 4, 0, None) == 1


def test_python_layer_reports_missing_device_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(Exception):
        pk.Plan(32, 16)


@pytest.mark.parametrize("n,m,p,eps,status,msg", [
    (256, 128, 48, 1e-7, 2, b"p must be 16, 32, 64 or 128"),
    (250, 64, 64, 1e-7, 1, b"p must divide n"),
    (2048, 64, 32, 1e-7, 2, b"n / p above 32"),
    (256, 128, 64, 0.0, 1, b"0 < eps < 1"),
    (256, 128, 16, 1e-12, 2, b"no r <= 25"),   # m/2 / p = 4 needs more terms than 25
])
def test_poly_create_rejected_on_the_host(n, m, p, eps, status, msg):
    L = pk.lib()
    h = ctypes.c_void_p(123)
    assert L.pftpie_poly_create(n, m, p, eps, ctypes.byref(h)) == status
    assert h.value is None
    assert msg in L.pftpie_last_error()


def test_grouped_calls_reject_bad_arguments_on_the_host():
    L = pk.lib()
    d = (_lib.Desc * 2)(_lib.Desc(32, 8, 0, 0), _lib.Desc(64, 16, 1024, 64))
    nb = ctypes.c_size_t(0)
    assert L.pft2d_grouped_workspace_size(d, 2, 0, ctypes.byref(nb)) == 0
    assert nb.value >= 256 + (2 + 1) * 24
    assert L.pft2d_grouped_workspace_size(d, 2, 1, ctypes.byref(nb)) == 0
    assert L.pft2d_grouped_workspace_size(d, 2, 0, None) == 1
    assert L.pft2d_grouped_workspace_size(None, 2, 0, ctypes.byref(nb)) == 1
    bad = (_lib.Desc * 1)(_lib.Desc(8, 9, 0, 0))
    assert L.pft2d_grouped_workspace_size(bad, 1, 0, ctypes.byref(nb)) == 1
    p = ctypes.c_void_p(1 << 20)
    for args, msg in [((d, -1, p, p, 0, p, 1 << 20, None), b"count < 0"),
                      ((None, 2, p, p, 0, p, 1 << 20, None), b"NULL"),
                      ((d, 2, p, p, 9, p, 1 << 20, None), b"unknown precision"),
                      ((d, 2, None, p, 0, p, 1 << 20, None), b"NULL data pointer"),
                      ((d, 2, ctypes.c_void_p((1 << 20) + 8), p, 0, p, 1 << 20, None), b"16-byte aligned"),
                      ((d, 2, p, p, 0, ctypes.c_void_p((1 << 20) + 64), 1 << 20, None), b"256-byte aligned")]:
        assert L.pft2d_forward_grouped(*args) == 1
        assert msg in L.pftpie_last_error()
    assert L.pft2d_adjoint_grouped(d, 0, None, None, 0, None, 0, None) == 0   # nothing to do
