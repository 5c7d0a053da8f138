"""pie_sweep_noalloc (the sweep on the library's fixed device scratch, for
callers that cannot allocate) against pie_sweep with a caller workspace,
through the C ABI: the same kernels run, so the results agree to the
sweep's FP32 one-sweep bound (1e-5 relative over the object, and for Phi);
two calls in a row, the second on a smaller problem, and the size limit."""

import ctypes

import numpy as np
import pytest
import torch

import workloads
from paper_2408_03532_amd import _lib

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def pk():
    import paper_2408_03532_amd as p
    p.lib()
    return p


def call_noalloc(scan, O, P, A, prm, order=None):
    stats = torch.zeros(4, dtype=torch.float64, device="cuda")
    cp = prm.c()
    st = _lib.lib().pie_sweep_noalloc(scan.handle, ctypes.c_void_p(O.data_ptr()), ctypes.c_void_p(P.data_ptr()),
                                      ctypes.c_void_p(A.data_ptr()),
                                      ctypes.c_void_p(order.data_ptr() if order is not None else 0),
                                      ctypes.byref(cp), ctypes.c_void_p(stats.data_ptr()),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, stats


def pair(pk, case, m, params, order=None, precision="fp32"):
    """(object, stats) after one sweep from the same state: pie_sweep with a
    caller workspace, then pie_sweep_noalloc."""
    n = case["probe"].shape[0]
    scan = pk.Scan(case["pos"], case["init"].shape, n, m, precision=precision)
    A = pk.crop_amplitudes(torch.from_numpy(case["intensity"]).cuda(), m)
    prm = pk.PieParams(**params)
    ordt = None if order is None else torch.from_numpy(np.asarray(order, dtype=np.int32)).cuda()
    O1 = torch.from_numpy(case["init"]).cuda()
    P1 = torch.from_numpy(case["probe"]).cuda()
    s1 = pk.pie_sweep(O1, P1, scan, A, prm, order=ordt)
    O2 = torch.from_numpy(case["init"]).cuda()
    P2 = torch.from_numpy(case["probe"]).cuda()
    rc, s2 = call_noalloc(scan, O2, P2, A, prm, ordt)
    torch.cuda.synchronize()
    assert rc == 0, _lib.lib().pftpie_last_error()
    return (O1.cpu().numpy(), s1.cpu().numpy(), P1.cpu().numpy()), (O2.cpu().numpy(), s2.cpu().numpy(),
                                                                   P2.cpu().numpy())


def test_noalloc_sweep_matches_workspace_sweep_twice(pk):
    # first call: the at-scale phase-1 sweep (900 positions, 128^2 probe,
    # m = 32, fully batched, overlap-normalised, ~150 MB of scratch)
    print("noalloc at scale", flush=True)
    big = workloads.pie_at_scale()
    (Oa, sa, _), (Ob, sb, _) = pair(pk, big, 32, dict(batch=900, norm=1, beta=1.0, alpha=1e-3))
    assert rel(Ob, Oa) <= 1e-5
    assert abs(sb[0] - sa[0]) <= 1e-5 * sa[0] and abs(sb[1] - sa[1]) <= 1e-5 * sa[1]
    # second call, smaller: the tiny workload, sequential plain steps with a
    # probe step and a permuted order (a different scratch layout; the
    # previous call's contents are still there)
    print("noalloc tiny", flush=True)
    tiny = workloads.tiny_pie()
    order = np.random.default_rng(3).permutation(64)
    (Oa, sa, Pa), (Ob, sb, Pb) = pair(pk, tiny, 16, dict(batch=1, norm=0, beta=1.0, gamma=0.3), order=order)
    assert rel(Ob, Oa) <= 1e-5 and rel(Pb, Pa) <= 1e-5
    assert abs(sb[0] - sa[0]) <= 1e-5 * sa[0]
    # and a batched chunked sweep of the tiny workload
    (Oa, sa, _), (Ob, sb, _) = pair(pk, tiny, 16, dict(batch=9, norm=1, beta=1.0, alpha=1e-3))
    assert rel(Ob, Oa) <= 1e-5 and abs(sb[0] - sa[0]) <= 1e-5 * sa[0]


def test_noalloc_rejects_sweeps_beyond_its_scratch(pk):
    # full-resolution phase at 900 positions (m = n = 128) needs about
    # 240 MB: rejected with a message, nothing touched
    big = workloads.pie_at_scale()
    scan = pk.Scan(big["pos"], (1024, 1024), 128, 128)
    O = torch.zeros(1024, 1024, dtype=torch.complex64, device="cuda")
    P = torch.zeros(128, 128, dtype=torch.complex64, device="cuda")
    A = torch.zeros(900, 128, 128, dtype=torch.float32, device="cuda")
    rc, _ = call_noalloc(scan, O, P, A, pk.PieParams(batch=900, norm=1))
    assert rc == 1
    assert b"fixed scratch" in _lib.lib().pftpie_last_error()
    assert scan.workspace_bytes(pk.PieParams(batch=900, norm=1)) > 160 << 20
