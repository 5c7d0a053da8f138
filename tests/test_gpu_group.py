"""GPU parity of the uneven batch (one persistent launch over descriptors of
different sizes, replayed as a hipGraph) against the FP64 oracle, and of the
plan autotuner (it changes launch choices, never results)."""

import numpy as np
import pytest
import torch

import workloads
from oracle import pft as opft

pytestmark = pytest.mark.gpu

TOLS = {"fp32": 1e-5, "split_bf16": 1e-4, "split_fp16": 1e-5}


@pytest.fixture(scope="module")
def pk():
    import paper_2408_03532_amd as p
    p.lib()
    return p


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def mixed_descs(sizes, seed=0, pad=0):
    rng = np.random.default_rng(seed)
    order = rng.permutation(len(sizes))
    d, io, oo = [], 0, 0
    for k in order:
        n, m = sizes[k]
        d.append((n, m, io, oo))
        io += n * n + pad
        oo += m * m + pad
    return np.array(d, dtype=np.int64), io, oo


SMALL = [(16, 4)] * 5 + [(40, 10)] * 4 + [(64, 16)] * 6 + [(128, 32)] * 3 + [(48, 48)] * 2 + [(256, 64)] * 2


@pytest.mark.parametrize("prec", sorted(TOLS))
def test_small_mixed_forward_and_adjoint(pk, prec):
    d, tin, tout = mixed_descs(SMALL, pad=2)
    x = workloads.grouped_inputs(d, tin, seed=7)
    g = pk.Group(d, tin, tout, prec)
    y = g.run(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = opft.grouped_forward(d, x, tout)
    for n, m, io, oo in d:
        assert rel(y[oo:oo + m * m], ref[oo:oo + m * m]) <= TOLS[prec] * 3
    assert rel(y, ref) <= TOLS[prec]
    da = workloads.adjoint_descs(d)
    ya = workloads.grouped_inputs(da, tout, seed=8, adjoint=True)
    ga = pk.Group(da, tout, tin, prec, adjoint=True)
    xa = ga.run(torch.from_numpy(ya).cuda()).cpu().numpy()
    refa = opft.grouped_adjoint(da, ya, tin)
    assert rel(xa, refa) <= TOLS[prec]


def test_graph_replay_with_new_buffers_and_the_per_call_form(pk):
    """The group's graph replayed on alternating buffers (its kernel node is
    updated, never rebuilt), with the program's own work and
    synchronisations between replays; every replay equals the per-call
    grouped transform (same kernel, no graph) bit for bit."""
    d, tin, tout = mixed_descs(SMALL, seed=3)
    x1 = workloads.grouped_inputs(d, tin, seed=1)
    x2 = workloads.grouped_inputs(d, tin, seed=2)
    g = pk.Group(d, tin, tout)
    a = torch.from_numpy(x1).cuda()
    b = torch.from_numpy(x2).cuda()
    outs = []
    for k in range(6):
        outs.append(g.run(a if k % 2 == 0 else b))
        (a * 2).sum().item()          # eager work and a host sync between replays
    torch.cuda.synchronize()
    r1 = opft.grouped_forward(d, x1, tout)
    r2 = opft.grouped_forward(d, x2, tout)
    assert rel(outs[0].cpu().numpy(), r1) <= 1e-5
    assert rel(outs[1].cpu().numpy(), r2) <= 1e-5
    for k in range(2, 6):
        assert torch.equal(outs[k], outs[k % 2])
    direct = torch.zeros(tout, dtype=torch.complex64, device="cuda")
    pk.pft2d_grouped(d, a, direct)
    assert torch.equal(direct, outs[0])


@pytest.mark.parametrize("prec", sorted(TOLS))
def test_per_call_grouped_forward_and_adjoint(pk, prec):
    """pft2d_forward_grouped / pft2d_adjoint_grouped over host descriptors
    and a caller workspace, against the oracle; a second call with fewer
    descriptors reuses the workspace."""
    print("grouped per call", prec, flush=True)
    d, tin, tout = mixed_descs(SMALL, seed=5, pad=2)
    x = workloads.grouped_inputs(d, tin, seed=17)
    ws = torch.empty(pk.grouped_workspace_bytes(d), dtype=torch.uint8, device="cuda")
    y = torch.zeros(tout, dtype=torch.complex64, device="cuda")
    pk.pft2d_grouped(d, torch.from_numpy(x).cuda(), y, prec, workspace=ws)
    assert rel(y.cpu().numpy(), opft.grouped_forward(d, x, tout)) <= TOLS[prec]
    sub = d[:7]
    y2 = torch.zeros(tout, dtype=torch.complex64, device="cuda")
    pk.pft2d_grouped(sub, torch.from_numpy(x).cuda(), y2, prec, workspace=ws)
    ref2 = opft.grouped_forward(sub, x, tout)
    assert rel(y2.cpu().numpy(), ref2) <= TOLS[prec]
    da = workloads.adjoint_descs(d)
    ya = workloads.grouped_inputs(da, tout, seed=18, adjoint=True)
    xa = torch.zeros(tin, dtype=torch.complex64, device="cuda")
    pk.pft2d_grouped(da, torch.from_numpy(ya).cuda(), xa, prec, adjoint=True)
    assert rel(xa.cpu().numpy(), opft.grouped_adjoint(da, ya, tin)) <= TOLS[prec]


def test_per_call_grouped_rejects_bad_calls(pk):
    from paper_2408_03532_amd import _lib
    d = np.array([(32, 8, 0, 0), (64, 16, 1024, 64)], dtype=np.int64)
    x = torch.zeros(1024 + 4096, dtype=torch.complex64, device="cuda")
    y = torch.zeros(64 + 256, dtype=torch.complex64, device="cuda")
    pk.pft2d_grouped(d, x, y)                            # creates the plans
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(pk.PftpieError, match="workspace"):
        pk.pft2d_grouped(d, x, y, workspace=small)
    with pytest.raises(pk.PftpieError, match="overlap"):
        pk.pft2d_grouped(np.array([(32, 8, 0, 0), (32, 8, 1024, 32)]), x, y)
    with pytest.raises(pk.PftpieError, match="overlap"):
        pk.pft2d_grouped(d, x, x[8:])
    arr = (_lib.Desc * 1)(_lib.Desc(48, 12, 0, 0))       # no live plan of (48, 12)
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    st = _lib.lib().pft2d_forward_grouped(arr, 1, ctypes_ptr(x), ctypes_ptr(y), 0, ctypes_ptr(ws), 4096, None)
    assert st == 1 and b"no live plan" in _lib.lib().pftpie_last_error()


def ctypes_ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("prec", sorted(TOLS))
def test_uneven_workload_full_size_sampled(pk, prec):
    """8192 descriptors, n in {64, 128, 256, 512} in equal shares, m = n/4;
    8 sampled descriptors per size checked against the oracle."""
    print("group full", prec, flush=True)
    d, tin, tout = workloads.grouped_descs()
    rng = np.random.default_rng(11)
    idx = np.concatenate([rng.choice(np.nonzero(d[:, 0] == s)[0], 8, replace=False) for s in workloads.GROUP_SIZES])
    x = workloads.grouped_inputs(d, tin, idx=idx)        # only sampled blocks non-zero
    xt = torch.from_numpy(x).cuda()
    g = pk.Group(d, tin, tout, prec)
    y = g.run(xt).cpu().numpy()
    for i in idx:
        n, m, io, oo = (int(v) for v in d[i])
        ref = opft.forward(x[io:io + n * n].reshape(n, n), m)
        assert rel(y[oo:oo + m * m].reshape(m, m), ref) <= TOLS[prec] * 3
    others = np.setdiff1d(np.arange(len(d)), idx)[:64]
    for i in others:                                      # zero blocks transform to zero
        n, m, io, oo = (int(v) for v in d[i])
        assert not np.any(y[oo:oo + m * m])


def test_invalid_descriptors(pk):
    d = np.array([(32, 8, 0, 0), (32, 8, 1024, 32)], dtype=np.int64)      # outputs overlap
    with pytest.raises(pk.PftpieError, match="overlap"):
        pk.Group(d, 2048, 128)
    with pytest.raises(pk.PftpieError, match="outside"):
        pk.Group(np.array([(32, 8, 1500, 0)]), 2048, 64)
    g = pk.Group(np.array([(32, 8, 0, 0)]), 1024, 64)
    with pytest.raises(ValueError):
        g.run(torch.zeros(10, dtype=torch.complex64, device="cuda"))


def test_autotuner_keeps_results(pk, tmp_path, monkeypatch):
    monkeypatch.setenv("PFTPIE_TUNE_CACHE", str(tmp_path / "tune.txt"))
    plan = pk.Plan(128, 32)
    x = torch.from_numpy(workloads.pft_patches(128, range(8))).cuda()
    before = plan.forward(x).cpu().numpy()
    ms = pk.autotune(plan, 64)
    assert ms > 0
    after = plan.forward(x).cpu().numpy()
    assert rel(after, before) <= 1e-6
    assert (tmp_path / "tune.txt").read_text().count("\n") == 1
    plan2 = pk.Plan(128, 32)
    assert pk.autotune(plan2, 64) == pytest.approx(ms)   # read back from the cache


@pytest.mark.parametrize("prec", sorted(TOLS))
@pytest.mark.parametrize("adjoint", [False, True])
def test_group_autotuner_keeps_results(pk, prec, adjoint):
    """The group's own autotuner (per-class column tiles per wave or per
    item, workgroups per compute unit, timed on random inputs of the real
    descriptor mix) changes launch choices only: the tuned group matches
    the untuned one and the oracle to the precision's tolerance."""
    print("group autotune", prec, adjoint, flush=True)
    d, tin, tout = mixed_descs(SMALL + [(512, 128)] * 2, seed=13)
    if adjoint:
        d, tin, tout = workloads.adjoint_descs(d), tout, tin
    x = workloads.grouped_inputs(d, tin, seed=19, adjoint=adjoint)
    g = pk.Group(d, tin, tout, prec, adjoint=adjoint)
    xt = torch.from_numpy(x).cuda()
    before = g.run(xt).cpu().numpy()
    ms = g.autotune()
    assert ms > 0
    after = g.run(xt).cpu().numpy()
    # another tile split changes the float summation order (and in FP32 may
    # switch between the three- and four-product forms): within tolerance
    assert rel(after, before) <= TOLS[prec]
    ref = opft.grouped_adjoint(d, x, tout) if adjoint else opft.grouped_forward(d, x, tout)
    assert rel(after, ref) <= TOLS[prec]
