"""GPU parity of the ePIE probe step of eq. (6) as printed (the probe moves
at the updated object, with the exit wave and projection formed again)
against the FP64 oracle, for the dense contraction (m < n) and the
full-window fast transform (m = n), in random orders without replacement,
and on the blind circular-window geometry of Sec. 4.2.

Tolerances: relative L2 <= 1e-5 for object and probe after one sweep from a
common state (FP32), Phi <= 1e-5 relative.
"""

import numpy as np
import pytest
import torch

import workloads
from oracle import pie as opie

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def pk():
    import paper_2408_03532_amd as p
    p.lib()
    return p


@pytest.fixture(scope="module")
def tiny():
    return workloads.tiny_pie()


@pytest.fixture(scope="module")
def blind():
    return workloads.blind_circular()


def amps(pk, intensity, m):
    """Each side crops the data itself (Algorithm 3): the library's crop
    kernel on the device, the oracle's crop in float64 on the host."""
    return pk.crop_amplitudes(torch.from_numpy(intensity).cuda(), m), opie.amplitudes(intensity, m)


def run(pk, case, init, probe0, amp, m, prm, order):
    n = probe0.shape[0]
    scan = pk.Scan(case["pos"], init.shape, n, m)
    O = torch.from_numpy(init.astype(np.complex64)).cuda()
    P = torch.from_numpy(probe0.astype(np.complex64)).cuda()
    ordt = torch.from_numpy(np.asarray(order, dtype=np.int32)).cuda()
    st = pk.pie_sweep(O, P, scan, amp, prm, order=ordt)
    return O.cpu().numpy(), P.cpu().numpy(), st.cpu().numpy(), scan.plan.method


@pytest.mark.parametrize("m", [16, 32])
@pytest.mark.parametrize("beta,gamma", [(1.0, 0.5), (0.6, 1.0)])
def test_literal_probe_step_matches_oracle(pk, tiny, m, beta, gamma):
    print("literal epie", m, beta, gamma, flush=True)
    n = tiny["probe"].shape[0]
    A, amp = amps(pk, tiny["intensity"], m)
    P0 = tiny["probe"] * (1.0 + 0.05j)
    order = np.random.default_rng(11).permutation(len(tiny["pos"]))
    prm = dict(batch=1, norm=0, beta=beta, gamma=gamma)
    O, P, st, method = run(pk, tiny, tiny["init"], P0, A, m,
                           pk.PieParams(probe_update="literal", **prm), order)
    assert method == ("fft" if m == n else "dense")
    Or, Pr, sr = opie.pie_sweep(tiny["init"], P0, tiny["pos"], amp, m, order=order,
                                probe_update="literal", **prm)
    assert rel(O, Or) <= 1e-5
    assert rel(P, Pr) <= 1e-5
    assert abs(st[0] - sr[0]) <= 1e-5 * sr[0]
    # the printed form and the simultaneous form are different iterations
    _, Ps, _ = opie.pie_sweep(tiny["init"], P0, tiny["pos"], amp, m, order=order, **prm)
    assert rel(P, Ps) > 1e-4


def test_literal_probe_step_needs_sequential_plain_steps(pk, tiny):
    n = tiny["probe"].shape[0]
    scan = pk.Scan(tiny["pos"], tiny["init"].shape, n, 16)
    O = torch.from_numpy(tiny["init"]).cuda()
    P = torch.from_numpy(tiny["probe"]).cuda()
    A, _ = amps(pk, tiny["intensity"], 16)
    for bad in (dict(batch=4), dict(norm=1)):
        prm = pk.PieParams(gamma=0.5, probe_update="literal", **bad)
        with pytest.raises(pk.PftpieError):
            pk.pie_sweep(O, P, scan, A, prm)


@pytest.mark.parametrize("m", [32, 128])
def test_blind_circular_sweep_matches_oracle(pk, blind, m):
    # one blind ePIE sweep (flat circular probe of radius 58 in 128^2
    # windows, 16 positions, random order) from the initial object and the
    # smaller initial circle, partial (m = 32) and full window (m = 128)
    print("blind circular sweep", m, flush=True)
    A, amp = amps(pk, blind["intensity"], m)
    order = np.random.default_rng(12).permutation(len(blind["pos"]))
    prm = dict(batch=1, norm=0, beta=1.0, gamma=0.5)
    O, P, st, _ = run(pk, blind, blind["init"], blind["probe_init"], A, m,
                      pk.PieParams(probe_update="literal", **prm), order)
    Or, Pr, sr = opie.pie_sweep(blind["init"], blind["probe_init"], blind["pos"], amp, m, order=order,
                                probe_update="literal", **prm)
    assert rel(O, Or) <= 1e-5
    assert rel(P, Pr) <= 1e-5
    assert abs(st[0] - sr[0]) <= 1e-5 * sr[0]


def test_blind_hybrid_random_order_reduces_the_objective(pk, blind):
    # Algorithm 3 on the blind geometry: PFT sweeps at m = 32 then
    # full-window sweeps, a fresh random order each sweep, literal probe
    # steps (the unnormalised steps of eqs. (5)-(6) are kept small, as the
    # paper advises: beta = 0.5, gamma = 0.1; beta = gamma = 1 diverges on
    # this geometry in the oracle as well); the objective of the last
    # full-window sweep is below half the first
    print("blind hybrid", flush=True)
    O = torch.from_numpy(blind["init"]).cuda()
    P = torch.from_numpy(blind["probe_init"]).cuda()
    I = torch.from_numpy(blind["intensity"]).cuda()
    prm = pk.PieParams(batch=1, norm=0, beta=0.5, gamma=0.1, probe_update="literal")
    hist = pk.hybrid_pie(O, P, blind["pos"], I, 32, iters_pft=10, tol_pft=0.0, iters_full=20, tol_full=0.0,
                         params=prm, order="random", order_seed=3)
    full = [h for h in hist if h[0] == 1]
    assert len([h for h in hist if h[0] == 0]) == 10 and len(full) == 20
    assert full[-1][2] < 0.5 * full[0][2]
    assert np.isfinite(O.cpu().numpy()).all() and np.isfinite(P.cpu().numpy()).all()
