"""GPU parity of the PIE sweep (pie_sweep through the C ABI) against the FP64
oracle.

Tolerances (relative L2 over the object, FP32 path):
  one sweep from a common state       <= 1e-5
  ten sweeps of the tiny workload     <= 1e-4
  Phi per sweep                       <= 1e-5 (relative)
  noise-free fixed point ||O'-O||/||O|| <= 1e-6
The one-sweep bound follows the transform's own 1e-5 (two partial
transforms per position, each ~1e-6 in practice); the ten-sweep bound allows
the ten-fold accumulation of per-sweep rounding.
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


def amps(pk, intensity, m):
    """Each side crops the data itself (Algorithm 3): the library's crop
    kernel on the device, the oracle's crop in float64 on the host."""
    dev = pk.crop_amplitudes(torch.from_numpy(intensity).cuda(), m)
    return dev, opie.amplitudes(intensity, m)


def run_gpu(pk, case, obj0, probe0, amp, m, params, order=None, sweeps=1, precision="fp32"):
    n = case["probe"].shape[0]
    scan = pk.Scan(case["pos"], obj0.shape, n, m, precision=precision)
    O = torch.from_numpy(obj0.astype(np.complex64)).cuda()
    P = torch.from_numpy(probe0.astype(np.complex64)).cuda()
    A = amp if torch.is_tensor(amp) else torch.from_numpy(amp.astype(np.float32)).cuda()
    ordt = None if order is None else torch.from_numpy(np.asarray(order, dtype=np.int32)).cuda()
    stats = []
    for _ in range(sweeps):
        st = pk.pie_sweep(O, P, scan, A, params, order=ordt)
        stats.append(st.cpu().numpy().copy())
    torch.cuda.synchronize()
    return O.cpu().numpy(), P.cpu().numpy(), stats


MODES = [dict(batch=1, norm=0, beta=1.0, gamma=0.0),
         dict(batch=64, norm=1, beta=1.0, gamma=0.0, alpha=1e-3),
         dict(batch=7, norm=1, beta=0.8, gamma=0.5, alpha=1e-3),
         dict(batch=1, norm=0, beta=0.9, gamma=0.3),
         dict(batch=64, norm=0, beta=0.05, gamma=0.0),
         dict(batch=10, norm=0, beta=0.05, gamma=0.02)]


@pytest.mark.parametrize("mode", MODES, ids=lambda d: "-".join(f"{k}{v}" for k, v in d.items()))
def test_one_sweep_matches_oracle(pk, tiny, mode):
    print("pie one sweep", mode, flush=True)
    m = tiny["m"]
    init = tiny["init"]
    P0 = tiny["probe"] * (1.0 + 0.05j) if mode.get("gamma", 0) else tiny["probe"]
    A, amp = amps(pk, tiny["intensity"], m)
    O, P, st = run_gpu(pk, tiny, init, P0, A, m, pk.PieParams(**mode))
    Or, Pr, sr = opie.pie_sweep(init, P0, tiny["pos"], amp, m, **mode)
    assert rel(O, Or) <= 1e-5
    if mode.get("gamma", 0):
        assert rel(P, Pr) <= 1e-5
    assert abs(st[0][0] - sr[0]) <= 1e-5 * sr[0]
    assert abs(st[0][1] - sr[1]) <= 1e-4 * sr[1]
    assert abs(st[0][2] - sr[2]) <= 1e-6 * sr[2]
    assert st[0][3] == 0


@pytest.mark.parametrize("batch,norm", [(1, 0), (64, 1)])
def test_tiny_workload_ten_sweeps(pk, tiny, batch, norm):
    m = tiny["m"]
    params = dict(batch=batch, norm=norm, beta=1.0, gamma=0.0, alpha=1e-3)
    A, amp = amps(pk, tiny["intensity"], m)
    O, _, st = run_gpu(pk, tiny, tiny["init"], tiny["probe"], A, m, pk.PieParams(**params), sweeps=10)
    Or = tiny["init"]
    phis = []
    for _ in range(10):
        Or, _, s = opie.pie_sweep(Or, tiny["probe"], tiny["pos"], amp, m, **params)
        phis.append(s[0])
    assert rel(O, Or) <= 1e-4
    for a, b in zip(st, phis):
        assert abs(a[0] - b) <= 1e-4 * b


def test_permuted_order_matches_oracle(pk, tiny):
    m = tiny["m"]
    perm = np.random.default_rng(5).permutation(64)
    A, amp = amps(pk, tiny["intensity"], m)
    for params in (dict(batch=1, norm=0, beta=1.0), dict(batch=9, norm=1, beta=1.0, alpha=1e-3)):
        O, _, _ = run_gpu(pk, tiny, tiny["init"], tiny["probe"], A, m, pk.PieParams(**params),
                          order=perm)
        Or, _, _ = opie.pie_sweep(tiny["init"], tiny["probe"], tiny["pos"], amp, m, order=perm, **params)
        assert rel(O, Or) <= 1e-5


@pytest.mark.parametrize("m,batch,norm,gamma", [(16, 1, 0, 0.0), (16, 64, 1, 0.0), (32, 64, 1, 0.5),
                                                (8, 5, 0, 0.2)])
def test_noise_free_fixed_point(pk, tiny, m, batch, norm, gamma):
    A, amp = amps(pk, tiny["intensity"], m)
    O, P, st = run_gpu(pk, tiny, tiny["obj"], tiny["probe"], A, m,
                       pk.PieParams(batch=batch, norm=norm, beta=1.0, gamma=gamma))
    assert rel(O, tiny["obj"]) <= 1e-6
    assert rel(P, tiny["probe"]) <= 1e-6
    assert st[0][0] <= 1e-10 * np.sum(amp.astype(np.float64) ** 2) / (64 * 32 * 32)


def test_crop_amplitudes_kernel(pk, tiny):
    I = torch.from_numpy(tiny["intensity"]).cuda()
    for m in (16, 5, 32):
        got = pk.crop_amplitudes(I, m).cpu().numpy()
        ref = opie.amplitudes(tiny["intensity"], m)
        assert np.max(np.abs(got - ref) / np.maximum(ref, 1e-30)) <= 2e-7


def test_at_scale_one_sweep(pk):
    """Phase-1 shape of the warm-started workload: 1024^2 object, 128^2
    aperture probe, 900 jittered positions, m = 32, fully batched,
    overlap-normalised; one sweep from the random initial guess."""
    case = workloads.pie_at_scale()
    m = case["m"]
    A, amp = amps(pk, case["intensity"], m)
    params = dict(batch=900, norm=1, beta=1.0, gamma=0.0, alpha=1e-3)
    O, _, st = run_gpu(pk, case, case["init"], case["probe"], A, m, pk.PieParams(**params))
    Or, _, sr = opie.pie_sweep(case["init"], case["probe"], case["pos"], amp, m, **params)
    assert rel(O, Or) <= 1e-5
    assert abs(st[0][0] - sr[0]) <= 1e-5 * sr[0]
    # ||dO||^2 and ||O||^2 over the whole object (the scan leaves a border
    # of the object unlit, which the update's statistics must include)
    assert abs(st[0][1] - sr[1]) <= 1e-4 * sr[1]
    assert abs(st[0][2] - sr[2]) <= 1e-6 * sr[2]
    assert st[0][3] == 0


@pytest.mark.parametrize("norm", [0, 1])
def test_single_position_with_larger_batch(pk, tiny, norm):
    # one position and batch > 1: the chunk is that position alone, updated
    # in place; the sweep statistics still cover its change
    m = tiny["m"]
    case = dict(tiny, pos=tiny["pos"][5:6])
    A, amp = amps(pk, tiny["intensity"][5:6], m)
    params = dict(batch=4, norm=norm, beta=1.0, gamma=0.0, alpha=1e-3)
    O, _, st = run_gpu(pk, case, tiny["init"], tiny["probe"], A, m, pk.PieParams(**params))
    Or, _, sr = opie.pie_sweep(tiny["init"], tiny["probe"], case["pos"], amp, m, **params)
    assert rel(O, Or) <= 1e-5
    assert abs(st[0][0] - sr[0]) <= 1e-5 * sr[0]
    assert sr[1] > 0 and abs(st[0][1] - sr[1]) <= 1e-4 * sr[1]
    assert abs(st[0][2] - sr[2]) <= 1e-6 * sr[2]


def test_ragged_window_and_sizes(pk):
    """n = 24 (not a multiple of 16), m = 10, object 61 x 53, positions on
    the object's edges."""
    rng = np.random.default_rng(3)
    H, W, n, m = 61, 53, 24, 10
    obj = (rng.uniform(0.5, 1, (H, W)) * np.exp(1j * rng.uniform(-1, 1, (H, W)))).astype(np.complex64)
    probe = workloads.gaussian_probe(n, 5.0, 0.03)
    pos = np.array([[0, 0], [H - n, W - n], [0, W - n], [H - n, 0], [17, 11], [20, 29]], dtype=np.int32)
    amp = np.abs(rng.standard_normal((len(pos), m, m))).astype(np.float32) * 30
    case = dict(pos=pos, probe=probe)
    for params in (dict(batch=1, norm=0, beta=1.0), dict(batch=6, norm=1, beta=1.0, gamma=0.3, alpha=1e-3)):
        O, P, _ = run_gpu(pk, case, obj, probe, amp, m, pk.PieParams(**params))
        Or, Pr, _ = opie.pie_sweep(obj, probe, pos, amp, m, **params)
        assert rel(O, Or) <= 1e-5 and rel(P, Pr) <= 1e-5


def test_invalid_arguments_are_rejected(pk, tiny):
    n, m = 32, 16
    with pytest.raises(pk.PftpieError, match="outside the object"):
        pk.Scan(np.array([[0, 0], [97, 0]]), (128, 128), n, m)
    scan = pk.Scan(tiny["pos"], (128, 128), n, m)
    O = torch.zeros(128, 128, dtype=torch.complex64, device="cuda")
    P = torch.zeros(32, 32, dtype=torch.complex64, device="cuda")
    A = torch.zeros(64, m, m, dtype=torch.float32, device="cuda")
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(pk.PftpieError, match="workspace"):
        pk.pie_sweep(O, P, scan, A, pk.PieParams(batch=64, norm=1), workspace=small)
    with pytest.raises(pk.PftpieError, match="batch"):
        pk.pie_sweep(O, P, scan, A, pk.PieParams(batch=0))
    with pytest.raises(pk.PftpieError, match="overlap"):
        pk.pie_sweep(O, O.view(-1)[: 32 * 32].view(32, 32), scan, A, pk.PieParams())


@pytest.mark.parametrize("precision,tol", [("split_bf16", 1e-4), ("split_fp16", 1e-5)])
def test_split_precision_sweeps(pk, tiny, precision, tol):
    """One sweep in each split precision against the FP64 oracle."""
    m = tiny["m"]
    for mode in (dict(batch=1, norm=0, beta=1.0), dict(batch=64, norm=1, beta=1.0, alpha=1e-3),
                 dict(batch=8, norm=1, beta=0.8, gamma=0.5, alpha=1e-3)):
        P0 = tiny["probe"] * (1.0 + 0.05j) if mode.get("gamma", 0) else tiny["probe"]
        A, amp = amps(pk, tiny["intensity"], m)
        O, P, st = run_gpu(pk, tiny, tiny["init"], P0, A, m, pk.PieParams(**mode),
                           precision=precision)
        Or, Pr, sr = opie.pie_sweep(tiny["init"], P0, tiny["pos"], amp, m, **mode)
        assert rel(O, Or) <= tol
        assert rel(P, Pr) <= tol
        assert abs(st[0][0] - sr[0]) <= tol * sr[0]


@pytest.mark.parametrize("precision,tol", [("split_bf16", 1e-4), ("split_fp16", 1e-5)])
def test_at_scale_one_sweep_split(pk, precision, tol):
    """The phase-1 sweep of the warm-started workload (900 positions, 128^2
    probe, m = 32, fully batched, overlap-normalised) in the split
    precisions: the launch configuration the benchmark times."""
    print("pie at scale", precision, flush=True)
    case = workloads.pie_at_scale()
    m = case["m"]
    A, amp = amps(pk, case["intensity"], m)
    params = dict(batch=900, norm=1, beta=1.0, gamma=0.0, alpha=1e-3)
    O, _, st = run_gpu(pk, case, case["init"], case["probe"], A, m, pk.PieParams(**params),
                       precision=precision)
    Or, _, sr = opie.pie_sweep(case["init"], case["probe"], case["pos"], amp, m, **params)
    assert rel(O, Or) <= tol
    assert abs(st[0][0] - sr[0]) <= tol * sr[0]


@pytest.mark.parametrize("params", [dict(batch=9, norm=1, beta=1.0, alpha=1e-3),
                                    dict(batch=64, norm=0, beta=0.05),
                                    dict(batch=5, norm=1, beta=0.8, gamma=0.5, alpha=1e-3),
                                    dict(batch=1, norm=0, beta=1.0)],
                         ids=["b9-norm", "b64-plain", "b5-probe", "b1-sequential"])
def test_order_with_missing_position_reuses_workspace(pk, tiny, params):
    """A sweep with a full permutation leaves every rank in the workspace;
    a second sweep over the same workspace whose order drops one position
    (an entry outside [0, J)) must not gather any stale slot: the dropped
    position contributes nothing and the chunks keep their places."""
    print("pie order missing", params, flush=True)
    m = tiny["m"]
    J = len(tiny["pos"])
    A, amp = amps(pk, tiny["intensity"], m)
    perm = np.random.default_rng(9).permutation(J).astype(np.int32)
    bad = perm.copy()
    bad[11] = J + 7
    n = tiny["probe"].shape[0]
    scan = pk.Scan(tiny["pos"], tiny["init"].shape, n, m)
    prm = pk.PieParams(**params)
    ws = torch.empty(scan.workspace_bytes(prm), dtype=torch.uint8, device="cuda")
    P0 = tiny["probe"] * (1.0 + 0.05j) if params.get("gamma", 0) else tiny["probe"]
    O = torch.from_numpy(tiny["init"]).cuda()
    P = torch.from_numpy(P0.astype(np.complex64)).cuda()
    pk.pie_sweep(O, P, scan, A, prm, order=torch.from_numpy(perm).cuda(), workspace=ws)
    O = torch.from_numpy(tiny["init"]).cuda()
    P = torch.from_numpy(P0.astype(np.complex64)).cuda()
    pk.pie_sweep(O, P, scan, A, prm, order=torch.from_numpy(bad).cuda(), workspace=ws)
    Or, Pr, _ = opie.pie_sweep(tiny["init"], P0, tiny["pos"], amp, m, order=bad, **params)
    assert rel(O.cpu().numpy(), Or) <= 1e-5
    assert rel(P.cpu().numpy(), Pr) <= 1e-5


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("split_bf16", 1e-4), ("split_fp16", 1e-5)])
def test_zero_exit_wave_projects_to_the_amplitude(pk, tiny, precision, tol):
    """A window of zero object gives u = 0 exactly; the projection then takes
    theta(0) = 0, i.e. u' = a (real), in every precision."""
    print("pie zero window", precision, flush=True)
    m = tiny["m"]
    n = tiny["probe"].shape[0]
    A, amp = amps(pk, tiny["intensity"], m)
    init = tiny["init"].copy()
    r, c = tiny["pos"][0]
    init[r:r + n, c:c + n] = 0
    params = dict(batch=64, norm=1, beta=1.0, alpha=1e-3)
    O, _, st = run_gpu(pk, tiny, init, tiny["probe"], A, m, pk.PieParams(**params), precision=precision)
    Or, _, sr = opie.pie_sweep(init, tiny["probe"], tiny["pos"], amp, m, **params)
    assert rel(O, Or) <= tol
    assert abs(st[0][0] - sr[0]) <= tol * sr[0]
    # the zero window moved to a non-zero estimate
    assert np.linalg.norm(O[r:r + n, c:c + n]) > 0


def test_sequential_overlap_normalised_dense(pk, tiny):
    """batch = 1 with the overlap-normalised step on the dense contraction.
    alpha = 0.1: at alpha = 1e-3 the per-pixel step 1/(|P|^2 + alpha max)
    reaches 1000 on the probe's tails and sixty-four chained FP32 steps
    amplify rounding far beyond the transform's error (the iterate itself
    is ill-conditioned there, in any arithmetic)."""
    m = tiny["m"]
    A, amp = amps(pk, tiny["intensity"], m)
    params = dict(batch=1, norm=1, beta=1.0, alpha=0.1)
    O, _, st = run_gpu(pk, tiny, tiny["init"], tiny["probe"], A, m, pk.PieParams(**params))
    Or, _, sr = opie.pie_sweep(tiny["init"], tiny["probe"], tiny["pos"], amp, m, **params)
    assert rel(O, Or) <= 1e-5
    assert abs(st[0][0] - sr[0]) <= 1e-5 * sr[0]


@pytest.mark.parametrize("precision,tol", [("split_bf16", 1e-4), ("split_fp16", 1e-6)])
def test_noise_free_fixed_point_split(pk, tiny, precision, tol):
    A, amp = amps(pk, tiny["intensity"], tiny["m"])
    O, _, _ = run_gpu(pk, tiny, tiny["obj"], tiny["probe"], A, tiny["m"],
                      pk.PieParams(batch=64, norm=1, beta=1.0, alpha=1e-3), precision=precision)
    assert rel(O, tiny["obj"]) <= tol


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("split_fp16", 1e-5)])
@pytest.mark.parametrize("params", [dict(batch=1, norm=0, beta=1.0, gamma=0.3),
                                    dict(batch=1, norm=1, beta=1.0, alpha=0.1)], ids=["plain", "norm"])
def test_sequential_sweep_on_a_large_object(pk, precision, tol, params):
    """Sequential sweeps of small windows run in one persistent workgroup;
    an object too large for it to hold (300 x 300) takes the variant that
    updates global memory: both match the oracle, as the LDS variant does on
    the tiny workload (the other sequential tests)."""
    print("pie sequential large object", precision, params, flush=True)
    rng = np.random.default_rng(8)
    H = W = 300
    n, m = 32, 16
    obj = (rng.uniform(0.5, 1, (H, W)) * np.exp(1j * rng.uniform(-1, 1, (H, W)))).astype(np.complex64)
    probe = workloads.gaussian_probe(n, 6.0, np.pi / 144.0)
    pos = workloads.raster(5, 5, 20, 90)
    case = dict(pos=pos, probe=probe)
    amp = np.abs(rng.standard_normal((len(pos), m, m))).astype(np.float32) * 40
    O, P, st = run_gpu(pk, case, obj, probe, amp, m, pk.PieParams(**params), precision=precision)
    Or, Pr, sr = opie.pie_sweep(obj, probe, pos, amp, m, **params)
    assert rel(O, Or) <= tol and rel(P, Pr) <= tol
    assert abs(st[0][0] - sr[0]) <= tol * sr[0] and abs(st[0][1] - sr[1]) <= 1e-4 * sr[1]


@pytest.mark.parametrize("norm", [0, 1])
def test_sequential_sweep_of_mixed_overlap(pk, tiny, norm):
    """batch = 1 over a scan whose windows partly overlap: a 3 x 3 grid of
    disjoint windows (step 40 > n = 32) and a cluster of four overlapping
    ones, in a shuffled order with one entry outside [0, J).  Positions of
    disjoint windows run side by side on the device; the result must be the
    one-by-one sweep in the given order."""
    m = tiny["m"]
    grid = [(4 + 40 * a, 4 + 40 * b) for a in range(3) for b in range(3)]
    cluster = [(60, 60), (66, 62), (62, 70), (70, 68)]
    pos = np.asarray(grid + cluster, dtype=np.int32)
    J = len(pos)
    inten = workloads.intensities(tiny["obj"], tiny["probe"], pos)
    A, amp = amps(pk, inten, m)
    case = dict(tiny, pos=pos)
    order = np.random.default_rng(17).permutation(J).astype(np.int32)
    order[5] = J + 3  # skipped
    params = dict(batch=1, norm=norm, beta=1.0, alpha=0.1)
    O, _, st = run_gpu(pk, case, tiny["init"], tiny["probe"], A, m, pk.PieParams(**params), order=order)
    Or, _, sr = opie.pie_sweep(tiny["init"], tiny["probe"], pos, amp, m, order=order, **params)
    assert rel(O, Or) <= 1e-5
    assert abs(st[0][0] - sr[0]) <= 1e-5 * sr[0]
    assert abs(st[0][1] - sr[1]) <= 1e-4 * sr[1]


@pytest.mark.parametrize("box", [(96, 88), (96, 120), (100, 104), (112, 124)])
def test_sequential_sweep_near_the_lds_limit(pk, tiny, box):
    """batch = 1 with m = 32 over bounding boxes whose object rows, probe and
    tables come close to the compute unit's LDS: whether the launch holds
    them in LDS (its own static arrays counted) or falls back to the loop on
    global memory, the sweep is eq. (5) in sweep order."""
    h, w = box
    n = tiny["probe"].shape[0]
    m = 32
    pos = np.asarray([(0, 0), (h - n, 0), (0, w - n), (h - n, w - n), ((h - n) // 2, (w - n) // 2)], dtype=np.int32)
    inten = workloads.intensities(tiny["obj"], tiny["probe"], pos)
    A, amp = amps(pk, inten, m)
    case = dict(tiny, pos=pos)
    params = dict(batch=1, norm=0, beta=1.0)
    O, _, st = run_gpu(pk, case, tiny["init"], tiny["probe"], A, m, pk.PieParams(**params))
    Or, _, sr = opie.pie_sweep(tiny["init"], tiny["probe"], pos, amp, m, **params)
    assert rel(O, Or) <= 1e-5
    assert abs(st[0][0] - sr[0]) <= 1e-5 * sr[0]
