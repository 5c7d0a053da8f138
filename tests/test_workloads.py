"""The seeded input recipes: shapes, value ranges, determinism, subsets."""

import numpy as np

import workloads


def test_tiny_pie_shapes_and_ranges():
    c = workloads.tiny_pie()
    assert c["obj"].shape == (128, 128) and c["obj"].dtype == np.complex64
    amp = np.abs(c["obj"])
    assert amp.min() >= 0.8 - 1e-6 and amp.max() <= 1.0 + 1e-6
    assert np.max(np.abs(np.angle(c["obj"]))) <= np.pi / 2 + 1e-5
    assert c["probe"].shape == (32, 32) and abs(np.abs(c["probe"]).max() - 1) < 0.05
    assert c["pos"].shape == (64, 2) and c["pos"].min() == 20 and c["pos"].max() == 76
    assert c["intensity"].shape == (64, 32, 32) and c["m"] == 16 and "amp" not in c
    again = workloads.tiny_pie()
    assert np.array_equal(again["obj"], c["obj"]) and np.array_equal(again["init"], c["init"])


def test_pft_patch_subsets_are_consistent():
    full = workloads.pft_patches(32, range(130))
    sub = workloads.pft_patches(32, [129, 3, 64])
    assert np.array_equal(sub, full[[129, 3, 64]])
    y = workloads.pft_coeffs(8, [5, 70])
    assert y.shape == (2, 8, 8) and not np.array_equal(y[0], y[1])
    assert abs(np.std(full.real) - 1) < 0.02 and abs(np.std(full.imag) - 1) < 0.02


def test_grouped_descriptors_are_packed_aligned_and_balanced():
    d, tin, tout = workloads.grouped_descs(count=64, seed=5)
    assert d.shape == (64, 4)
    for s in workloads.GROUP_SIZES:
        assert np.sum(d[:, 0] == s) == 16
    assert np.all(d[:, 1] == d[:, 0] // 4)
    assert np.all(d[:, 2] % 32 == 0) and np.all(d[:, 3] % 32 == 0)
    assert d[-1, 2] + d[-1, 0] ** 2 == tin and d[-1, 3] + d[-1, 1] ** 2 == tout
    x = workloads.grouped_inputs(d, tin, idx=[3])
    n, _, io, _ = d[3]
    assert np.count_nonzero(x) == n * n and np.count_nonzero(x[io:io + n * n]) == n * n
    a = workloads.adjoint_descs(d)
    assert np.array_equal(a[:, 2], d[:, 3])


def test_scan_positions_stay_inside_objects():
    rs = workloads.streams(3)
    pos = workloads.raster(30, 30, 24, 100, rng=rs[2], jitter=2)
    assert pos.min() >= 98 and pos.max() + 128 <= 1024
    assert len(np.unique(pos, axis=0)) == 900


def test_poisson_scaling_hits_the_photon_budget():
    rng = np.random.default_rng(0)
    inten = np.abs(rng.standard_normal((50, 16, 16))).astype(np.float32) * 3
    noisy = workloads.poisson(rng, inten, 1e4)
    s = 1e4 / np.mean(inten.astype(np.float64).sum(axis=(1, 2)))
    counts = noisy.astype(np.float64) * s
    assert np.allclose(counts, np.round(counts), atol=1e-2)
    assert abs(counts.sum(axis=(1, 2)).mean() / 1e4 - 1) < 0.01


def test_masked_field_recipe_small():
    from oracle import pft
    c = workloads.masked_field(field=256, m=32, coarse=32, sigma_f=4.0)
    n = 128
    assert c["obj"].shape == (256, 256) and c["probe"].shape == (n, n) and c["amp"].shape == (9, 32, 32)
    assert np.allclose(np.abs(c["obj"]), 1.0, atol=1e-6)
    # serpentine scan: down the first column, up the second, down the third
    assert c["pos"].tolist() == [[0, 0], [64, 0], [128, 0], [128, 64], [64, 64], [0, 64],
                                 [0, 128], [64, 128], [128, 128]]
    # amplitudes: magnitudes of the kept coefficients of the masked field's
    # 256-point DFT (the oracle's transform with period and window shift)
    for j in (0, 4, 8):
        r, col = c["pos"][j]
        u = pft.forward(c["probe"] * c["obj"][r:r + n, col:col + n], 32, period=256, shift=(r, col))
        assert np.max(np.abs(np.abs(u) - c["amp"][j])) <= 1e-6 * np.max(np.abs(u))
    sub = workloads.masked_field(field=256, m=32, coarse=32, sigma_f=4.0, amp_positions=[4], with_init=False)
    assert sub["init"] is None and np.array_equal(sub["amp"][0], c["amp"][4])
