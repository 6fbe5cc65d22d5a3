"""Seeded workload generators: sizes, seeds and layout of the six workloads."""
import numpy as np

import workloads


def test_sizes_and_layout():
    w = workloads.make("cantilever")
    assert w["n"] == 20 and w["bc"][0] == 1 and w["field"].shape == (1, 1, 12)
    w = workloads.make("twisted_rod")
    assert w["n"] == 4096 and w["bc"][-1] == 2 and w["drive_period"] == 10_000
    w = workloads.make("cilia_carpet")
    assert len(w["rod_member"]) == 1024
    lens = np.diff(w["rod_offset"])
    assert lens.min() >= 16 and lens.max() <= 128
    assert 70_000 < w["n"] < 77_000
    assert w["field"].shape == (2000, 1, 12)
    np.testing.assert_allclose(np.linalg.norm(w["field"][:, 0, :3], axis=1), 1.0)
    w = workloads.make("rod_array")
    assert w["n"] == 262_144 and len(w["rod_member"]) == 512
    assert w["field"].shape[0] == 40_000
    assert w["field"][:, 0, 2].min() == -2.0 and w["field"][:, 0, 2].max() == 2.0
    w = workloads.make("ensemble")
    assert w["n"] == 64 * 4096 and w["n_members"] == 64
    assert w["field"].shape == (1, 64, 12)
    w = workloads.make("adjoint_rod")
    assert w["n"] == 256 and np.linalg.norm(w["target"] - w["x_ref"][0]) <= 0.5 * 255


def test_seeded_and_perturbed():
    a = workloads.make("twisted_rod", n=64)
    b = workloads.make("twisted_rod", n=64)
    np.testing.assert_array_equal(a["x0"], b["x0"])
    free = a["bc"] == 0
    d = a["x0"] - a["x_ref"]
    assert np.all(d[~free] == 0)
    assert 0.5e-3 < d[free].std() < 2e-3
