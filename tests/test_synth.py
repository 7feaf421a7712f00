"""The shared seeded-input module: SplitMix64 known answers and generator shapes."""
import json
import os

import numpy as np

import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_splitmix64_known_answers():
    # the published SplitMix64 sequence from state 0 (Steele, Lea and Flood, 2014)
    a, b = (int(v, 16) for v in GOLD["splitmix64_seed0"])
    assert synth.splitmix64(0) == a
    assert synth.splitmix64(synth.GOLDEN) == b
    z = synth._splitmix64_np(np.array([0, synth.GOLDEN], dtype=np.uint64))
    assert int(z[0]) == a and int(z[1]) == b


def test_uniform_is_counter_based():
    u = synth.uniform(5, 3, np.arange(1000, dtype=np.uint64))
    assert np.all((u >= 0) & (u < 1)) and abs(u.mean() - 0.5) < 0.05
    assert synth.uniform(5, 3, 417)[()] == u[417]
    assert not np.array_equal(u, synth.uniform(5, 4, np.arange(1000, dtype=np.uint64)))


def test_slab_and_droplet_profiles():
    r = synth.slab(64, 4, 0.3, 0.02, 16, 48, 2.0)
    assert r.shape == (4, 64) and r.flags.c_contiguous
    assert abs(r[0, 32] - 0.3) < 1e-12 and abs(r[0, 0] - 0.02) < 1e-12
    assert abs(r[0, 16] - 0.16) < 1e-3                  # mid-value at the interface
    d = synth.droplet(64, 64, 0.3, 0.02, 10)
    assert abs(d[32, 32] - 0.3) < 1e-9 and abs(d[0, 0] - 0.02) < 1e-12
    n = synth.slab(64, 4, 0.3, 0.02, noise=0.01, seed=9)
    assert np.all(np.abs(n / r - 1) <= 0.01)


def test_droplet_layout_non_overlapping():
    c, rad = synth.droplet_layout(512, 512, 8, 10, 30, gap=16, seed=3)
    for i in range(8):
        for j in range(i):
            dx = abs(c[i][0] - c[j][0]); dx = min(dx, 512 - dx)
            dy = abs(c[i][1] - c[j][1]); dy = min(dy, 512 - dy)
            assert np.hypot(dx, dy) >= rad[i] + rad[j] + 16


def test_sweep_runs_ranges():
    runs = synth.sweep_runs(256)
    assert len(runs) == 256
    for r in runs:
        assert r["nx"] % 32 == 0 and 64 <= r["nx"] <= 512
        assert r["ny"] % 16 == 0 and 16 <= r["ny"] <= 64
        assert 0.5 <= r["t_over_tc"] <= 0.95 and 0.6 <= r["tau"] <= 1.5 and 0 <= r["sigma"] <= 0.2
    assert len({r["nx"] for r in runs}) == 15 and len({r["ny"] for r in runs}) == 4
