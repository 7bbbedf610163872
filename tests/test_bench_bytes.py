"""The bench's count of touched grid values (the grid part of the algorithmic
bytes), CPU only: one node touches 27 points per lattice; coincident nodes
share them; a brute-force set union over small random node sets agrees."""
import importlib.util
import os

import numpy as np

from paper_1612_03399_amd import workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)


def brute(X, grid, offsets):
    n = (grid.nx, grid.ny, grid.nz)
    pts = set()
    for li, off in enumerate(offsets):
        for x in X:
            c = [int(np.floor(x[a] / grid.h - off[a] + 0.5)) for a in range(3)]
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        pts.add((li, (c[0] + dx) % n[0], (c[1] + dy) % n[1], (c[2] + dz) % n[2]))
    return len(pts)


def test_single_and_coincident_nodes():
    g = W.Grid(16, 16, 16, 1.0 / 16)
    x = np.array([[0.31, 0.52, 0.77]])
    assert bench.touched_points(x, g) == 81
    assert bench.touched_points(np.vstack([x, x]), g) == 81
    far = np.vstack([x, x + 0.4])
    assert bench.touched_points(far, g) == 162
    # the cell-centred lattice alone
    assert bench.touched_points(x, g, ((0.5, 0.5, 0.5),)) == 27


def test_matches_brute_force_union_with_wrap():
    rng = np.random.default_rng(3)
    g = W.Grid(12, 10, 14, 0.1)
    for _ in range(5):
        X = rng.uniform(0, 1.0, size=(40, 3)) * np.array([1.2, 1.0, 1.4])
        assert bench.touched_points(X, g) == brute(X, g, bench.MAC_OFFSETS)


def test_device_count_matches_numpy():
    """The torch count the bench uses on large batches (run here on the CPU
    device) agrees with the numpy union."""
    rng = np.random.default_rng(4)
    g = W.Grid(12, 10, 14, 0.1)
    for _ in range(3):
        X = rng.uniform(0, 1.0, size=(60, 3)) * np.array([1.2, 1.0, 1.4])
        assert bench.touched_points_device(X, g, device="cpu") == bench.touched_points(X, g)
    off = bench.MAC_OFFSETS + ((0.5, 0.5, 0.5),)
    X = rng.uniform(0, 1.0, size=(30, 3))
    assert (bench.touched_points_device(X, g, off, device="cpu")
            == bench.touched_points(X, g, off))


def test_parallel_oracle_baseline_reproduces_the_serial_step():
    """The bench's multi-process oracle (bodies split in ranges, per-process
    force fields summed by slab) gives the serial oracle's field."""
    wl = W.small_suspension(6, 2, 32)
    u = wl.velocity()
    logs = []
    out = bench.cpu_baseline(wl, u, logs.append, single_budget_s=0.0)
    assert out["kind"] == "oracle" and out["single_thread_value"] > 0
    if out["cores"] > 1:
        assert out["parallel_field_rel_diff"] <= 1e-13
        assert out["value"] == out["parallel_value"]
