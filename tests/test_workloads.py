"""The seeded generators are deterministic and produce the documented shapes and ranges."""
import math

import numpy as np

from paper_1610_05258_amd import workloads as wl


def test_stratified_cells_and_determinism():
    x, y = wl.stratified_2d(5, 6, 4, 3, 2.0, 1.0)
    x2, y2 = wl.stratified_2d(5, 6, 4, 3, 2.0, 1.0)
    assert np.array_equal(x, x2) and np.array_equal(y, y2)
    cx = np.floor(x / (2.0 / 6)).astype(int)
    cy = np.floor(y / (1.0 / 4)).astype(int)
    assert np.array_equal(np.bincount(cx + 6 * cy, minlength=24), np.full(24, 3))


def test_zalesak_disk_and_rotation():
    prob, a, x, y = wl.zalesak_2d(n=64, ppc=4)
    assert a.dtype == np.float32 and prob["x"].dtype == np.float32
    frac = a.mean()
    disk = math.pi * 0.15 ** 2 - 0.05 * 0.25
    assert abs(frac - disk) < 0.01
    xr, yr = wl.zalesak_rotate(x, y, 2 * math.pi)
    assert np.allclose(xr, x, atol=1e-12) and np.allclose(yr, y, atol=1e-12)
    xq, yq = wl.zalesak_rotate(x, y, math.pi / 2)
    assert abs(wl.zalesak_disk(xq, yq).mean() - frac) < 0.01    # area preserved


def test_taylor_green_workload():
    prob, vals = wl.taylor_green_2d(seed=2, n=32, ppc=8, steps=5, dt=1e-3)
    assert vals.shape == (3, 32 * 32 * 8) and vals.dtype == np.float32
    assert prob["x"].min() >= 0 and prob["x"].max() <= np.float32(2 * math.pi)
    batch = wl.uneven_batch(seed=3, count=5)
    assert len(batch) == 5
    for p, v in batch:
        assert 32 <= p["nx"] <= 512 and v.shape[0] == 2
