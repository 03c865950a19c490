"""Seeded workload generators: determinism, shapes and distributions (no GPU)."""
import numpy as np

import workloads as W


def test_small_fp64_gram_shapes_and_time_channel():
    x, y = W.small_fp64_gram(0)
    assert x.shape == (8, 65, 4) and y.shape == (8, 65, 4) and x.dtype == np.float64
    np.testing.assert_allclose(x[:, :, 3], np.broadcast_to(np.arange(65) / 64, (8, 65)))
    assert np.all(x[:, 0, :] == 0)
    x2, _ = W.small_fp64_gram(0)
    assert np.array_equal(x, x2)
    inc = np.diff(x[:, :, :3], axis=1)
    assert abs(inc.std() - 1 / 8) < 0.01


def test_batched_interp_gram():
    x, y = W.batched_interp_gram(0, n=16)
    assert x.shape == (16, 257, 8) and x.dtype == np.float32
    inc = np.diff(x.astype(np.float64), axis=1)
    assert abs(inc.std() - 0.5 / 16) < 0.002
    assert not np.array_equal(x, y)


def test_uneven_pairs_lengths():
    xs, ys = W.uneven_pairs(0, npairs=64)
    lens = np.array([len(a) for a in xs] + [len(b) for b in ys])
    assert lens.min() >= 32 and lens.max() <= 2048
    assert all(a.shape[1] == 16 and a.dtype == np.float32 for a in xs)


def test_mmd_sets_drift():
    x, y = W.mmd_sets(0)
    assert x.shape == (64, 513, 5)
    dx = np.diff(x.astype(np.float64), axis=1).mean()
    dy = np.diff(y.astype(np.float64), axis=1).mean()
    assert abs(dx) < 2e-3 and abs(dy - 0.3 / 512) < 2e-3


def test_large_gram_cell_constant_scale():
    x, y = W.large_gram(0, n=4, steps=64)
    dx = np.diff(x.astype(np.float64), axis=1)
    dy = np.diff(y.astype(np.float64), axis=1)
    c = np.einsum("aid,bjd->abij", dx, dy)
    assert 0.8 < c.std() < 1.2


def test_long_paths_gram():
    x, y = W.long_paths_gram(0, n=2, steps=512)
    assert x.shape == (2, 513, 8) and y.shape == (2, 513, 8) and x.dtype == np.float32
    assert np.all(x[:, 0] == 0) and not np.array_equal(x, y)
    inc = np.diff(x.astype(np.float64), axis=1)
    assert abs(inc.std() - 0.5 / np.sqrt(512)) < 0.002
