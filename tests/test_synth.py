"""The seeded generator is deterministic and produces the documented structure."""
import numpy as np

import synth


def test_deterministic_and_structured():
    a = synth.make(1, H=64, W=48, B=8)
    b = synth.make(1, H=64, W=48, B=8)
    np.testing.assert_array_equal(a.y, b.y)
    np.testing.assert_array_equal(a.masks, b.masks)
    assert a.gt.dtype == np.float32 and a.y.dtype == np.float32 and a.masks.dtype == np.uint8
    assert a.gt.shape == (8, 64, 48) and a.y.shape == (1, 64, 48) and a.masks.shape == (8, 64, 48)
    assert set(np.unique(a.masks)) <= {0, 1}
    assert 0.0 <= a.gt.min() and a.gt.max() <= 1.0
    assert abs(a.masks.mean() - 0.5) < 0.02
    c = synth.make(1, snapshot=1, H=64, W=48, B=8)
    assert not np.array_equal(a.y, c.y)


def test_blob_sum_matches_direct_evaluation():
    rng = np.random.default_rng([1, 2])
    vol = synth.blob_volume(rng, 4, 9, 11, 5)
    rng = np.random.default_rng([1, 2])
    cz, cy, cx = rng.uniform(0, 4, 5), rng.uniform(0, 9, 5), rng.uniform(0, 11, 5)
    sxy, sz, a = rng.uniform(3, 6, 5), rng.uniform(1, 2, 5), rng.uniform(0.3, 1, 5)
    z, y, x = np.meshgrid(np.arange(4), np.arange(9), np.arange(11), indexing="ij")
    ref = sum(a[i] * np.exp(-((x - cx[i]) ** 2 + (y - cy[i]) ** 2) / (2 * sxy[i] ** 2)
                            - (z - cz[i]) ** 2 / (2 * sz[i] ** 2)) for i in range(5))
    np.testing.assert_allclose(vol, ref, rtol=1e-12, atol=1e-14)


def test_batch_shapes_cover_the_grid():
    shapes = synth.batch_shapes()
    assert len(shapes) == 64
    assert {(h, w) for h, w, _ in shapes} <= set(synth.BATCH_SIZES)
    assert {r for _, _, r in shapes} <= set(synth.BATCH_DEPTHS)
    assert shapes == synth.batch_shapes()
