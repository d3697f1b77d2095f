"""The seeded input generators (CPU): determinism and the threaded smoothing.

Large models smooth their noise in slabs on a thread pool; every slab's lines
are filtered by the same call as in one whole-array pass, so the model must
be the same bit for bit whichever path built it."""
import numpy as np
from scipy.ndimage import gaussian_filter1d

import synth


def serial_noise(seed, shape, sigma):
    p = np.random.default_rng(seed).standard_normal(shape, dtype=np.float32)
    for ax in range(3):
        p = gaussian_filter1d(p, sigma, axis=ax, mode="reflect")
    return p / float(p.std())


def test_threaded_smoothing_equals_one_pass():
    shape = (200, 180, 160)          # above the threading threshold
    assert np.prod(shape) >= 1 << 22
    a = synth._smooth_noise(np.random.default_rng(5), shape, 4.0)
    assert np.array_equal(a, serial_noise(5, shape, 4.0))
    for ax in range(3):
        p = np.random.default_rng(ax).standard_normal((37, 41, 43)).astype(np.float32)
        assert np.array_equal(synth._filter_axis(p, 4.0, ax, 5),
                              gaussian_filter1d(p, 4.0, axis=ax, mode="reflect"))


def test_models_are_seeded():
    a = synth.layered_velocity(40, 30, 50, 5, seed=9)
    b = synth.layered_velocity(40, 30, 50, 5, seed=9)
    c = synth.layered_velocity(40, 30, 50, 5, seed=10)
    assert a.dtype == np.float32 and np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 1350.0 and a.max() <= 4950.0
    shapes = synth.batch_shapes()
    assert shapes == synth.batch_shapes() and len(shapes) == 64
    assert all(128 <= v <= 384 and v % 16 == 0 for s in shapes for v in s[:3])
    reqs = synth.serve_requests()
    assert len(reqs) == 256 and all(np.diff([r["t"] for r in reqs]) > 0)
