"""Seeded input generators: the video-like feature sequence."""
import numpy as np

import synth


def test_sequence_frames_are_standardized_and_moved_copies():
    eps = 0.3
    base = synth.feature_map(32, 32, 8, 4.0, 12).astype(np.float64)
    for t in (0, 1, 2, -3):
        ft = synth.sequence_frame(32, 32, 8, 4.0, 12, t, eps=eps, step_px=(3.0, 0.0)).astype(np.float64)
        assert np.allclose(ft.mean(axis=(0, 1)), 0.0, atol=1e-5)
        assert np.allclose(ft.std(axis=(0, 1)), 1.0, atol=1e-5)
        # an integer shift along x (the W axis) is an exact periodic roll of the base field
        moved = np.roll(base, 3 * t, axis=1)
        corr = np.mean(ft * moved, axis=(0, 1))
        # the fresh part is independent: correlation sqrt(1 - eps^2) up to sampling noise
        assert np.all(np.abs(corr - np.sqrt(1 - eps * eps)) < 0.15), corr
        if t != 0:
            unmoved = np.mean(ft * base, axis=(0, 1))
            assert np.mean(corr) > np.mean(unmoved) + 0.1


def test_sequence_frames_are_deterministic_and_distinct():
    a = synth.sequence_frame(16, 16, 2, 2.0, 5, 3)
    b = synth.sequence_frame(16, 16, 2, 2.0, 5, 3)
    c = synth.sequence_frame(16, 16, 2, 2.0, 5, 4)
    d = synth.sequence_frame(16, 16, 2, 2.0, 5, 0)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    assert not np.array_equal(d, synth.feature_map(16, 16, 2, 2.0, 5))
