"""Pins of the coherence-weighted merging oracle (Section 4.4, Eq. 8-9)."""
import numpy as np

from oracle import merge


def _frames(n, shape=(5, 7), seed=0):
    rng = np.random.default_rng(seed)
    return [rng.normal(size=shape) + 1j * rng.normal(size=shape) for _ in range(n)]


def test_identical_frames_are_fully_coherent():
    f = _frames(1)[0]
    m, C = merge.coherence_merge([f, f, f], eps=1e-6)
    np.testing.assert_allclose(C, 3 * np.abs(f) / (1e-6 + 3 * np.abs(f)), rtol=1e-14)
    np.testing.assert_allclose(m, C * np.abs(f), rtol=1e-14)


def test_opposite_frames_cancel():
    f = _frames(1, seed=1)[0]
    m, C = merge.coherence_merge([f, -f], eps=1e-6)
    assert np.all(C == 0) and np.all(m == 0)


def test_bounds_and_phase_invariance():
    fs = _frames(4, seed=2)
    m, C = merge.coherence_merge(fs, eps=1e-3)
    assert np.all(C >= 0) and np.all(C < 1)
    # a common phase on every frame changes nothing
    rot = np.exp(0.7j)
    m2, C2 = merge.coherence_merge([rot * f for f in fs], eps=1e-3)
    np.testing.assert_allclose(C2, C, rtol=1e-13)
    np.testing.assert_allclose(m2, m, rtol=1e-13)


def test_single_frame_and_by_hand():
    f = np.array([3 + 4j, 0j])
    m, C = merge.coherence_merge([f], eps=1.0)
    np.testing.assert_allclose(C, [5 / 6, 0.0], rtol=1e-15)
    np.testing.assert_allclose(m, [25 / 6, 0.0], rtol=1e-15)
    # two frames with a right angle between them: |S| = sqrt(2) |f|, A = 2 |f|
    g = np.array([1 + 0j])
    m, C = merge.coherence_merge([g, 1j * g], eps=0.5)
    np.testing.assert_allclose(C, [np.sqrt(2) / 2.5], rtol=1e-15)
    np.testing.assert_allclose(m, [np.sqrt(2) / 2.5 * np.sqrt(2) / 2], rtol=1e-15)


def test_stream_window():
    fs = _frames(5, seed=3)
    seq = merge.merge_sequence(fs, window=3, eps=1e-6)
    assert len(seq) == 5
    np.testing.assert_allclose(seq[0][1], merge.coherence_merge(fs[:1], 1e-6)[1])
    np.testing.assert_allclose(seq[4][0], merge.coherence_merge(fs[2:5], 1e-6)[0])
