"""Pins of the depth-dependent average oracle (Section 4.4, DDA).

Each pin fixes the result independently of the oracle's own loop: a library mean, the
identity, closed forms of a ramp in time, and the default table's end points and shape.
"""
import numpy as np
import pytest

from oracle import dda


def _frames(n, shape=(4, 5, 6), seed=0):
    rng = np.random.default_rng(seed)
    return [rng.gamma(2.0, size=shape) for _ in range(n)]


@pytest.mark.parametrize("n_frames,window", [(1, 3), (2, 3), (3, 3), (7, 3), (5, 1)])
def test_uniform_weights_are_the_window_mean(n_frames, window):
    fs = _frames(n_frames)
    W = np.full((fs[0].shape[-1], window), 0.37)
    for i, (avg, img) in enumerate(dda.dda_sequence(fs, W)):
        ref = np.mean(np.stack(fs[max(0, i - window + 1):i + 1]), axis=0)
        np.testing.assert_allclose(avg, ref, rtol=1e-14)
        np.testing.assert_array_equal(img, np.max(avg, axis=-1))


def test_newest_only_weights_give_the_newest_frame():
    fs = _frames(6, seed=1)
    W = np.zeros((fs[0].shape[-1], 4))
    W[:, 0] = 2.5
    for i, (avg, _) in enumerate(dda.dda_sequence(fs, W)):
        np.testing.assert_allclose(avg, fs[i], rtol=2e-16)


def test_constant_stream_is_a_fixed_point_and_rows_scale_freely():
    f = _frames(1, seed=2)[0]
    rng = np.random.default_rng(3)
    W = rng.uniform(0.0, 1.0, size=(f.shape[-1], 5))
    W[:, 0] += 0.1
    avg, _ = dda.dda([f] * 5, W)
    np.testing.assert_allclose(avg, f, rtol=1e-14)
    fs = _frames(5, seed=4)
    a1, _ = dda.dda(fs, W)
    a2, _ = dda.dda(fs, W * rng.uniform(0.5, 3.0, size=(f.shape[-1], 1)))
    np.testing.assert_allclose(a2, a1, rtol=1e-13)


@pytest.mark.parametrize("n_depth,window", [(64, 3), (9, 5), (2, 4), (1, 6), (100, 1)])
def test_default_table(n_depth, window):
    n = dda.default_frames(n_depth, window)
    assert n[0] == (1 if n_depth > 1 else window) and n[-1] == window
    assert np.all(np.diff(n) >= 0) and np.all((n >= 1) & (n <= window))
    W = dda.default_weights(n_depth, window)
    assert W.shape == (n_depth, window)
    np.testing.assert_array_equal(W.sum(axis=1), n)
    # every row is a prefix of ones: the n_d newest frames
    assert np.all(np.diff(W, axis=1) <= 0)


def test_default_table_by_hand():
    # N_w = 3 over 5 planes: (N_w - 1) d / 4 = 0, 0.5, 1, 1.5, 2 -> rounded half up 0, 1, 1, 2, 2
    np.testing.assert_array_equal(dda.default_frames(5, 3), [1, 2, 2, 3, 3])
    np.testing.assert_array_equal(dda.default_frames(3, 4), [1, 3, 4])


@pytest.mark.parametrize("n_depth,window", [(9, 5), (16, 3)])
def test_default_table_on_a_ramp_in_time(n_depth, window):
    # frame k holds the value k everywhere: the average of the n newest of frames 0..i is
    # i - (n - 1) / 2, with n = min(n_d, i + 1) at depth d
    frames = [np.full((3, 2, n_depth), float(k)) for k in range(9)]
    n_d = dda.default_frames(n_depth, window)
    for i, (avg, img) in enumerate(dda.dda_sequence(frames, dda.default_weights(n_depth, window))):
        n = np.minimum(n_d, i + 1)
        np.testing.assert_allclose(avg, np.broadcast_to(i - (n - 1) / 2.0, avg.shape), rtol=1e-15)
        # the nearest plane averages the fewest frames, so it holds the maximum of a rising ramp
        np.testing.assert_allclose(img, float(i), rtol=1e-15)
