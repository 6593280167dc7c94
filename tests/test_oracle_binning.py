"""Pins of the binning oracle (photon binner, Section 4.1)."""
import numpy as np

import scenes
from oracle import binning


def test_matches_bincount_library_routine():
    ev = scenes.random_events(200_000, 16, 12, 64, 20, seed=3, invalid_frac=0.1)
    hist, dropped = binning.bin_events(ev["pixel"], ev["t_ps"], 16, 12, 64, 20)
    p = ev["pixel"].astype(np.int64)
    t = ev["t_ps"].astype(np.int64)
    ok = (p >= 0) & (p < 16 * 12) & (t // 20 < 64)
    ref = np.bincount(p[ok] * 64 + t[ok] // 20, minlength=16 * 12 * 64)
    assert np.array_equal(hist.ravel(), ref.astype(np.uint64))
    assert dropped == int((~ok).sum())


def test_conservation():
    ev = scenes.random_events(50_000, 8, 8, 32, 7, seed=4, invalid_frac=0.2)
    hist, dropped = binning.bin_events(ev["pixel"], ev["t_ps"], 8, 8, 32, 7)
    assert int(hist.sum()) + dropped == len(ev)


def test_permutation_invariance():
    ev = scenes.random_events(30_000, 8, 8, 32, 7, seed=5, invalid_frac=0.05)
    h1, d1 = binning.bin_events(ev["pixel"], ev["t_ps"], 8, 8, 32, 7)
    rng = np.random.default_rng(0)
    ev2 = ev[rng.permutation(len(ev))]
    h2, d2 = binning.bin_events(ev2["pixel"], ev2["t_ps"], 8, 8, 32, 7)
    ev3 = ev[np.argsort(ev["pixel"], kind="stable")]
    h3, d3 = binning.bin_events(ev3["pixel"], ev3["t_ps"], 8, 8, 32, 7)
    assert np.array_equal(h1, h2) and np.array_equal(h1, h3)
    assert d1 == d2 == d3


def test_brute_force_8x8x8():
    ev = scenes.random_events(10_000, 8, 8, 8, 5, seed=6, invalid_frac=0.1)
    h1, d1 = binning.bin_events(ev["pixel"], ev["t_ps"], 8, 8, 8, 5, t0_ps=3)
    h2, d2 = binning.bin_events_loop(ev["pixel"], ev["t_ps"], 8, 8, 8, 5, t0_ps=3)
    assert np.array_equal(h1, h2) and d1 == d2


def test_edges_and_degenerate():
    # left-closed bins, t0 offset, the last valid picosecond, empty input
    pix = np.array([0, 0, 0, 0, 3, -1, 4], dtype=np.int32)
    t = np.array([10, 14, 15, 10 + 4 * 5 - 1, 10 + 4 * 5, 12, 12], dtype=np.uint32)
    h, d = binning.bin_events(pix, t, 2, 2, 4, 5, t0_ps=10)
    assert h[0, 0, 0] == 2 and h[0, 0, 1] == 1 and h[0, 0, 3] == 1
    assert d == 3  # late event, negative pixel, pixel == nx*ny
    h, d = binning.bin_events(np.zeros(0, np.int32), np.zeros(0, np.uint32), 2, 2, 4, 5)
    assert h.sum() == 0 and d == 0
    h, d = binning.bin_events(np.array([0], np.int32), np.array([3], np.uint32), 2, 2, 4, 5,
                              t0_ps=10)
    assert h.sum() == 0 and d == 1  # earlier than t0
