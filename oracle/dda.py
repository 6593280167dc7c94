"""Depth-dependent average of the last N_w depth volumes (Section 4.4, DDA) -- FP64, test
infrastructure only.

The method keeps a ring of the N_w most recent reconstructed volumes (magnitudes, depth
last) and averages them with weights that depend on the depth; the image is the maximum
over depth of the average.  The paper does not give the weights.  Reading used here: a
table W[d][a] >= 0 (a = how many frames back, 0 = the newest), each voxel value at depth d
is sum_a W[d][a] v_{i-a} / sum_a W[d][a] over the frames present (a < min(i + 1, N_w)),
and W[d][0] > 0 so that the sum of weights never vanishes.  Default table: at depth index
d of n_depth the n_d newest frames weigh 1 and the older ones 0, with n_d growing
linearly from 1 at the nearest plane to N_w at the farthest, rounded half up:
n_d = 1 + floor((N_w - 1) d / (n_depth - 1) + 1/2); a single plane averages all N_w.
Far planes return less light, so they get the longer window; near planes keep the
frame rate.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence, Tuple

import numpy as np


def default_frames(n_depth: int, window: int) -> np.ndarray:
    """n_d for every depth index d (exact rational rounding)."""
    if n_depth == 1:
        return np.array([window], dtype=np.int64)
    out = []
    for d in range(n_depth):
        x = Fraction((window - 1) * d, n_depth - 1) + Fraction(1, 2)
        out.append(1 + (x.numerator // x.denominator))
    return np.array(out, dtype=np.int64)


def default_weights(n_depth: int, window: int) -> np.ndarray:
    """W[d][a] = 1 for a < n_d, else 0 (float64, shape n_depth x window)."""
    n = default_frames(n_depth, window)
    return (np.arange(window)[None, :] < n[:, None]).astype(np.float64)


def dda(frames: Sequence[np.ndarray], weights: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Average of the given frames (oldest first, at most N_w = weights.shape[1] of them,
    depth on the last axis).  Returns (average volume, max over depth)."""
    W = np.asarray(weights, dtype=np.float64)
    m = len(frames)
    assert 1 <= m <= W.shape[1]
    num = np.zeros(np.shape(frames[-1]), dtype=np.float64)
    den = np.zeros(W.shape[0], dtype=np.float64)
    for a in range(m):                       # a frames back from the newest
        num += W[:, a] * np.asarray(frames[m - 1 - a], dtype=np.float64)
        den += W[:, a]
    avg = num / den
    return avg, avg.max(axis=-1)


def dda_sequence(frames: Sequence[np.ndarray], weights: np.ndarray) -> List[Tuple[np.ndarray, np.ndarray]]:
    """The average and image after each frame of a stream."""
    window = np.shape(weights)[1]
    return [dda(frames[max(0, i - window + 1):i + 1], weights) for i in range(len(frames))]
