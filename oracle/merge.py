"""Coherence-weighted temporal merging of complex reconstructions (Section 4.4, Eq. 8-9)
-- FP64, test infrastructure only.

Over the window of the most recent frames f_j (complex volumes of one operator),

    C = |sum_j f_j| / (eps + sum_j |f_j|),      merged = C * |sum_j f_j| / W,

with W the number of frames in the window.  Eq. 9 divides by N_w, the window length; the
paper does not say what happens before N_w frames exist.  Reading used here: W is the
number of frames present (min(i + 1, N_w) after the i-th frame).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def coherence_merge(frames: Sequence[np.ndarray], eps: float) -> Tuple[np.ndarray, np.ndarray]:
    """Eq. 8-9 over the given frames (oldest first).  Returns (merged, C)."""
    fs = [np.asarray(f, dtype=np.complex128) for f in frames]
    S = np.sum(fs, axis=0)
    A = np.sum([np.abs(f) for f in fs], axis=0)
    C = np.abs(S) / (eps + A)
    return C * np.abs(S) / len(fs), C


def merge_sequence(frames: Sequence[np.ndarray], window: int, eps: float) -> List[Tuple[np.ndarray, np.ndarray]]:
    """The merged frame and coherence after each frame of a stream."""
    out = []
    for i in range(len(frames)):
        out.append(coherence_merge(frames[max(0, i - window + 1):i + 1], eps))
    return out
