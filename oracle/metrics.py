"""Error measures used to compare a result with the oracle (test infrastructure only)."""
from __future__ import annotations

import numpy as np


def _as_f64(a) -> np.ndarray:
    a = np.asarray(a)
    return a.astype(np.complex128) if np.iscomplexobj(a) else a.astype(np.float64)


def rel_l2(x, ref) -> float:
    """||x - ref|| / ||ref|| (complex values compared as complex); an all-zero reference is
    only matched by an all-zero x."""
    x = _as_f64(x)
    ref = _as_f64(ref)
    n = np.linalg.norm(ref.ravel())
    d = np.linalg.norm((x - ref).ravel())
    if n == 0:
        return 0.0 if d == 0 else float("inf")
    return float(d / n)


def max_rel(x, ref) -> float:
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    m = np.abs(ref).max()
    return float(np.abs(x - ref).max() / (m if m > 0 else 1.0))


def psnr_maxnorm(img, ref_img) -> float:
    a = np.asarray(img, dtype=np.float64)
    b = np.asarray(ref_img, dtype=np.float64)
    a = a / (a.max() if a.max() > 0 else 1.0)
    b = b / (b.max() if b.max() > 0 else 1.0)
    mse = np.mean((a - b) ** 2)
    return float("inf") if mse == 0 else float(10.0 * np.log10(1.0 / mse))


def argmax_index(v):
    return np.unravel_index(int(np.argmax(v)), np.shape(v))


def argmax_distance(x, ref) -> float:
    a = np.array(argmax_index(x), dtype=np.float64)
    b = np.array(argmax_index(ref), dtype=np.float64)
    return float(np.abs(a - b).max())
