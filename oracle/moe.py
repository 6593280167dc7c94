"""Mixture of experts of the f-k and RSD reconstructions (Section 4.4, Eq. 10) -- FP64,
test infrastructure only.

Both branches are reduced to their max-over-depth images (the f-k branch ends in a
depth maximum of |Psi|^2, the RSD branch reduces its |I| volume to an image).  The
product of experts is

    f = f_fk * (f_rsd + eps)^beta,

with beta = 0.3 and eps a small constant; beta = 1 is the plain product.  The paper
normalises the mixed result; it does not say how the branch images are scaled before
mixing.  Reading used here: each branch image is divided by its maximum (so eps is
relative to the RSD image's peak), and the mixed image is divided by its maximum.
An all-zero image stays zero.
"""
from __future__ import annotations

import numpy as np

from . import fk as ofk
from . import rsd as orsd

BETA = 0.3
EPS = 1e-6


def _maxnorm(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    m = x.max() if x.size else 0.0
    return x / m if m > 0 else np.zeros_like(x)


def mix(img_fk: np.ndarray, img_rsd: np.ndarray, beta: float = BETA, eps: float = EPS) -> np.ndarray:
    """Eq. 10 on max-normalised branch images, max-normalised result."""
    a = _maxnorm(img_fk)
    b = _maxnorm(img_rsd)
    return _maxnorm(a * np.power(b + eps, beta))


def moe(tau: np.ndarray, wall_w: float, wall_h: float, bin_ps: float, pad: int, freq_bins, w,
        depths, beta: float = BETA, eps: float = EPS, sigma_s: int = 2, sigma_t: int = 0,
        delta: float = 0.0):
    """Both branches on the same transient (each written as its own oracle), then Eq. 10.

    Returns (mixed image, f-k image, RSD image)."""
    ny, nx, _ = tau.shape
    _, img_fk = ofk.fk(tau, wall_w, wall_h, bin_ps, pad)
    _, img_rsd = orsd.rsd(tau, wall_w / nx, wall_h / ny, bin_ps, pad, freq_bins, w, depths,
                          sigma_s, sigma_t, delta)
    return mix(img_fk, img_rsd, beta, eps), img_fk, img_rsd
