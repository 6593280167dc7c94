"""The discrete Fourier transform as its definition (test infrastructure only).

X[k] = sum_n x[n] exp(-2 pi i n k / M), applied along one axis as a matrix
product.  The phase index n*k is reduced modulo M in exact integer arithmetic
before the exponential, so every twiddle is exp(-2 pi i m / M) with 0 <= m < M.
The inverse uses the conjugate matrix and divides by M (ifft semantics, as in
the f-k pipeline of Algorithm 1).  No fast algorithm, no blocking.
"""
from __future__ import annotations

import numpy as np


def dft_matrix(m: int, inverse: bool = False) -> np.ndarray:
    n = np.arange(m, dtype=np.int64)
    nk = np.outer(n, n) % m
    sign = 1.0 if inverse else -1.0
    return np.exp(sign * 2j * np.pi * nk / m)


def dft(x: np.ndarray, axis: int, inverse: bool = False) -> np.ndarray:
    """Unnormalised forward DFT (or 1/M-normalised inverse) along ``axis``."""
    x = np.asarray(x, dtype=np.complex128)
    shape = x.shape
    axis = axis % x.ndim
    m = shape[axis]
    f = dft_matrix(m, inverse)  # symmetric: F[n, k] = F[k, n]
    a = int(np.prod(shape[:axis], dtype=np.int64))
    b = int(np.prod(shape[axis + 1:], dtype=np.int64))
    xv = np.ascontiguousarray(x).reshape(a, m, b)
    y = np.empty_like(xv)
    if b == 1:
        y[:, :, 0] = xv[:, :, 0] @ f
    else:
        for i in range(a):          # X[k, :] = sum_n F[k, n] x[n, :]
            y[i] = f @ xv[i]
    if inverse:
        y /= m
    return y.reshape(shape)


def dftn(x: np.ndarray, axes, inverse: bool = False) -> np.ndarray:
    for ax in axes:
        x = dft(x, ax, inverse)
    return x
