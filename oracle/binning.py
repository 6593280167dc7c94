"""Photon-event binning (test infrastructure only).

Follows the photon binner of Section 4.1 (the GPU histogramming of raw photon
records into one time histogram per relay-wall point).  Definition used: an
event (pixel, t_ps) is valid iff 0 <= pixel < nx*ny, t_ps >= t0_ps and
b = floor((t_ps - t0_ps) / bin_ps) < nt; a valid event adds one to
hist[pixel][b] (pixel = y*nx + x, time contiguous), an invalid one adds one to
the dropped count.
"""
from __future__ import annotations

import numpy as np


def bin_events(pixel: np.ndarray, t_ps: np.ndarray, nx: int, ny: int, nt: int,
               bin_ps: int, t0_ps: int = 0):
    """Returns (hist[ny][nx][nt] as uint64, dropped)."""
    pixel = np.asarray(pixel).astype(np.int64)
    t = np.asarray(t_ps).astype(np.int64)
    ok = (pixel >= 0) & (pixel < nx * ny) & (t >= t0_ps)
    b = np.where(ok, (t - t0_ps) // bin_ps, 0)
    ok &= b < nt
    flat = pixel[ok] * nt + b[ok]
    hist = np.zeros(nx * ny * nt, dtype=np.uint64)
    # one increment per valid event, in event order
    np.add.at(hist, flat, np.uint64(1))
    dropped = int((~ok).sum())
    return hist.reshape(ny, nx, nt), dropped


def bin_events_loop(pixel, t_ps, nx, ny, nt, bin_ps, t0_ps=0):
    """The same definition as a pure-Python loop, for tiny inputs."""
    hist = [[[0] * nt for _ in range(nx)] for _ in range(ny)]
    dropped = 0
    for p, t in zip(pixel.tolist(), t_ps.tolist()):
        if p < 0 or p >= nx * ny or t < t0_ps:
            dropped += 1
            continue
        b = (t - t0_ps) // bin_ps
        if b >= nt:
            dropped += 1
            continue
        hist[p // nx][p % nx][b] += 1
    return np.array(hist, dtype=np.uint64), dropped
