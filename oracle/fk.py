"""f-k migration, FP64 (test infrastructure only).

Follows the f-k pipeline as the paper states it: Section 3.1 (Eq. 1-2: Stolt
interpolation migrates the wall measurement to t = 0, the volume is |Psi|^2),
Section 4.2 (scaling fused with zero padding, 3D FFT, on-the-fly Stolt with
the |fz|/sqrt Jacobian, active half only, inverse 3D FFT) and Algorithms 1-2 of
the supplementary material.  Readings taken where the paper is silent:
  * scaling by the normalised time index t/(nt-1), no square root;
  * the fftshift/ifftshift pair of Algorithm 1 is read as signed-frequency
    indexing, with no data movement;
  * Stolt constants per axis, s_x = c dt / (2 dx), s_y = c dt / (2 dy), which
    equal Algorithm 1's s = Nx d_max / (4 Nz apt/2) with d_max = nt c dt and
    apt = nx dx, independent of padding;
  * linear interpolation along the frequency axis only, zero outside the grid
    (interpn fill 0), the last sample taken at the top edge itself;
  * mask Z > 0 (the signed -M/2 plane counts as negative), Jacobian Z / Z';
  * forward DFT unnormalised, inverse normalised by 1/(Mx My Mt).
"""
from __future__ import annotations

import numpy as np

from .dft import dft

C_LIGHT = 299_792_458.0


def stolt_constants(dx: float, dy: float, bin_ps: float):
    """s_x, s_y of Algorithm 1 (s = Nx d_max / (4 Nz apt/2)) per axis."""
    c_dt = C_LIGHT * bin_ps * 1e-12
    return c_dt / (2.0 * dx), c_dt / (2.0 * dy)


def signed_index(m: int) -> np.ndarray:
    """Signed frequency of DFT bin k: k for k < m/2, k - m otherwise."""
    k = np.arange(m)
    return np.where(k < m // 2, k, k - m)


def scale_and_pad(tau: np.ndarray, pad: int) -> np.ndarray:
    """Algorithm 1, first block: Psi * linspace(0, 1, Nz) along t, then zero padding."""
    ny, nx, nt = tau.shape
    t_norm = np.arange(nt, dtype=np.float64) / (nt - 1)
    g = np.asarray(tau, dtype=np.float64) * t_norm[None, None, :]
    G = np.zeros((pad * ny, pad * nx, pad * nt), dtype=np.complex128)
    G[:ny, :nx, :nt] = g
    return G


def forward(G: np.ndarray) -> np.ndarray:
    """Unnormalised 3D DFT (t, then x, then y -- order is immaterial)."""
    return dft(dft(dft(G, 2), 1), 0)


def stolt(S: np.ndarray, sx: float, sy: float) -> np.ndarray:
    """Stolt remap with Jacobian (Algorithm 1 remap block; Listing 2 semantics).

    out(ky, kx, kz) = [Z > 0] * (Z / Z') * S(ky, kx, Z') with
    Z' = sqrt(sx^2 X^2 + sy^2 Y^2 + Z^2) and X, Y, Z the signed frequencies
    normalised to [-1, 1).  S(ky, kx, .) is sampled at Z' by linear
    interpolation over the frequency samples of that column, zero beyond the
    last sample.
    """
    My, Mx, Mt = S.shape
    half = Mt // 2
    X = signed_index(Mx) / (Mx / 2)
    Y = signed_index(My) / (My / 2)
    Z = signed_index(Mt) / (Mt / 2)
    out = np.zeros_like(S)
    for iy in range(My):
        Zp = np.sqrt(sx ** 2 * X[:, None] ** 2 + sy ** 2 * Y[iy] ** 2 + Z[None, :] ** 2)
        q = Zp * half                    # fractional signed index along the column, >= 0
        inside = q <= half - 1
        i0 = np.minimum(np.floor(q), half - 1).astype(np.int64)
        fr = q - i0
        i1 = np.minimum(i0 + 1, half - 1)
        col = S[iy]                      # (Mx, Mt); signed index k >= 0 is array index k
        v0 = np.take_along_axis(col, i0, axis=1)
        v1 = np.take_along_axis(col, i1, axis=1)
        val = np.where(inside, (1.0 - fr) * v0 + fr * v1, 0.0)
        jac = np.where(Z[None, :] > 0, np.abs(Z[None, :]) / np.maximum(Zp, 1e-6), 0.0)
        out[iy] = val * jac
    return out


def inverse(S: np.ndarray) -> np.ndarray:
    """Normalised inverse 3D DFT."""
    return dft(dft(dft(S, 0, inverse=True), 1, inverse=True), 2, inverse=True)


def fk(tau: np.ndarray, wall_w: float, wall_h: float, bin_ps: float, pad: int = 2,
       s_override=None, return_psi: bool = False):
    """Full f-k migration of a confocal transient tau[ny][nx][nt].

    Returns (vol[ny][nx][nt] = |Psi|^2 on the unpadded grid, img = max over z).
    """
    ny, nx, nt = tau.shape
    dx, dy = wall_w / nx, wall_h / ny
    sx, sy = stolt_constants(dx, dy, bin_ps) if s_override is None else s_override
    G = scale_and_pad(tau, pad)
    S = forward(G)
    del G
    out = stolt(S, sx, sy)
    del S
    psi = inverse(out)[:ny, :nx, :nt]
    vol = np.abs(psi) ** 2
    img = vol.max(axis=2)
    if return_psi:
        return vol, img, psi
    return vol, img
