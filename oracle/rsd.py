"""Phasor DFT and radial RSD propagation, FP64 (test infrastructure only).

The radial RSD is an approximation (the paper enforces radial symmetry and
truncates the ring integral), so it is written as the paper's steps in the
paper's order: Section 4.3 Eq. 4-7 (ring decomposition, ring basis
B = 2 pi r J0(2 pi r rho), stored kernel K_r(rho, f, d) by trapezoid quadrature,
propagation sum), the supplementary sampling rules (r_max, rho_max, N_r, N_rho,
cutoff, bin coordinate, smoothstep taper), the runtime lookup of Listing 3
(clamped interpolation indices) and Algorithm 4 (pad top-left, batched 2D DFT,
accumulate over frequencies, batched inverse 2D DFT, magnitude, max over depth).

The exact RSD of the phase-only kernel k(x, d, f) = exp(i kappa (sigma_s
sqrt(|x|^2 + d^2) + sigma_t d + Delta)) is also given twice, as a direct
spatial sum and as a dense-kernel FFT convolution (Algorithm 3's operator);
they pin the radial form.  J0 comes from scipy.special.j0.

Readings taken where the paper is silent: kappa_f = 2 pi k_f / (nt c dt); forward DFT
exp(-i), kernel exp(+i); Delta = 0; output |I|; the amplitude falloff is
dropped as the paper does; ceilings of quantities that are integers in exact
arithmetic use a 1e-9 relative tolerance; a stored radial sample is zero when
its bin coordinate exceeds the cutoff coordinate by more than 1e-9 bins.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import j0 as bessel_j0

from .dft import dft

C_LIGHT = 299_792_458.0
TAPER_BINS = 8.0


def phasor(tau: np.ndarray, freq_bins) -> np.ndarray:
    """P[f][y][x] = sum_t tau[y][x][t] exp(-2 pi i k_f t / nt) (binner-side DFT)."""
    ny, nx, nt = tau.shape
    k = np.asarray(freq_bins, dtype=np.int64)
    t = np.arange(nt, dtype=np.int64)
    E = np.exp(-2j * np.pi * ((k[:, None] * t[None, :]) % nt) / nt)  # (Nf, nt)
    P = np.asarray(tau, dtype=np.float64).reshape(-1, nt) @ E.T          # (npix, Nf)
    return P.T.reshape(len(k), ny, nx)


def phasor_from_events(pixel, t_ps, nx: int, ny: int, nt: int, bin_ps: int, t0_ps: int, freq_bins):
    """Phasors straight from photon records (Section 4.1, phasor binning): each valid
    event in bin b of its pixel adds exp(-2 pi i k_f b / nt) to P[f][pixel].  In exact
    arithmetic this is the binner-side DFT of the histogram, which is how it is written
    here (the histogram of the binning oracle, then `phasor`)."""
    from .binning import bin_events
    hist, dropped = bin_events(pixel, t_ps, nx, ny, nt, bin_ps, t0_ps)
    return phasor(hist.astype(np.float64), freq_bins), dropped


def wavenumbers(freq_bins, nt: int, c_dt: float) -> np.ndarray:
    """kappa_f = 2 pi k_f / (nt c dt) in rad/m (round-trip path units)."""
    return 2.0 * np.pi * np.asarray(freq_bins, dtype=np.float64) / (nt * c_dt)


def _ceil_tol(x: float) -> int:
    return int(math.ceil(x - 1e-9 * abs(x)))


def _pow2_at_least(n: int) -> int:
    return 1 << max(0, (int(n) - 1).bit_length())


@dataclasses.dataclass
class RadialGeometry:
    r_max: float
    rho_max: float
    lam_min: float
    n_r_min: int
    n_r: int
    dr: float
    n_rho_min: int
    n_rho: int
    f_s: float
    rho_cut: float
    rho_cut_bin: float
    cut_idx: int
    last_base: int


def radial_geometry(Mx: int, My: int, dx: float, dy: float, lam_min: float,
                    sigma_s: int) -> RadialGeometry:
    """Supplementary sampling rules: aperture radius, radial Nyquist limit, ring and
    radius counts (powers of two, N_r floored at 2), ring sampling rate and cutoff."""
    r_max = math.sqrt((0.5 * Mx * dx) ** 2 + (0.5 * My * dy) ** 2)
    rho_max = math.sqrt((0.5 / dx) ** 2 + (0.5 / dy) ** 2)
    n_r_min = _ceil_tol(2.0 * sigma_s * r_max / lam_min) + 1
    n_r = max(2, _pow2_at_least(n_r_min))
    dr = r_max / (n_r - 1)
    n_rho_min = _ceil_tol(2.0 * r_max * rho_max) + 1
    n_rho = _pow2_at_least(n_rho_min)
    f_s = (n_r - 1) / r_max
    rho_cut = min(rho_max, 0.5 * f_s)
    rho_cut_bin = rho_cut * (n_rho - 1) / rho_max
    cut_idx = min(n_rho - 1, int(math.ceil(rho_cut_bin)))
    last_base = max(0, min(cut_idx - 1, n_rho - 2))
    return RadialGeometry(r_max, rho_max, lam_min, n_r_min, n_r, dr, n_rho_min, n_rho,
                          f_s, rho_cut, rho_cut_bin, cut_idx, last_base)


def ring_basis(r: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """Eq. 5: B(r, rho) = 2 pi r J0(2 pi r rho); returns [rho][r]."""
    return 2.0 * np.pi * r[None, :] * bessel_j0(2.0 * np.pi * r[None, :] * rho[:, None])


def trapezoid_weights(n_r: int, dr: float) -> np.ndarray:
    q = np.full(n_r, dr)
    q[0] = q[-1] = 0.5 * dr
    return q


def radial_kernel(geom: RadialGeometry, kappa: np.ndarray, depths: np.ndarray,
                  sigma_s: int, sigma_t: int, delta: float) -> np.ndarray:
    """Eq. 4-6: K_r[rho][f][d] = exp(i kappa (sigma_t d + Delta)) *
    sum_j q_j exp(i sigma_s kappa sqrt(r_j^2 + d^2)) B(r_j, rho), zero beyond the cutoff."""
    r = np.arange(geom.n_r) * geom.dr
    q = trapezoid_weights(geom.n_r, geom.dr)
    rho = np.arange(geom.n_rho) * geom.rho_max / (geom.n_rho - 1)
    B = ring_basis(r, rho)                                                     # (Nrho, Nr)
    A = np.exp(1j * sigma_s * kappa[:, None, None]
               * np.sqrt(r[None, None, :] ** 2 + depths[None, :, None] ** 2))  # (Nf, Nd, Nr)
    K = (A * q[None, None, :]) @ B.T                                           # (Nf, Nd, Nrho)
    K = K * np.exp(1j * kappa[:, None] * (sigma_t * depths[None, :] + delta))[:, :, None]
    keep = np.arange(geom.n_rho) <= geom.rho_cut_bin + 1e-9
    K[:, :, ~keep] = 0.0
    return np.ascontiguousarray(K.transpose(2, 0, 1))                          # [rho][f][d]


def signed_index(m: int) -> np.ndarray:
    k = np.arange(m)
    return np.where(k < m // 2, k, k - m)


def radius_map(My: int, Mx: int, dx: float, dy: float, geom: RadialGeometry) -> np.ndarray:
    """Pixel-to-radius map in bin units: |(v'/(Mx dx), u'/(My dy))| (N_rho - 1) / rho_max."""
    u = signed_index(My)[:, None] / (My * dy)
    v = signed_index(Mx)[None, :] / (Mx * dx)
    return np.sqrt(u ** 2 + v ** 2) * (geom.n_rho - 1) / geom.rho_max


def taper(rho_t: np.ndarray, rho_cut_bin: float) -> np.ndarray:
    """Smoothstep over the last 8 bins below the cutoff (1 below, 0 at and above)."""
    t = (rho_cut_bin - rho_t) / TAPER_BINS
    return np.where(rho_t <= rho_cut_bin - TAPER_BINS, 1.0,
                    np.where(rho_t < rho_cut_bin, t * t * (3.0 - 2.0 * t), 0.0))


def interp_indices(rho_t: np.ndarray, geom: RadialGeometry):
    """Listing 3 lookup: i0 = clamp(floor, 0, lastBase), i1 = min(i0 + 1, cutIdx), alpha."""
    i0 = np.clip(np.floor(rho_t).astype(np.int64), 0, geom.last_base)
    i1 = np.minimum(i0 + 1, geom.cut_idx)
    alpha = rho_t - i0
    return i0, i1, alpha


@dataclasses.dataclass
class RsdSetup:
    geom: RadialGeometry
    kappa: np.ndarray
    depths: np.ndarray
    K: np.ndarray          # [rho][f][d]
    rho_t: np.ndarray      # [My][Mx]


def setup(ny, nx, nt, dx, dy, c_dt, pad, freq_bins, depths, sigma_s=2, sigma_t=0,
          delta=0.0) -> RsdSetup:
    """Plan-time quantities (precomputed once in the paper)."""
    My, Mx = pad * ny, pad * nx
    kappa = wavenumbers(freq_bins, nt, c_dt)
    lam_min = 2.0 * np.pi / kappa.max()
    geom = radial_geometry(Mx, My, dx, dy, lam_min, sigma_s)
    depths = np.asarray(depths, dtype=np.float64)
    K = radial_kernel(geom, kappa, depths, sigma_s, sigma_t, delta)
    rho_t = radius_map(My, Mx, dx, dy, geom)
    return RsdSetup(geom, kappa, depths, K, rho_t)


def propagate(Ph: np.ndarray, w: np.ndarray, st: RsdSetup, chunk: int = 2048) -> np.ndarray:
    """Algorithm 4 loop: C(u,v,d) = sum_f w_f Ph(u,v,f) a(rho) lerp(K_r(., f, d), rho)."""
    Nf, My, Mx = Ph.shape
    Nd = st.depths.size
    rho_t = st.rho_t.ravel()
    a = taper(rho_t, st.geom.rho_cut_bin)
    i0, i1, alpha = interp_indices(rho_t, st.geom)
    Pw = (Ph.reshape(Nf, -1) * np.asarray(w)[:, None]).T               # (npix, Nf)
    C = np.zeros((My * Mx, Nd), dtype=np.complex128)
    for s in range(0, My * Mx, chunk):
        e = min(My * Mx, s + chunk)
        h = (1.0 - alpha[s:e, None, None]) * st.K[i0[s:e]] + alpha[s:e, None, None] * st.K[i1[s:e]]
        h = a[s:e, None, None] * h                                     # (n, Nf, Nd)
        c = np.einsum("pf,pfd->pd", Pw[s:e], h)
        C[s:e] = np.where(a[s:e, None] > 0, c, 0.0)
    return C.T.reshape(Nd, My, Mx)


def rsd(tau: np.ndarray, dx: float, dy: float, bin_ps: float, pad: int, freq_bins, w,
        depths, sigma_s: int = 2, sigma_t: int = 0, delta: float = 0.0, return_complex=False):
    """Radial RSD of a transient tau[ny][nx][nt] (Algorithm 4).

    Returns (vol[Nd][ny][nx] = |I|, img = max over depth)."""
    ny, nx, nt = tau.shape
    My, Mx = pad * ny, pad * nx
    c_dt = C_LIGHT * bin_ps * 1e-12
    P = phasor(tau, freq_bins)                                   # step 1
    Pt = np.zeros((P.shape[0], My, Mx), dtype=np.complex128)    # step 2: pad top-left
    Pt[:, :ny, :nx] = P
    Ph = dft(dft(Pt, 1), 2)
    st = setup(ny, nx, nt, dx, dy, c_dt, pad, freq_bins, depths, sigma_s, sigma_t, delta)
    C = propagate(Ph, np.asarray(w, dtype=np.complex128), st)   # steps 7-9
    I = dft(dft(C, 1, inverse=True), 2, inverse=True)           # step 10
    Ic = I[:, :ny, :nx]
    vol = np.abs(Ic)                                            # step 11
    img = vol.max(axis=0)
    if return_complex:
        return vol, img, Ic
    return vol, img


# ---------------------------------------------------------------------------
# exact RSD of the phase-only kernel (pins for the radial approximation)
# ---------------------------------------------------------------------------


def rsd_direct(P: np.ndarray, dx: float, dy: float, kappa, w, depths, sigma_s=2,
               sigma_t=0, delta=0.0) -> np.ndarray:
    """I(x_v, d) = sum_f w_f sum_{x_s} P(x_s, f) k(x_s - x_v, d, f), complex [Nd][ny][nx]."""
    Nf, ny, nx = P.shape
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    yy = yy.ravel()
    xx = xx.ravel()
    ddy = (yy[None, :] - yy[:, None]) * dy   # [v][s]
    ddx = (xx[None, :] - xx[:, None]) * dx
    rho2 = ddx ** 2 + ddy ** 2
    out = np.zeros((len(depths), ny * nx), dtype=np.complex128)
    Pf = P.reshape(Nf, -1)
    for j, d in enumerate(depths):
        R = np.sqrt(rho2 + d * d)
        for f in range(Nf):
            kmat = np.exp(1j * kappa[f] * (sigma_s * R + sigma_t * d + delta))
            out[j] += w[f] * (kmat @ Pf[f])
    return out.reshape(len(depths), ny, nx)


def rsd_dense_fft(P: np.ndarray, dx: float, dy: float, kappa, w, depths, sigma_s=2,
                  sigma_t=0, delta=0.0) -> np.ndarray:
    """Dense-kernel form with padding 2: K = DFT2 of k sampled on the signed padded
    grid, C = sum_f w_f DFT2(pad(P_f)) K_fd, I = IDFT2(C) cropped; complex [Nd][ny][nx]."""
    Nf, ny, nx = P.shape
    My, Mx = 2 * ny, 2 * nx
    Pt = np.zeros((Nf, My, Mx), dtype=np.complex128)
    Pt[:, :ny, :nx] = P
    Ph = dft(dft(Pt, 1), 2)
    u = signed_index(My)[:, None] * dy
    v = signed_index(Mx)[None, :] * dx
    rho2 = u ** 2 + v ** 2
    out = np.zeros((len(depths), ny, nx), dtype=np.complex128)
    for j, d in enumerate(depths):
        C = np.zeros((My, Mx), dtype=np.complex128)
        R = np.sqrt(rho2 + d * d)
        for f in range(Nf):
            k = np.exp(1j * kappa[f] * (sigma_s * R + sigma_t * d + delta))
            C += w[f] * Ph[f] * dft(dft(k, 0), 1)
        out[j] = dft(dft(C, 0, inverse=True), 1, inverse=True)[:ny, :nx]
    return out
