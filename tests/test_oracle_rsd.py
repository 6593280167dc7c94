"""Pins of the phasor DFT and radial RSD oracle."""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import j0

import scenes
from oracle import rsd as orsd
from oracle.metrics import argmax_index, psnr_maxnorm, rel_l2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_worked_example_sampling_counts():
    g = json.load(open(os.path.join(GOLDEN, "rsd_worked_example.json")))
    inp, exp = g["inputs"], g["expected"]
    dx = math.sqrt(2.0) / (2.0 * inp["rho_max_per_m"])
    n = inp["n"] * inp["pad"]
    geom = orsd.radial_geometry(n, n, dx, dx, inp["lambda_min_m"], inp["sigma_s"])
    assert geom.n_r_min == exp["n_r_min"] and geom.n_r == exp["n_r"]
    assert geom.n_rho_min == exp["n_rho_min"] and geom.n_rho == exp["n_rho"]
    assert round(geom.rho_max, 2) == exp["rho_max_per_m"]
    assert round(geom.rho_cut, 2) == exp["rho_cutoff_per_m"]


@pytest.mark.parametrize("m,expect", [(64, 128), (128, 256), (256, 512), (512, 1024)])
def test_square_grid_identity(m, expect):
    # 2 r_max rho_max = M exactly on square grids, so N_rho = next power of two of M + 1
    for dx in (1.0 / 32, 0.0123, 0.5):
        geom = orsd.radial_geometry(m, m, dx, dx, 0.05, 2)
        assert geom.n_rho == expect and geom.n_rho_min == m + 1


def test_bessel_values():
    assert j0(0.0) == 1.0
    assert abs(j0(2.404825557695773)) < 1e-15 and abs(j0(5.520078110286311)) < 1e-15


def test_ring_quadrature_reproduces_gaussian_hankel_pair():
    # The 2D Fourier transform of exp(-pi r^2) is exp(-pi rho^2); through the ring basis
    # and trapezoid weights: sum_j q_j exp(-pi r_j^2) B(r_j, rho) ~= exp(-pi rho^2).
    # The trapezoid error must be the Euler-Maclaurin leading term -dr^2/12 f'(0) with
    # f'(0) = 2 pi (f(r) = 2 pi r J0(2 pi r rho) exp(-pi r^2), f'(r_max) ~ 0), to 1%.
    for lam in (0.05, 0.01):
        geom = orsd.radial_geometry(64, 64, 0.125, 0.125, lam, 2)  # r_max = 4 sqrt(2)
        r = np.arange(geom.n_r) * geom.dr
        q = orsd.trapezoid_weights(geom.n_r, geom.dr)
        rho = np.linspace(0.0, 2.0, 41)
        got = orsd.ring_basis(r, rho) @ (q * np.exp(-np.pi * r ** 2))
        em = -geom.dr ** 2 / 12.0 * 2.0 * np.pi
        err = got - np.exp(-np.pi * rho ** 2)
        assert np.max(np.abs(err - em)) < 0.01 * abs(em)


def test_phasor_matches_library_fft():
    rng = np.random.default_rng(1)
    tau = rng.poisson(4.0, size=(5, 6, 64)).astype(np.float64)
    k = np.array([1, 3, 7, 31])
    P = orsd.phasor(tau, k)
    ref = np.fft.rfft(tau, axis=2)[..., k]
    assert np.max(np.abs(P - np.moveaxis(ref, 2, 0))) < 1e-11 * np.abs(ref).max()


def test_taper_shape():
    rc = 100.3
    x = np.linspace(80, 110, 3001)
    a = orsd.taper(x, rc)
    assert np.all(a[x <= rc - 8] == 1.0) and np.all(a[x >= rc] == 0.0)
    assert np.all(np.diff(a) <= 0.0)
    assert abs(orsd.taper(np.array([rc - 4.0]), rc)[0] - 0.5) < 1e-12


def _small_case(n=16, nd=12, pos=(0.1, -0.15, 0.5)):
    cfg = scenes.small_config(n, n, 256, bin_ps=32, depth_range=(0.3, 0.8), n_depth=nd)
    tau = scenes.transient(cfg, noise=False, objects=[scenes.point_object(*pos)]).astype(np.float64)
    p = scenes.rsd_params(cfg)
    depths = p.depth0 + p.depth_step * np.arange(p.n_depth)
    return cfg, tau, p, depths


def test_dense_fft_equals_direct_sum():
    cfg, tau, p, depths = _small_case(12, 6)
    P = orsd.phasor(tau, p.freq_bins)
    kap = orsd.wavenumbers(p.freq_bins, cfg.nt, cfg.c_dt)
    Id = orsd.rsd_direct(P, cfg.dx, cfg.dy, kap, p.weights, depths)
    If = orsd.rsd_dense_fft(P, cfg.dx, cfg.dy, kap, p.weights, depths)
    assert rel_l2(If.real, Id.real) < 1e-12 and rel_l2(If.imag, Id.imag) < 1e-12


def test_radial_approximates_direct_sum():
    cfg, tau, p, depths = _small_case(24, 12)
    vol, img = orsd.rsd(tau, cfg.dx, cfg.dy, cfg.bin_ps, 2, p.freq_bins, p.weights, depths)
    P = orsd.phasor(tau, p.freq_bins)
    kap = orsd.wavenumbers(p.freq_bins, cfg.nt, cfg.c_dt)
    Id = np.abs(orsd.rsd_direct(P, cfg.dx, cfg.dy, kap, p.weights, depths))
    assert argmax_index(vol) == argmax_index(Id)
    assert rel_l2(vol / (cfg.dx * cfg.dy), Id) < 0.10
    assert psnr_maxnorm(img, Id.max(axis=0)) > 40.0


def test_radial_approximates_direct_sum_on_a_mixed_radix_grid():
    """A 20 x 18 scan of 240 bins (padded 40 x 36; factors 3, 5): the same agreement."""
    pos = (0.1, -0.15, 0.5)
    cfg = scenes.small_config(20, 18, 240, bin_ps=32, depth_range=(0.3, 0.8), n_depth=10)
    tau = scenes.transient(cfg, noise=False, objects=[scenes.point_object(*pos)]).astype(np.float64)
    p = scenes.rsd_params(cfg)
    depths = p.depth0 + p.depth_step * np.arange(p.n_depth)
    vol, img = orsd.rsd(tau, cfg.dx, cfg.dy, cfg.bin_ps, 2, p.freq_bins, p.weights, depths)
    P = orsd.phasor(tau, p.freq_bins)
    kap = orsd.wavenumbers(p.freq_bins, cfg.nt, cfg.c_dt)
    Id = np.abs(orsd.rsd_direct(P, cfg.dx, cfg.dy, kap, p.weights, depths))
    assert argmax_index(vol) == argmax_index(Id)
    assert rel_l2(vol / (cfg.dx * cfg.dy), Id) < 0.10
    assert psnr_maxnorm(img, Id.max(axis=0)) > 40.0


def test_point_reflector_peak():
    pos = (0.1, -0.15, 0.5)
    cfg, tau, p, depths = _small_case(16, 24, pos)
    vol, img = orsd.rsd(tau, cfg.dx, cfg.dy, cfg.bin_ps, 2, p.freq_bins, p.weights, depths)
    d, y, x = argmax_index(vol)
    assert abs(x - ((pos[0] + 0.5) / cfg.dx - 0.5)) <= 1
    assert abs(y - ((pos[1] + 0.5) / cfg.dy - 0.5)) <= 1
    assert abs(d - (pos[2] - depths[0]) / (depths[1] - depths[0])) <= 1


def test_linearity():
    cfg, tau, p, depths = _small_case(8, 5)
    v1, _ = orsd.rsd(tau, cfg.dx, cfg.dy, cfg.bin_ps, 2, p.freq_bins, p.weights, depths)
    v2, _ = orsd.rsd(-2.5 * tau, cfg.dx, cfg.dy, cfg.bin_ps, 2, p.freq_bins, p.weights, depths)
    assert np.max(np.abs(v2 - 2.5 * v1)) < 1e-11 * v2.max()


def test_propagation_scalar_loop_8x8():
    cfg, tau, p, depths = _small_case(8, 4)
    st = orsd.setup(8, 8, 256, cfg.dx, cfg.dy, cfg.c_dt, 2, p.freq_bins, depths)
    rng = np.random.default_rng(9)
    Nf = len(p.freq_bins)
    Ph = rng.normal(size=(Nf, 16, 16)) + 1j * rng.normal(size=(Nf, 16, 16))
    C = orsd.propagate(Ph, p.weights, st)
    ref = np.zeros_like(C)
    g = st.geom
    for u in range(16):
        for v in range(16):
            rt = st.rho_t[u, v]
            t = (g.rho_cut_bin - rt) / 8.0
            a = 1.0 if rt <= g.rho_cut_bin - 8 else (t * t * (3 - 2 * t) if rt < g.rho_cut_bin else 0.0)
            if a <= 0:
                continue
            i0 = min(max(int(math.floor(rt)), 0), g.last_base)
            i1 = min(i0 + 1, g.cut_idx)
            al = rt - i0
            for d in range(len(depths)):
                for f in range(Nf):
                    h = a * ((1 - al) * st.K[i0, f, d] + al * st.K[i1, f, d])
                    ref[d, u, v] += p.weights[f] * Ph[f, u, v] * h
    assert np.max(np.abs(C - ref)) < 1e-12 * np.abs(ref).max()


def test_phasor_from_events_is_the_per_event_sum():
    """Brute force on a tiny input: the sum over events of their unit phasors."""
    import scenes
    nx, ny, nt, bin_ps = 3, 2, 16, 10
    ev = scenes.random_events(300, nx, ny, nt, bin_ps, seed=11, invalid_frac=0.1)
    bins = [1, 3, 7]
    P, dropped = orsd.phasor_from_events(ev["pixel"], ev["t_ps"], nx, ny, nt, bin_ps, 0, bins)
    ref = np.zeros((len(bins), ny * nx), dtype=np.complex128)
    nd = 0
    for pix, t in zip(ev["pixel"].tolist(), ev["t_ps"].tolist()):
        b = t // bin_ps
        if not (0 <= pix < nx * ny) or b >= nt:
            nd += 1
            continue
        for i, k in enumerate(bins):
            ref[i, pix] += complex(math.cos(2 * math.pi * k * b / nt), -math.sin(2 * math.pi * k * b / nt))
    assert nd == dropped
    np.testing.assert_allclose(P.reshape(len(bins), -1), ref, rtol=0, atol=1e-9)


def test_rel_l2_compares_complex_values_as_complex():
    a = np.array([1 + 1j, 2 - 1j])
    b = np.array([1 + 1j, 2 + 1j])
    assert rel_l2(a, b) == pytest.approx(2 / np.sqrt(7), rel=1e-15)


# ---------------------------------------------------------------------------
# the modality pair (sigma_s, sigma_t) and the calibration offset Delta of Eq. 4
# ---------------------------------------------------------------------------


def _rsd_complex(tau, cfg, p, depths, **kw):
    _, _, field = orsd.rsd(tau, cfg.dx, cfg.dy, cfg.bin_ps, 2, p.freq_bins, p.weights, depths,
                           return_complex=True, **kw)
    return field


@pytest.mark.parametrize("m", [3, 17])
def test_delta_is_an_optical_path_offset(m):
    """Eq. 4's factor exp(i kappa Delta) with Delta = m c dt multiplies phasor f by
    exp(2 pi i k_f m / nt), which by the DFT shift theorem is the phasor of the transient
    advanced by m bins: a calibration offset of the optical path is the same as removing
    m bins of extra path from the measurement.  A flipped sign (advance by -m) or a
    dropped Delta fails."""
    cfg, tau, p, depths = _small_case(8, 5)
    delta = m * cfg.c_dt
    got = _rsd_complex(tau, cfg, p, depths, delta=delta)
    ref = _rsd_complex(np.roll(tau, -m, axis=2), cfg, p, depths)
    assert rel_l2(got, ref) < 1e-12
    # planted mistakes in the oracle's inputs: the pin tells them apart
    assert rel_l2(_rsd_complex(tau, cfg, p, depths, delta=-delta), ref) > 1e-2
    assert rel_l2(_rsd_complex(tau, cfg, p, depths), ref) > 1e-2


def test_sigma_t_is_a_depth_dependent_path_offset():
    """With sigma_t = 1, Eq. 4 adds kappa d to the phase: at a depth on the bin grid,
    d = j c dt, depth plane j equals the sigma_t = 0 plane of the transient advanced by j
    bins (shift theorem), plane by plane."""
    cfg, tau, p, _ = _small_case(8, 5)
    js = [20, 45, 70]
    depths = np.array([j * cfg.c_dt for j in js])
    got = _rsd_complex(tau, cfg, p, depths, sigma_s=1, sigma_t=1)
    for i, j in enumerate(js):
        ref = _rsd_complex(np.roll(tau, -j, axis=2), cfg, p, depths[i:i + 1], sigma_s=1, sigma_t=0)
        assert rel_l2(got[i], ref[0]) < 1e-12
        # sigma_t dropped or of the wrong sign does not match
        wrong = _rsd_complex(np.roll(tau, j, axis=2), cfg, p, depths[i:i + 1], sigma_s=1, sigma_t=0)
        assert rel_l2(got[i], wrong[0]) > 1e-2


def _non_confocal_point(cfg, pos):
    """Noise-free transient of a point reflector lit from the wall point beneath it: the
    illumination leg is z0, the return leg |p - x_s|, so a photon arrives at
    (z0 + |p - x_s|) / c, with 1/|p - x_s|^2 falloff and a Gaussian pulse of 1 bin."""
    xs, ys = scenes.scan_positions(cfg)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    R = np.sqrt((X - pos[0]) ** 2 + (Y - pos[1]) ** 2 + pos[2] ** 2)
    tb = (pos[2] + R) / cfg.c_dt
    t = np.arange(cfg.nt)
    return np.exp(-0.5 * (t[None, None, :] - tb[:, :, None]) ** 2) / R[:, :, None] ** 2


def test_non_confocal_point_reflector_focus():
    """Modality (1, 1) of Section 4.3: the reflector focuses at its position and at the
    depth plane nearest z0.  A dropped sigma_t (path R instead of R + d) or a flipped one
    (R - d) puts the peak at another depth; the confocal phase 2R agrees with R + z0 at
    the apex only, so its focus is far weaker than the matched kernel's."""
    pos = (0.12, -0.1, 0.45)
    cfg = scenes.small_config(16, 16, 256, bin_ps=32, depth_range=(0.3, 0.8), n_depth=24)
    tau = _non_confocal_point(cfg, pos)
    p = scenes.rsd_params(cfg)
    depths = p.depth0 + p.depth_step * np.arange(p.n_depth)

    def peak(**kw):
        vol, _ = orsd.rsd(tau, cfg.dx, cfg.dy, cfg.bin_ps, 2, p.freq_bins, p.weights, depths, **kw)
        return argmax_index(vol)

    d, y, x = peak(sigma_s=1, sigma_t=1)
    assert abs(x - ((pos[0] + 0.5) / cfg.dx - 0.5)) <= 1
    assert abs(y - ((pos[1] + 0.5) / cfg.dy - 0.5)) <= 1
    d_true = (pos[2] - depths[0]) / (depths[1] - depths[0])
    assert abs(d - d_true) <= 1
    for kw in ({"sigma_s": 1, "sigma_t": 0}, {"sigma_s": 1, "sigma_t": -1}):
        assert abs(peak(**kw)[0] - d_true) > 2

    def top(**kw):
        return orsd.rsd(tau, cfg.dx, cfg.dy, cfg.bin_ps, 2, p.freq_bins, p.weights, depths, **kw)[0].max()

    assert top(sigma_s=1, sigma_t=1) > 2.0 * top(sigma_s=2, sigma_t=0)
