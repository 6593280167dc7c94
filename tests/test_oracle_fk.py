"""Pins of the f-k oracle against the mathematics and physics (not against itself)."""
import math

import numpy as np
import pytest
from scipy.signal import hilbert
from scipy.special import erf

import scenes
from oracle import fk as ofk
from oracle.dft import dft, dftn
from oracle.metrics import argmax_index


def test_dft_parseval_and_round_trip():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(6, 10, 16)) + 1j * rng.normal(size=(6, 10, 16))
    X = dftn(x, (0, 1, 2))
    assert abs(np.sum(np.abs(X) ** 2) - x.size * np.sum(np.abs(x) ** 2)) < 1e-10 * np.sum(np.abs(X) ** 2)
    back = dftn(X, (0, 1, 2), inverse=True)
    assert np.max(np.abs(back - x)) < 1e-12


def test_dft_brute_force_triple_sum_and_library():
    rng = np.random.default_rng(2)
    tau = rng.poisson(3.0, size=(8, 8, 8)).astype(np.float64)
    G = ofk.scale_and_pad(tau, 2)  # 16^3
    S = ofk.forward(G)
    # non-separable triple sum over the non-zero block
    M = 16
    n = np.arange(8)
    k = np.arange(M)
    ref = np.zeros((M, M, M), dtype=np.complex128)
    g = G[:8, :8, :8]
    for a in range(M):
        ey = np.exp(-2j * np.pi * ((a * n) % M) / M)
        for b in range(M):
            ex = np.exp(-2j * np.pi * ((b * n) % M) / M)
            w = ey[:, None] * ex[None, :]
            for c in range(M):
                et = np.exp(-2j * np.pi * ((c * n) % M) / M)
                ref[a, b, c] = np.sum(g * w[:, :, None] * et[None, None, :])
    assert np.max(np.abs(S - ref)) < 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(S - np.fft.fftn(G))) < 1e-12 * np.max(np.abs(ref))


def test_stolt_scalar_loop_at_8cubed():
    rng = np.random.default_rng(3)
    S = rng.normal(size=(16, 16, 16)) + 1j * rng.normal(size=(16, 16, 16))
    sx, sy = 0.7, 0.9
    out = ofk.stolt(S, sx, sy)
    ref = np.zeros_like(S)
    for iy in range(16):
        Y = (iy if iy < 8 else iy - 16) / 8
        for ix in range(16):
            X = (ix if ix < 8 else ix - 16) / 8
            for iz in range(16):
                kz = iz if iz < 8 else iz - 16
                if kz <= 0:
                    continue
                Z = kz / 8
                Zp = math.sqrt(sx * sx * X * X + sy * sy * Y * Y + Z * Z)
                q = Zp * 8
                if q > 7:
                    continue
                i0 = int(math.floor(q))
                f = q - i0
                v = S[iy, ix, i0] if i0 == 7 else (1 - f) * S[iy, ix, i0] + f * S[iy, ix, i0 + 1]
                ref[iy, ix, iz] = v * Z / Zp
    assert np.max(np.abs(out - ref)) < 1e-13


def test_stolt_jacobian_is_a_change_of_variables():
    # With g smooth along omega, sum_kz Z/Z' g(Z') dkz = integral of g over [a, inf):
    # the Jacobian makes the remap measure preserving (q dq = kz dkz).
    Mt = 1024
    half = Mt // 2
    S = np.zeros((2, 2, Mt), dtype=np.complex128)
    om = np.arange(half)
    mu, sig = 200.0, 25.0
    S[:, :, :half] = np.exp(-((om - mu) / sig) ** 2)
    for sx in (0.0, 0.2, 0.35):
        out = ofk.stolt(S, sx, 0.0)
        a = sx * half * 1.0  # column kx' = -1 of Mx = 2 has |X| = 1
        total = out[0, 1, :].real.sum()
        exact = 0.5 * math.sqrt(math.pi) * sig * (1.0 - erf((a - mu) / sig))
        assert abs(total - exact) < 2e-3 * exact


def test_dft_mixed_radix_lengths_brute_force():
    """Padded lengths with factors 3, 5, 7 (6 x 10 x 14): the same triple sum."""
    rng = np.random.default_rng(3)
    tau = rng.poisson(3.0, size=(3, 5, 7)).astype(np.float64)
    G = ofk.scale_and_pad(tau, 2)
    S = ofk.forward(G)
    My, Mx, Mt = S.shape
    assert (My, Mx, Mt) == (6, 10, 14)
    g = G[:3, :5, :7]
    ref = np.zeros(S.shape, dtype=np.complex128)
    for a in range(My):
        for b in range(Mx):
            for c in range(Mt):
                ph = ((a * np.arange(3))[:, None, None] * Mx * Mt + (b * np.arange(5))[None, :, None] * My * Mt
                      + (c * np.arange(7))[None, None, :] * My * Mx) % (My * Mx * Mt)
                ref[a, b, c] = np.sum(g * np.exp(-2j * np.pi * ph / (My * Mx * Mt)))
    assert np.max(np.abs(S - ref)) < 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(S - np.fft.fftn(G))) < 1e-12 * np.max(np.abs(ref))


def test_point_reflector_focuses_on_a_mixed_radix_grid():
    """A 30 x 26 scan of 192 bins pads to 60 x 52 x 384 (factors 3, 5, 13)."""
    cfg = scenes.small_config(30, 26, 192, bin_ps=32)
    pos = (0.1, -0.2, 0.5)
    tau = scenes.transient(cfg, noise=False, objects=[scenes.point_object(*pos)])
    vol, img = ofk.fk(tau, 1.0, 1.0, 32.0, pad=2)
    y, x, z = argmax_index(vol)
    ex = (pos[0] + 0.5) / cfg.dx - 0.5
    ey = (pos[1] + 0.5) / cfg.dy - 0.5
    ez = 2.0 * pos[2] / cfg.c_dt
    assert abs(x - ex) <= 1 and abs(y - ey) <= 1 and abs(z - ez) <= 1
    assert argmax_index(img) == (y, x)


@pytest.mark.parametrize("pos", [(0.1, -0.2, 0.5), (-0.3, 0.25, 0.7)])
def test_point_reflector_focuses_at_closed_form(pos):
    cfg = scenes.small_config(32, 32, 256, bin_ps=32)
    tau = scenes.transient(cfg, noise=False, objects=[scenes.point_object(*pos)])
    vol, img = ofk.fk(tau, 1.0, 1.0, 32.0, pad=2)
    y, x, z = argmax_index(vol)
    ex = (pos[0] + 0.5) / cfg.dx - 0.5
    ey = (pos[1] + 0.5) / cfg.dy - 0.5
    ez = 2.0 * pos[2] / cfg.c_dt   # confocal round trip t = 2 z0 / c at the apex
    assert abs(x - ex) <= 1 and abs(y - ey) <= 1 and abs(z - ez) <= 1
    assert argmax_index(img) == (y, x)


def test_stolt_constant_maximises_focus():
    cfg = scenes.small_config(32, 32, 256, bin_ps=32)
    tau = scenes.transient(cfg, noise=False, objects=[scenes.point_object(0.1, -0.2, 0.5)])
    sx, sy = ofk.stolt_constants(cfg.dx, cfg.dy, 32.0)
    peak = {f: ofk.fk(tau, 1, 1, 32.0, 2, s_override=(f * sx, f * sy))[0].max()
            for f in (0.8, 1.0, 1.25)}
    assert peak[1.0] > 2 * peak[0.8] and peak[1.0] > 2 * peak[1.25]


def test_analytic_signal_special_case():
    # pad 1 and an input constant over x, y: only kx = ky = 0 survives, Z' = Z there,
    # and each column is |IDFT(G [0 < k < Mt/2])|^2 = |a - G0/M - G_{M/2} (-1)^n / M|^2 / 4
    rng = np.random.default_rng(4)
    nt = 64
    line = rng.poisson(5.0, size=nt).astype(np.float64)
    tau = np.broadcast_to(line, (4, 8, nt)).copy()
    vol, _ = ofk.fk(tau, 0.5, 0.25, 32.0, pad=1)
    g = line * np.arange(nt) / (nt - 1)
    Gk = np.fft.fft(g)
    a = hilbert(g)
    n = np.arange(nt)
    ref = 0.25 * np.abs(a - Gk[0] / nt - Gk[nt // 2] * (-1.0) ** n / nt) ** 2
    assert np.max(np.abs(vol - ref[None, None, :])) < 1e-12 * ref.max()


def test_invariants_scale_shift_hermitian():
    rng = np.random.default_rng(5)
    tau = rng.poisson(2.0, size=(8, 8, 32)).astype(np.float64)
    tau[:, -1, :] = 0.0
    vol, _ = ofk.fk(tau, 1.0, 1.0, 32.0, pad=2)
    vol3, _ = ofk.fk(3.0 * tau, 1.0, 1.0, 32.0, pad=2)
    assert np.max(np.abs(vol3 - 9.0 * vol)) < 1e-10 * vol3.max()
    shifted = np.roll(tau, 1, axis=1)
    vs, _ = ofk.fk(shifted, 1.0, 1.0, 32.0, pad=2)
    assert np.max(np.abs(vs[:, 1:, :] - vol[:, :-1, :])) < 1e-10 * vol.max()
    S = ofk.forward(ofk.scale_and_pad(tau, 2))
    conj_flip = np.conj(S[(-np.arange(16)) % 16][:, (-np.arange(16)) % 16][:, :, (-np.arange(64)) % 64])
    assert np.max(np.abs(S - conj_flip)) < 1e-10 * np.abs(S).max()


def test_scaling_weights_are_the_linspace_of_algorithm_1():
    """Algorithm 1 scales the transient by linspace(0, 1, Nz) along t: weight 0 at the
    first bin, 1 at the last (t / (nt - 1)); t / nt or (t + 1) / nt would not match."""
    for nt in (2, 7, 256):
        G = ofk.scale_and_pad(np.ones((1, 1, nt)), 1)
        w = G[0, 0, :].real
        assert np.max(np.abs(w - np.linspace(0.0, 1.0, nt))) < 1e-15
        assert np.max(np.abs(w - np.arange(nt) / nt)) > 1e-3
        assert np.max(np.abs(w - (np.arange(nt) + 1) / nt)) > 1e-3
