"""Pins of the mixture-of-experts oracle (Section 4.4, Eq. 10) against closed forms."""
import numpy as np
import pytest

import scenes
from oracle import fk as ofk, moe, rsd as orsd



def _imgs(seed=0, shape=(9, 11)):
    rng = np.random.default_rng(seed)
    return rng.gamma(0.5, 2.0, size=shape), rng.gamma(0.7, 3.0, size=shape)


def test_beta_zero_is_the_fk_image():
    a, b = _imgs(1)
    np.testing.assert_allclose(moe.mix(a, b, beta=0.0), a / a.max(), rtol=1e-15, atol=0)


def test_beta_one_is_the_plain_product():
    a, b = _imgs(2)
    p = (a / a.max()) * (b / b.max() + 1e-6)
    np.testing.assert_allclose(moe.mix(a, b, beta=1.0), p / p.max(), rtol=1e-14, atol=0)


def test_formula_by_hand_on_a_tiny_image():
    a = np.array([[4.0, 2.0], [0.0, 1.0]])
    b = np.array([[1.0, 8.0], [4.0, 0.0]])
    eps, beta = 1e-6, 0.3
    # a / 4, b / 8, then the power, then the maximum of the result
    raw = np.array([[1.0 * (0.125 + eps) ** beta, 0.5 * (1.0 + eps) ** beta],
                    [0.0, 0.25 * eps ** beta]])
    np.testing.assert_allclose(moe.mix(a, b, beta, eps), raw / raw.max(), rtol=1e-15)


def test_scale_invariance_and_range():
    a, b = _imgs(3)
    m = moe.mix(a, b)
    np.testing.assert_allclose(moe.mix(7.5 * a, 0.01 * b), m, rtol=1e-13)
    assert m.max() == 1.0 and m.min() >= 0.0


def test_gate_suppresses_where_rsd_is_dark():
    # equal f-k response at two pixels: the one RSD does not see is attenuated by
    # (eps / (1 + eps))^beta relative to the one it does
    a = np.array([1.0, 1.0])
    b = np.array([1.0, 0.0])
    m = moe.mix(a, b)
    np.testing.assert_allclose(m[1] / m[0], (1e-6 / (1 + 1e-6)) ** 0.3, rtol=1e-12)


def test_zero_images_stay_zero():
    z = np.zeros((3, 4))
    assert np.all(moe.mix(z, z) == 0)


def test_moe_composes_the_branch_oracles():
    cfg = scenes.small_config(16, 16, 128, bin_ps=64)
    tau = scenes.transient(cfg, noise=False, objects=[scenes.point_object(0.05, -0.1, 0.6)])
    assert tau.sum() > 0
    p = scenes.rsd_params(cfg, 16)
    depths = p.depth0 + p.depth_step * np.arange(p.n_depth)
    m, ifk, irsd = moe.moe(tau.astype(np.float64), cfg.wall_w, cfg.wall_h, cfg.bin_ps, 2,
                           p.freq_bins, p.weights, depths)
    _, ifk2 = ofk.fk(tau.astype(np.float64), cfg.wall_w, cfg.wall_h, cfg.bin_ps, 2)
    _, irsd2 = orsd.rsd(tau.astype(np.float64), cfg.dx, cfg.dy, cfg.bin_ps, 2, p.freq_bins,
                        p.weights, depths)
    assert np.array_equal(ifk, ifk2) and np.array_equal(irsd, irsd2)
    np.testing.assert_allclose(m, moe.mix(ifk2, irsd2), rtol=0, atol=0)
    # the point reflector is where both experts agree: the mixture keeps its peak
    assert np.unravel_index(np.argmax(m), m.shape) == np.unravel_index(np.argmax(ifk), ifk.shape)
