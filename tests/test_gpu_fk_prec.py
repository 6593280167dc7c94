"""GPU accuracy of the reduced-precision f-k path (Section 4.2, data quantization).

FP16 / BF16 hold the five complex intermediates at four bytes per value.  BF16 is stored
as is; FP16 is stored times a power of two per intermediate, computed on the device from
a bound on its magnitude.  Where the line lengths allow (strided lines of 256 or 512
points, 1024-point columns) the DFT stages run on the matrix cores: products of the
stored values with a constant DFT matrix rounded to the same format, accumulated in FP32,
the intermediate between the two products rounded to the format once more.  Each such
rounding is a relative error of at most u per element (2^-11 for FP16, 2^-8 for BF16;
FP16 values that the scaling leaves subnormal are too small to matter in L2: the bound
exceeds the RMS of an intermediate by at most 2^23).  The DFTs are unitary up to their
scale and the Stolt remap is a linear interpolation times kz/q <= 1, so |Psi|^2 stays
within about 10 u in relative L2: the bound used here (4.9e-3 for FP16, 3.9e-2 for BF16).
The paper reports 57 dB image PSNR for its FP16 f-k against FP32; FP16 here is held to
that level on the image against the FP64 oracle.
"""
import numpy as np
import pytest

import scenes
from oracle import fk as ofk
from oracle.metrics import argmax_index, psnr_maxnorm, rel_l2
from paper_2608_28183_amd import runtime

from gpu_util import run_fk, say

pytestmark = pytest.mark.gpu
UNIT = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}
PSNR_MIN = {"fp16": 57.0, "bf16": 40.0}


def tol(prec):
    return 10 * UNIT[prec]


@pytest.fixture(scope="module")
def ctx(lib):
    return runtime.Context(0)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_fk_reduced_c1(ctx, prec):
    cfg = scenes.CONFIGS["c1"]
    tau = scenes.config_transient("c1")
    say("fk c1", prec)
    vol, img = run_fk(ctx, tau, cfg.wall_w, cfg.wall_h, cfg.bin_ps, 2, prec=prec)
    rv, ri = ofk.fk(tau.astype(np.float64), cfg.wall_w, cfg.wall_h, cfg.bin_ps, 2)
    e_v, e_i, ps = rel_l2(vol, rv), rel_l2(img, ri), psnr_maxnorm(img, ri)
    say("  rel_l2 vol %.3e img %.3e psnr %.1f dB" % (e_v, e_i, ps))
    assert e_v < tol(prec) and e_i < tol(prec)
    assert ps >= PSNR_MIN[prec]
    assert argmax_index(vol) == argmax_index(rv)


# shapes that exercise every line length of the reduced-precision kernels, including
# 2048-point columns (32 samples per thread) and lines shorter than one tile
SHAPES = [(4, 4, 4, 2), (8, 8, 8, 1), (16, 8, 32, 2), (8, 32, 16, 1), (32, 16, 64, 2),
          (4, 1024, 8, 2), (1024, 4, 8, 2), (4, 4, 1024, 2), (8, 8, 2048, 1), (64, 64, 128, 2),
          (8, 2048, 8, 1), (128, 8, 16, 2)]


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_fk_reduced_shapes(ctx, shape, prec):
    ny, nx, nt, pad = shape
    say("fk reduced", prec, shape)
    rng = np.random.default_rng(ny * 131 + nx * 7 + nt + pad)
    tau = rng.poisson(3.0, size=(ny, nx, nt)).astype(np.float32)
    ww, wh, bps = 0.5 + 0.01 * nx, 0.4 + 0.01 * ny, 24.0
    vol, img = run_fk(ctx, tau, ww, wh, bps, pad, prec=prec)
    rv, ri = ofk.fk(tau.astype(np.float64), ww, wh, bps, pad)
    say("  rel_l2", rel_l2(vol, rv), rel_l2(img, ri))
    assert rel_l2(vol, rv) < tol(prec) and rel_l2(img, ri) < tol(prec)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_fk_reduced_zero_input(ctx, prec):
    tau = np.zeros((16, 16, 32), np.float32)
    vol, img = run_fk(ctx, tau, prec=prec, with_ws=False)
    assert np.all(vol == 0) and np.all(img == 0)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_fk_reduced_scale_invariant(ctx, prec):
    """Power-of-two storage scales derived from the input make the result exactly
    equivariant to a power-of-two input scale: tau 2^-k gives |Psi|^2 2^-2k bit for bit
    (as long as nothing leaves the FP32 normal range), where a fixed-scale FP16 store
    would underflow."""
    tau = scenes.config_transient("c1")
    k = 40
    v1, i1 = run_fk(ctx, tau, prec=prec)
    v2, i2 = run_fk(ctx, tau * np.float32(2.0 ** -k), prec=prec)
    live = v1 > v1.max() * 1e-20
    say("  live fraction", live.mean())
    assert np.array_equal(v2[live] * 2.0 ** (2 * k), v1[live])
    assert np.array_equal(i2 * 2.0 ** (2 * k), i1)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_fk_reduced_deterministic(ctx, prec):
    tau = scenes.config_transient("c1")
    v1, i1 = run_fk(ctx, tau, prec=prec)
    v2, i2 = run_fk(ctx, tau, prec=prec)
    assert np.array_equal(v1, v2) and np.array_equal(i1, i2)


# shapes on the matrix-core passes: strided lines of 256 and 512 points (forward with
# zero-padded inputs, inverse with cropped outputs, and unpadded), 1024-point columns with
# 512 stored samples (column pass, z-IFFT)
MFMA_SHAPES = [(128, 8, 512, 2), (8, 128, 512, 2), (16, 256, 64, 2), (256, 16, 64, 2),
               (256, 256, 32, 1), (32, 32, 512, 2)]


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("shape", MFMA_SHAPES)
def test_fk_reduced_matrix_core_shapes(ctx, shape, prec):
    ny, nx, nt, pad = shape
    say("fk matrix-core", prec, shape)
    rng = np.random.default_rng(ny * 17 + nx * 3 + nt + pad)
    tau = rng.poisson(3.0, size=(ny, nx, nt)).astype(np.float32)
    ww, wh, bps = 0.5 + 0.01 * nx, 0.4 + 0.01 * ny, 24.0
    vol, img = run_fk(ctx, tau, ww, wh, bps, pad, prec=prec)
    rv, ri = ofk.fk(tau.astype(np.float64), ww, wh, bps, pad)
    say("  rel_l2 vol %.3e img %.3e" % (rel_l2(vol, rv), rel_l2(img, ri)))
    assert rel_l2(vol, rv) < tol(prec) and rel_l2(img, ri) < tol(prec)
