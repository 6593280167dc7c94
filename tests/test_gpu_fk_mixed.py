"""GPU parity of nlos_fk on padded grids that are not powers of two (general mixed-radix
kernels, FP32) against the FP64 oracle, relative L2 <= 1e-4 as for the power-of-two path.

The shapes cover every radix of the general kernels (2, 3, 4, 5, 7, 8, 11, 13), odd nt
(a real time column without a partner in the packed x-FFT), grids where only some axes
are general (the others stay on the power-of-two kernels), and the longest lines of each
general pass.  The office-scene grid of the paper's Table 4 (360 x 260 x 512, padded to
720 x 520 x 1024) runs at full size against the closed-form focus of a point reflector.
"""
import numpy as np
import pytest
import torch

import scenes
from oracle import fk as ofk
from oracle.metrics import argmax_index, rel_l2
from paper_2608_28183_amd import nlos, runtime

from gpu_util import run_fk, say, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-4

# (ny, nx, nt, pad) -> padded (My, Mx, Mt)
SHAPES = [
    (12, 10, 24, 2),    # 24 x 20 x 48
    (26, 18, 30, 1),    # 26 x 18 x 30, unpadded
    (13, 15, 20, 2),    # 26 x 30 x 40, odd scan sizes
    (9, 7, 11, 2),      # 18 x 14 x 22: radices 3, 7, 11; odd nt
    (7, 11, 9, 2),      # 14 x 22 x 18, odd nt
    (36, 26, 64, 2),    # 72 x 52 x 128: general y and x, power-of-two t
    (16, 16, 75, 2),    # 32 x 32 x 150: general t only
    (8, 520, 8, 1),     # 520-point x lines (8 x 5 x 13)
    (520, 8, 8, 1),     # 520-point y lines
    (507, 4, 4, 2),     # 1014-point y lines (2 x 3 x 13 x 13)
    (4, 1155, 4, 2),    # 2310-point x lines (2 x 3 x 5 x 7 x 11)
    (4, 4, 1500, 2),    # 3000-point t columns (2^3 x 3 x 5^3)
    (52, 72, 128, 2),   # the office grid at a fifth of its size
    (4, 2048, 4, 2),    # the longest general line, 4096 points along x (one-column tiles)
    (4, 4, 2048, 2),    # 4096-point t columns and z lines
]


@pytest.fixture(scope="module")
def ctx(lib):
    return runtime.Context(0)


@pytest.mark.parametrize("shape", SHAPES)
def test_fk_mixed_radix_shapes(ctx, shape):
    ny, nx, nt, pad = shape
    say("fk mixed", shape)
    rng = np.random.default_rng(ny * 131 + nx * 7 + nt + pad)
    tau = rng.poisson(3.0, size=(ny, nx, nt)).astype(np.float32)
    ww, wh, bps = 0.5 + 0.01 * nx, 0.4 + 0.01 * ny, 24.0
    vol, img = run_fk(ctx, tau, ww, wh, bps, pad)
    rv, ri = ofk.fk(tau.astype(np.float64), ww, wh, bps, pad)
    say("  rel_l2", rel_l2(vol, rv), rel_l2(img, ri))
    assert rel_l2(vol, rv) < TOL and rel_l2(img, ri) < TOL


def test_fk_mixed_radix_complex_field(ctx):
    ny, nx, nt = 26, 30, 48
    tau = np.random.default_rng(11).poisson(2.0, size=(ny, nx, nt)).astype(np.float32)
    plan = runtime.FkPlan(ctx, ny, nx, nt, 0.9, 0.8, 32.0, 2)
    psi = torch.empty((ny, nx, nt, 2), device="cuda")
    nlos.nlos_fk_complex(ctx.handle, plan.handle, to_dev(tau), psi, plan.workspace())
    torch.cuda.synchronize()
    a = psi.cpu().numpy().astype(np.float64)
    _, _, rpsi = ofk.fk(tau.astype(np.float64), 0.9, 0.8, 32.0, 2, return_psi=True)
    say("  field rel_l2", rel_l2(a[..., 0] + 1j * a[..., 1], rpsi))
    assert rel_l2(a[..., 0] + 1j * a[..., 1], rpsi) < TOL


def test_fk_mixed_radix_zero_input_and_pool_workspace(ctx):
    vol, img = run_fk(ctx, np.zeros((26, 30, 40), np.float32), with_ws=False)
    assert np.all(vol == 0) and np.all(img == 0)


def test_fk_office_grid_full_size(ctx):
    """360 x 260 x 512 at 5 mm pitch, padded to 720 x 520 x 1024: a point reflector
    focuses at its closed-form voxel, and two runs agree bit for bit."""
    cfg = scenes.CONFIGS["office"]
    pos = (0.3, -0.2, 0.6)
    tau = scenes.transient(cfg, noise=False, objects=[scenes.point_object(*pos)])
    say("fk office", tau.shape)
    v1, i1 = run_fk(ctx, tau, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad)
    v2, i2 = run_fk(ctx, tau, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad)
    assert np.array_equal(v1, v2) and np.array_equal(i1, i2)
    y, x, z = argmax_index(v1)
    ex = (pos[0] + 0.5 * cfg.wall_w) / cfg.dx - 0.5
    ey = (pos[1] + 0.5 * cfg.wall_h) / cfg.dy - 0.5
    ez = 2.0 * pos[2] / cfg.c_dt
    say("  peak", (y, x, z), "expected", (ey, ex, ez))
    assert abs(x - ex) <= 1 and abs(y - ey) <= 1 and abs(z - ez) <= 1
    assert argmax_index(i1) == (y, x)
