"""GPU parity of nlos_rsd on grids that are not powers of two (general mixed-radix
kernels for the phasor t-DFT and the spatial 2D transforms) against the FP64 radial-RSD
oracle, relative L2 <= 1e-4 as for the power-of-two path; the office grid of the paper's
Table 4 (360 x 260, 512 bins, padded to 720 x 520) at full size against the closed-form
focus of a point reflector."""
import numpy as np
import pytest
import torch

import scenes
from oracle import rsd as orsd
from oracle.metrics import argmax_index, rel_l2
from paper_2608_28183_amd import nlos, runtime

from gpu_util import run_rsd, rsd_plan_for, say, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def ctx(lib):
    return runtime.Context(0)


def oracle_rsd(cfg, tau, p, pad=2, return_complex=False):
    depths = p.depth0 + p.depth_step * np.arange(p.n_depth)
    return orsd.rsd(tau.astype(np.float64), cfg.dx, cfg.dy, cfg.bin_ps, pad, p.freq_bins, p.weights, depths,
                    p.sigma_s, p.sigma_t, p.delta, return_complex=return_complex)


# (nx, ny, nt, pad, n_depth): general x and y with a power-of-two t, general t only, all
# general, unpadded general, radices 7 / 11 / 13
CASES = [
    (36, 26, 128, 2, 12),   # 72 x 52 spatial grid
    (16, 16, 150, 2, 8),    # phasor t-DFT of 150 samples
    (30, 26, 120, 2, 10),   # 60 x 52, t 120
    (20, 18, 96, 1, 16),    # unpadded 20 x 18, t 96
    (14, 11, 154, 2, 6),    # 28 x 22, t 154 = 2 x 7 x 11
    (13, 16, 104, 2, 5),    # 26 x 32, t 104 = 8 x 13
    (13, 11, 128, 2, 6),    # 26 x 22, t 128: an odd pixel count (the last real pair is one line)
]


@pytest.mark.parametrize("case", CASES)
def test_rsd_mixed_radix(ctx, case):
    nx, ny, nt, pad, nd = case
    cfg = scenes.small_config(nx, ny, nt, bin_ps=48, depth_range=(0.3, 0.8), n_depth=nd, seed=nx + ny + nt)
    tau = scenes.transient(cfg)
    say("rsd mixed", case)
    vol, img, p = run_rsd(ctx, cfg, tau, pad=pad)
    rv, ri = oracle_rsd(cfg, tau, p, pad)
    say("  rel_l2", rel_l2(vol, rv), rel_l2(img, ri))
    assert rel_l2(vol, rv) < TOL and rel_l2(img, ri) < TOL


def test_rsd_mixed_radix_fp16_kernel(ctx):
    """FP16 storage of the radial kernel on a general grid: the same 2e-3 bound as on
    power-of-two grids (one rounding of each kernel value)."""
    cfg = scenes.small_config(30, 26, 120, bin_ps=48, depth_range=(0.3, 0.8), n_depth=10, seed=9)
    tau = scenes.transient(cfg)
    vol, img, p = run_rsd(ctx, cfg, tau, kernel_prec="fp16")
    rv, ri = oracle_rsd(cfg, tau, p)
    say("  fp16 kernel rel_l2", rel_l2(vol, rv))
    assert rel_l2(vol, rv) < 2e-3 and argmax_index(vol) == argmax_index(rv)


def test_rsd_mixed_radix_complex_field(ctx):
    cfg = scenes.small_config(30, 26, 120, bin_ps=48, depth_range=(0.3, 0.8), n_depth=7, seed=5)
    tau = scenes.transient(cfg)
    plan, p = rsd_plan_for(ctx, cfg, pad=2)
    field = torch.empty((cfg.ny, cfg.nx, p.n_depth, 2), device="cuda")
    nlos.nlos_rsd_complex(ctx.handle, plan.handle, to_dev(tau), field, plan.workspace())
    torch.cuda.synchronize()
    a = field.cpu().numpy().astype(np.float64)
    I = np.moveaxis(a[..., 0] + 1j * a[..., 1], 2, 0)
    _, _, Ic = oracle_rsd(cfg, tau, p, 2, return_complex=True)
    say("  field rel_l2", rel_l2(I, Ic))
    assert rel_l2(I, Ic) < TOL


def test_rsd_office_grid_full_size(ctx):
    """360 x 260 x 512 padded to 720 x 520: a point reflector focuses at its closed-form
    voxel (lateral within one pixel, depth within one plane), and two runs agree bit for
    bit."""
    cfg = scenes.CONFIGS["office"]
    pos = (0.3, -0.2, 0.9)
    tau = scenes.transient(cfg, noise=False, objects=[scenes.point_object(*pos)])
    say("rsd office", tau.shape)
    v1, i1, p = run_rsd(ctx, cfg, tau, pad=cfg.pad, n_depth=51)
    v2, i2, _ = run_rsd(ctx, cfg, tau, pad=cfg.pad, n_depth=51)
    assert np.array_equal(v1, v2) and np.array_equal(i1, i2)
    d, y, x = argmax_index(v1)
    ex = (pos[0] + 0.5 * cfg.wall_w) / cfg.dx - 0.5
    ey = (pos[1] + 0.5 * cfg.wall_h) / cfg.dy - 0.5
    ed = (pos[2] - p.depth0) / p.depth_step
    say("  peak", (d, y, x), "expected", (ed, ey, ex), "freqs", len(p.freq_bins))
    assert abs(x - ex) <= 1 and abs(y - ey) <= 1 and abs(d - ed) <= 1
