"""GPU parity of the mixture of experts (Section 4.4, Eq. 10) against the FP64 oracle.

Two schedules: independent branches overlapped on two streams, and the paper's shared
spatial spectrum (both branches derived from one x/y DFT of the transient: the RSD
phasors by a temporal DFT of the spectrum's columns, the f-k t-scaling applied as the
columns load).  Each branch image and the mixture must match the oracle, which runs the
two reconstructions separately, to relative L2 <= 1e-4."""
import os

import numpy as np
import pytest
import torch

import scenes
from oracle import moe as omoe
from oracle.metrics import argmax_index, rel_l2
from paper_2608_28183_amd import runtime

from gpu_util import run_fk, run_rsd, say, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-4
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx(lib):
    return runtime.Context(0)


def moe_plan(ctx, cfg, pad=2, beta=0.3, eps=1e-6, n_depth=None, kernel_prec="fp32", shared=False):
    p = scenes.rsd_params(cfg, n_depth)
    plan = runtime.MoePlan(ctx, cfg.ny, cfg.nx, cfg.nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, pad,
                           p.freq_bins, p.weights, p.n_depth, p.depth0, p.depth_step, beta, eps,
                           kernel_prec=kernel_prec, shared_spectrum=shared)
    return plan, p


def run_moe(ctx, plan, tau, with_ws=True):
    ny, nx, _ = tau.shape
    img = torch.full((ny, nx), -1.0, device="cuda")
    ifk = torch.full((ny, nx), -1.0, device="cuda")
    irsd = torch.full((ny, nx), -1.0, device="cuda")
    plan(to_dev(tau.astype(np.float32)), img, ifk, irsd, plan.workspace() if with_ws else None)
    torch.cuda.synchronize()
    return [t.cpu().numpy().astype(np.float64) for t in (img, ifk, irsd)]


def oracle_moe(cfg, tau, p, pad=2, beta=0.3, eps=1e-6):
    depths = p.depth0 + p.depth_step * np.arange(p.n_depth)
    return omoe.moe(tau.astype(np.float64), cfg.wall_w, cfg.wall_h, cfg.bin_ps, pad, p.freq_bins,
                    p.weights, depths, beta, eps)


@pytest.mark.parametrize("shared", [False, True])
def test_moe_c1(ctx, shared):
    cfg = scenes.CONFIGS["c1"]
    tau = scenes.config_transient("c1")
    plan, p = moe_plan(ctx, cfg, shared=shared)
    say("moe c1", shared)
    img, ifk, irsd = run_moe(ctx, plan, tau)
    rimg, rfk, rrsd = oracle_moe(cfg, tau, p)
    say(f"  rel_l2 mix {rel_l2(img, rimg):.2e} fk {rel_l2(ifk, rfk):.2e} rsd {rel_l2(irsd, rrsd):.2e}")
    assert rel_l2(ifk, rfk) < TOL and rel_l2(irsd, rrsd) < TOL and rel_l2(img, rimg) < TOL
    assert img.max() == 1.0 and img.min() >= 0.0
    assert argmax_index(img) == argmax_index(rimg)


# (ny, nx, nt, pad, bin_ps): non-square, unpadded, short and long time axes (8 ns and more
# of time window, so that the scene's reflectors are inside it)
SHAPES = [(16, 32, 64, 2, 128), (32, 16, 128, 1, 64), (8, 8, 32, 2, 256), (16, 16, 512, 2, 32)]


@pytest.mark.parametrize("shared", [False, True])
@pytest.mark.parametrize("shape", SHAPES)
def test_moe_shapes(ctx, shape, shared):
    ny, nx, nt, pad, bin_ps = shape
    cfg = scenes.small_config(nx, ny, nt, bin_ps=bin_ps, pad=pad)
    tau = scenes.transient(cfg, seed=ny + nx + nt)
    assert tau.sum() > 0
    say("moe shape", shape)
    plan, p = moe_plan(ctx, cfg, pad=pad, n_depth=24, shared=shared)
    img, ifk, irsd = run_moe(ctx, plan, tau)
    rimg, rfk, rrsd = oracle_moe(cfg, tau, p, pad=pad)
    say(f"  rel_l2 mix {rel_l2(img, rimg):.2e} fk {rel_l2(ifk, rfk):.2e} rsd {rel_l2(irsd, rrsd):.2e}")
    assert rel_l2(ifk, rfk) < TOL and rel_l2(irsd, rrsd) < TOL and rel_l2(img, rimg) < TOL


@pytest.mark.parametrize("shared", [False, True])
def test_moe_branches_match_standalone_and_beta_one(ctx, shared):
    cfg = scenes.CONFIGS["c1"]
    tau = scenes.config_transient("c1")
    plan, p = moe_plan(ctx, cfg, beta=1.0, eps=1e-3, shared=shared)
    img, ifk, irsd = run_moe(ctx, plan, tau, with_ws=False)
    _, sfk = run_fk(ctx, tau, cfg.wall_w, cfg.wall_h, cfg.bin_ps, 2)
    _, srsd, _ = run_rsd(ctx, cfg, tau)
    say(f"  branch vs standalone: fk {rel_l2(ifk, sfk):.2e} rsd {rel_l2(irsd, srsd):.2e}")
    assert rel_l2(ifk, sfk) < 1e-5 and rel_l2(irsd, srsd) < 1e-5
    prod = (ifk / ifk.max()) * (irsd / irsd.max() + 1e-3)
    assert rel_l2(img, prod / prod.max()) < 1e-6


@pytest.mark.parametrize("shared", [False, True])
def test_moe_deterministic_and_zero(ctx, shared):
    cfg = scenes.CONFIGS["c1"]
    tau = scenes.config_transient("c1")
    plan, _ = moe_plan(ctx, cfg, shared=shared)
    a = run_moe(ctx, plan, tau)
    b = run_moe(ctx, plan, tau)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    z = run_moe(ctx, plan, np.zeros_like(tau))
    assert all(np.all(x == 0) for x in z)


@pytest.mark.parametrize("shared", [False, True])
def test_moe_full_size_c3(ctx, shared):
    """128x128x1024 padded to 256x256x2048 (f-k) and 256x256 (RSD, 129 frequencies, 64
    depths): the branch images against the stored oracle images, the mixture against
    Eq. 10 applied to them."""
    cfg = scenes.CONFIGS["c3"]
    tau = scenes.config_transient("c3")
    gfk = np.load(os.path.join(GOLDEN, "fk_c3.npz"), allow_pickle=False)
    grsd = np.load(os.path.join(GOLDEN, "rsd_c3.npz"), allow_pickle=False)
    assert str(gfk["tau_sha256"]) == scenes.checksum(tau) == str(grsd["tau_sha256"])
    say("moe c3 full size", shared)
    plan, _ = moe_plan(ctx, cfg, shared=shared)
    img, ifk, irsd = run_moe(ctx, plan, tau)
    rimg = omoe.mix(gfk["img"], grsd["img"])
    say(f"  rel_l2 mix {rel_l2(img, rimg):.2e} fk {rel_l2(ifk, gfk['img']):.2e} rsd {rel_l2(irsd, grsd['img']):.2e}")
    assert rel_l2(ifk, gfk["img"]) < TOL and rel_l2(irsd, grsd["img"]) < TOL and rel_l2(img, rimg) < TOL
    assert argmax_index(img) == argmax_index(rimg)
