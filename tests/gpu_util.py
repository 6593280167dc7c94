"""Helpers shared by the GPU parity tests (test infrastructure)."""
import sys

import numpy as np
import torch

import scenes
from paper_2608_28183_amd import runtime


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def run_fk(ctx, tau, wall_w=1.0, wall_h=1.0, bin_ps=32.0, pad=2, prec="fp32", with_ws=True):
    ny, nx, nt = tau.shape
    plan = runtime.FkPlan(ctx, ny, nx, nt, wall_w, wall_h, bin_ps, pad, prec)
    t = to_dev(tau.astype(np.float32))
    vol = torch.full((ny, nx, nt), -1.0, device="cuda")
    img = torch.full((ny, nx), -1.0, device="cuda")
    ws = plan.workspace() if with_ws else None
    plan(t, vol, img, ws)
    torch.cuda.synchronize()
    return vol.cpu().numpy().astype(np.float64), img.cpu().numpy().astype(np.float64)


def rsd_plan_for(ctx, cfg, pad=2, n_depth=None, kernel_prec="fp32", params=None, data_prec="fp32"):
    p = scenes.rsd_params(cfg, n_depth) if params is None else params
    plan = runtime.RsdPlan(ctx, cfg.ny, cfg.nx, cfg.nt, cfg.dx, cfg.dy, cfg.bin_ps, pad,
                           p.freq_bins, p.weights, p.n_depth, p.depth0, p.depth_step,
                           p.sigma_s, p.sigma_t, p.delta, data_prec, kernel_prec)
    return plan, p


def run_rsd(ctx, cfg, tau, pad=2, n_depth=None, kernel_prec="fp32", params=None):
    plan, p = rsd_plan_for(ctx, cfg, pad, n_depth, kernel_prec, params)
    t = to_dev(tau.astype(np.float32))
    vol = torch.full((cfg.ny, cfg.nx, p.n_depth), -1.0, device="cuda")
    img = torch.full((cfg.ny, cfg.nx), -1.0, device="cuda")
    plan(t, vol, img, plan.workspace())
    torch.cuda.synchronize()
    # the library writes vol[y][x][d]; the oracle's layout is [d][y][x]
    v = np.moveaxis(vol.cpu().numpy().astype(np.float64), 2, 0)
    return v, img.cpu().numpy().astype(np.float64), p
