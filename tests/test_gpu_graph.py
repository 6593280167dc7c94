"""Graph replay (nlos_fk_graph_create / nlos_rsd_graph_create / nlos_graph_launch): every
replay equals the eager call on the same input bit for bit, with new inputs written into
the captured input buffer and eager work and synchronisations between the replays."""
import numpy as np
import pytest
import torch

import scenes
from paper_2608_28183_amd import runtime

from gpu_util import rsd_plan_for, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return runtime.Context(0)


def _inputs(shape, n, seed):
    rng = np.random.default_rng(seed)
    return [to_dev(rng.poisson(2.0 + k, size=shape).astype(np.float32)) for k in range(n)]


def _check_replays(plan, shape, zshape, inputs):
    ny, nx, _ = shape
    tau_s = torch.empty(shape, device="cuda")
    vol_s = torch.empty(zshape, device="cuda")
    img_s = torch.empty((ny, nx), device="cuda")
    g = plan.graph(tau_s, vol_s, img_s)
    other = torch.empty(zshape, device="cuda")
    for k, tau in enumerate(inputs):
        vol_e = torch.full(zshape, -1.0, device="cuda")
        img_e = torch.full((ny, nx), -1.0, device="cuda")
        plan(tau, vol_e, img_e)               # eager reference
        plan(inputs[-1 - k], other, None)     # unrelated eager work between replays
        torch.cuda.synchronize()
        tau_s.copy_(tau)
        g.replay()
        torch.cuda.synchronize()
        say("  replay", k, float((vol_s - vol_e).abs().max()))
        assert torch.equal(vol_s, vol_e) and torch.equal(img_s, img_e)
    g.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_fk_graph_replays_match_eager(ctx, prec):
    shape = (32, 32, 256)
    plan = runtime.FkPlan(ctx, *shape, 1.0, 1.0, 32.0, 2, prec)
    say("fk graph", prec)
    _check_replays(plan, shape, shape, _inputs(shape, 3, 1))


def test_fk_graph_mixed_radix(ctx):
    shape = (26, 30, 48)
    plan = runtime.FkPlan(ctx, *shape, 0.9, 0.8, 32.0, 2)
    _check_replays(plan, shape, shape, _inputs(shape, 3, 2))


def test_rsd_graph_replays_match_eager(ctx):
    cfg = scenes.CONFIGS["c1"]
    plan, p = rsd_plan_for(ctx, cfg)
    shape = (cfg.ny, cfg.nx, cfg.nt)
    _check_replays(plan, shape, (cfg.ny, cfg.nx, p.n_depth), _inputs(shape, 3, 3))


def test_graph_needs_a_large_enough_workspace(ctx):
    shape = (16, 16, 32)
    plan = runtime.FkPlan(ctx, *shape, 1.0, 1.0, 32.0, 2)
    t = torch.zeros(shape, device="cuda")
    small = torch.empty(plan.ws_bytes // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(Exception):
        plan.graph(t, torch.empty(shape, device="cuda"), None, small)
