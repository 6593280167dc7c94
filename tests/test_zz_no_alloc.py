"""nlos_fk_noalloc: the f-k entry point for callers that cannot allocate.

It runs nlos_fk's kernels on the library's static device scratch instead of a workspace,
so its outputs must equal nlos_fk's bit for bit.  Two calls in a row (the second on a
smaller input, leaving the first call's contents in the scratch), FP32 and FP16 plans,
and a plan whose workspace exceeds the scratch (rejected before anything is enqueued).
"""
import numpy as np
import pytest
import torch

import scenes
from oracle import fk as ofk
from oracle.metrics import rel_l2
from paper_2608_28183_amd import nlos, runtime

from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return runtime.Context(0)


def _tau(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.poisson(3.0, size=shape).astype(np.float32)


def _both(ctx, plan, tau, shape):
    ny, nx, nt = shape
    t = to_dev(tau)
    vol_a = torch.full(shape, -1.0, device="cuda")
    img_a = torch.full((ny, nx), -1.0, device="cuda")
    plan(t, vol_a, img_a, plan.workspace())
    vol_b = torch.full(shape, -2.0, device="cuda")
    img_b = torch.full((ny, nx), -2.0, device="cuda")
    nlos.nlos_fk_noalloc(ctx.handle, plan.handle, t, vol_b, img_b)
    torch.cuda.synchronize()
    return vol_a, img_a, vol_b, img_b


@pytest.mark.parametrize("prec,shapes", [
    ("fp32", [(64, 64, 512), (16, 32, 64)]),
    ("fp16", [(128, 128, 256), (8, 16, 32)]),
])
def test_noalloc_equals_nlos_fk_twice(ctx, prec, shapes):
    for i, shape in enumerate(shapes):
        ny, nx, nt = shape
        say(f"nlos_fk_noalloc {prec} call {i + 1}: {shape} padded x2")
        plan = runtime.FkPlan(ctx, ny, nx, nt, 1.0, 1.0, 32.0, 2, prec)
        assert plan.ws_bytes <= nlos.NLOS_STATIC_SCRATCH_BYTES
        tau = _tau(shape, 100 + i)
        vol_a, img_a, vol_b, img_b = _both(ctx, plan, tau, shape)
        assert torch.equal(vol_a, vol_b) and torch.equal(img_a, img_b)
        if prec == "fp32" and nt <= 64:
            rv, _ = ofk.fk(tau.astype(np.float64), 1.0, 1.0, 32.0, 2)
            e = rel_l2(vol_b.cpu().numpy(), rv)
            say(f"  rel_l2 vs the oracle {e:.2e}")
            assert e < 1e-4


def test_noalloc_image_only_and_volume_only(ctx):
    shape = (32, 32, 128)
    plan = runtime.FkPlan(ctx, *shape, 1.0, 1.0, 32.0, 2)
    tau = _tau(shape, 7)
    t = to_dev(tau)
    vol = torch.empty(shape, device="cuda")
    img = torch.empty(shape[:2], device="cuda")
    nlos.nlos_fk_noalloc(ctx.handle, plan.handle, t, vol, None)
    nlos.nlos_fk_noalloc(ctx.handle, plan.handle, t, None, img)
    torch.cuda.synchronize()
    assert torch.equal(vol.amax(dim=2), img)


def test_noalloc_rejects_a_workspace_beyond_the_scratch(ctx):
    plan = runtime.FkPlan(ctx, 256, 256, 512, 1.0, 1.0, 32.0, 2)
    assert plan.ws_bytes > nlos.NLOS_STATIC_SCRATCH_BYTES
    t = torch.zeros((256, 256, 512), device="cuda")
    img = torch.full((256, 256), -1.0, device="cuda")
    with pytest.raises(nlos.NlosError) as e:
        nlos.nlos_fk_noalloc(ctx.handle, plan.handle, t, None, img)
    assert e.value.status == nlos.NLOS_ERR_UNSUPPORTED
    assert "static scratch" in nlos.nlos_last_error(ctx.handle)
    torch.cuda.synchronize()
    assert torch.all(img == -1.0)  # nothing was enqueued
