"""Error returns of the compute calls on the GPU.

Every rejected call must return its status before anything is enqueued: the outputs keep
their sentinel values, and the context stays usable (the next valid call gives the same
result as one made before the failures).  Device-allocation failures are injected with
nlos_debug_fail_allocations.  A plan of another device needs a second GPU and is checked
only on the host side (the plan records its device and the compute calls compare it).
"""
import ctypes

import numpy as np
import pytest
import torch

import scenes
from paper_2608_28183_amd import nlos, runtime

from gpu_util import rsd_plan_for, say, to_dev

pytestmark = pytest.mark.gpu
SENTINEL = -7.25


@pytest.fixture(scope="module")
def ctx(lib):
    return runtime.Context(0)


def status(fn, *args):
    return getattr(nlos.lib(), fn)(*args)


def ptr(t, offset=0):
    return None if t is None else t.data_ptr() + offset


def outputs(shape_vol, shape_img):
    return (torch.full(shape_vol, SENTINEL, device="cuda"), torch.full(shape_img, SENTINEL, device="cuda"))


def untouched(*ts):
    torch.cuda.synchronize()
    return all(bool((t == SENTINEL).all()) for t in ts)


@pytest.fixture(scope="module")
def fk_case(ctx):
    cfg = scenes.CONFIGS["c1"]
    tau = to_dev(scenes.config_transient("c1").astype(np.float32))
    plan = runtime.FkPlan(ctx, cfg.ny, cfg.nx, cfg.nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad)
    vol, img = outputs(cfg.shape, (cfg.ny, cfg.nx))
    plan(tau, vol, img, plan.workspace())
    torch.cuda.synchronize()
    return cfg, tau, plan, vol.clone(), img.clone()


def test_fk_rejects_bad_arguments_before_any_launch(ctx, fk_case):
    cfg, tau, plan, ref_vol, ref_img = fk_case
    ws = torch.empty(plan.ws_bytes + 512, dtype=torch.uint8, device="cuda")
    c, p = ctx.handle, plan.handle
    cases = {
        "workspace too small": (nlos.NLOS_ERR_OUT_OF_MEMORY, lambda v, i: status(
            "nlos_fk", c, p, ptr(tau), ptr(v), ptr(i), ptr(ws), plan.ws_bytes - 256)),
        "workspace misaligned": (nlos.NLOS_ERR_INVALID_ARG, lambda v, i: status(
            "nlos_fk", c, p, ptr(tau), ptr(v), ptr(i), ptr(ws, 64), plan.ws_bytes)),
        "d_tau NULL": (nlos.NLOS_ERR_INVALID_ARG, lambda v, i: status(
            "nlos_fk", c, p, None, ptr(v), ptr(i), ptr(ws), plan.ws_bytes)),
        "d_tau misaligned": (nlos.NLOS_ERR_INVALID_ARG, lambda v, i: status(
            "nlos_fk", c, p, ptr(tau, 4), ptr(v), ptr(i), ptr(ws), plan.ws_bytes)),
        "both outputs NULL": (nlos.NLOS_ERR_INVALID_ARG, lambda v, i: status(
            "nlos_fk", c, p, ptr(tau), None, None, ptr(ws), plan.ws_bytes)),
        "plan NULL": (nlos.NLOS_ERR_INVALID_ARG, lambda v, i: status(
            "nlos_fk", c, None, ptr(tau), ptr(v), ptr(i), ptr(ws), plan.ws_bytes)),
        "ctx NULL": (nlos.NLOS_ERR_INVALID_ARG, lambda v, i: status(
            "nlos_fk", None, p, ptr(tau), ptr(v), ptr(i), ptr(ws), plan.ws_bytes)),
        "noalloc d_tau NULL": (nlos.NLOS_ERR_INVALID_ARG, lambda v, i: status(
            "nlos_fk_noalloc", c, p, None, ptr(v), ptr(i))),
    }
    for name, (want, call) in cases.items():
        vol, img = outputs(cfg.shape, (cfg.ny, cfg.nx))
        got = call(vol, img)
        say(f"fk {name}: {nlos.STATUS_NAMES.get(got, got)}")
        assert got == want, name
        assert untouched(vol, img), name
        if c is not None:
            assert nlos.nlos_last_error(c) != ""
    # the context still works, with the exact workspace at its exact size
    vol, img = outputs(cfg.shape, (cfg.ny, cfg.nx))
    assert status("nlos_fk", c, p, ptr(tau), ptr(vol), ptr(img), ptr(ws), plan.ws_bytes) == nlos.NLOS_OK
    torch.cuda.synchronize()
    assert torch.equal(vol, ref_vol) and torch.equal(img, ref_img)


def test_rsd_rejects_bad_arguments_before_any_launch(ctx):
    cfg = scenes.CONFIGS["c1"]
    tau = to_dev(scenes.config_transient("c1").astype(np.float32))
    plan, p = rsd_plan_for(ctx, cfg)
    ws = torch.empty(plan.ws_bytes + 512, dtype=torch.uint8, device="cuda")
    shape_vol = (cfg.ny, cfg.nx, p.n_depth)
    ref_vol, ref_img = outputs(shape_vol, (cfg.ny, cfg.nx))
    plan(tau, ref_vol, ref_img, ws)
    c, h = ctx.handle, plan.handle
    cases = {
        "workspace too small": (nlos.NLOS_ERR_OUT_OF_MEMORY, lambda v, i: status(
            "nlos_rsd", c, h, ptr(tau), ptr(v), ptr(i), ptr(ws), plan.ws_bytes - 8)),
        "workspace misaligned": (nlos.NLOS_ERR_INVALID_ARG, lambda v, i: status(
            "nlos_rsd", c, h, ptr(tau), ptr(v), ptr(i), ptr(ws, 128), plan.ws_bytes)),
        "d_tau NULL": (nlos.NLOS_ERR_INVALID_ARG, lambda v, i: status(
            "nlos_rsd", c, h, None, ptr(v), ptr(i), ptr(ws), plan.ws_bytes)),
        "both outputs NULL": (nlos.NLOS_ERR_INVALID_ARG, lambda v, i: status(
            "nlos_rsd", c, h, ptr(tau), None, None, ptr(ws), plan.ws_bytes)),
        "plan NULL": (nlos.NLOS_ERR_INVALID_ARG, lambda v, i: status(
            "nlos_rsd", c, None, ptr(tau), ptr(v), ptr(i), ptr(ws), plan.ws_bytes)),
        "phasors misaligned": (nlos.NLOS_ERR_INVALID_ARG, lambda v, i: status(
            "nlos_rsd_from_phasors", c, h, ptr(tau, 4), ptr(v), ptr(i), ptr(ws), plan.ws_bytes)),
    }
    for name, (want, call) in cases.items():
        vol, img = outputs(shape_vol, (cfg.ny, cfg.nx))
        got = call(vol, img)
        say(f"rsd {name}: {nlos.STATUS_NAMES.get(got, got)}")
        assert got == want, name
        assert untouched(vol, img), name
    vol, img = outputs(shape_vol, (cfg.ny, cfg.nx))
    plan(tau, vol, img, ws)
    torch.cuda.synchronize()
    assert torch.equal(vol, ref_vol) and torch.equal(img, ref_img)


def test_injected_device_allocation_failures(fk_case):
    cfg, tau, plan, ref_vol, ref_img = fk_case
    try:
        # a fresh context has no workspace pool: its first pool-backed call allocates one
        fresh = runtime.Context(0)
        nlos.nlos_debug_fail_allocations(1)
        vol, img = outputs(cfg.shape, (cfg.ny, cfg.nx))
        got = status("nlos_fk", fresh.handle, plan.handle, ptr(tau), ptr(vol), ptr(img), None, 0)
        say(f"fk with the pool allocation failing: {nlos.STATUS_NAMES.get(got, got)}")
        assert got == nlos.NLOS_ERR_OUT_OF_MEMORY
        assert untouched(vol, img)
        # the failure is consumed: the same call now allocates the pool and succeeds
        assert status("nlos_fk", fresh.handle, plan.handle, ptr(tau), ptr(vol), ptr(img), None, 0) == nlos.NLOS_OK
        torch.cuda.synchronize()
        assert torch.equal(vol, ref_vol) and torch.equal(img, ref_img)

        # context and plan creation
        nlos.nlos_debug_fail_allocations(1)
        out = ctypes.c_void_p()
        assert status("nlos_create", 0, None, ctypes.byref(out)) == nlos.NLOS_ERR_OUT_OF_MEMORY
        assert not out.value
        nlos.nlos_debug_fail_allocations(1)
        pout = ctypes.c_void_p()
        assert status("nlos_fk_plan_create", fresh.handle, ctypes.byref(plan.desc), ctypes.byref(pout)) \
            == nlos.NLOS_ERR_OUT_OF_MEMORY
        assert not pout.value
        # a second fk plan on the recovered context reconstructs like the first
        plan2 = runtime.FkPlan(fresh, cfg.ny, cfg.nx, cfg.nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad)
        vol, img = outputs(cfg.shape, (cfg.ny, cfg.nx))
        plan2(tau, vol, img)
        torch.cuda.synchronize()
        assert torch.equal(vol, ref_vol) and torch.equal(img, ref_img)
    finally:
        nlos.nlos_debug_fail_allocations(0)
