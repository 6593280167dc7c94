"""Parity at the full configuration sizes, in the launch configuration bench.py times.

f-k at 256x256x512 (padded 512x512x1024) and 128x128x1024 (padded 256x256x2048),
radial RSD at 128x128x1024 (129 frequencies, 64 depths): the GPU result is compared
with FP64 oracle values stored by tests/golden/make_golden.py (full max-over-depth
image, 1024 largest and 3072 random voxels).  The 64x64x512 raw-photon case runs the
oracle live: binning bit-exact, then f-k and RSD of the binned histogram.
"""
import os

import numpy as np
import pytest
import torch

import scenes
from oracle import binning, fk as ofk, rsd as orsd
from oracle.metrics import argmax_index, rel_l2
from paper_2608_28183_amd import nlos, runtime

from gpu_util import rsd_plan_for, say, to_dev

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-4


@pytest.fixture(scope="module")
def ctx(lib):
    return runtime.Context(0)


def load_golden(name, tau):
    g = np.load(os.path.join(GOLDEN, f"{name}.npz"), allow_pickle=False)
    assert str(g["tau_sha256"]) == scenes.checksum(tau), \
        f"{name}: the seeded input differs from the one the expected values were computed for"
    return g


def check_against_golden(g, vol, img, tol=TOL):
    assert vol.shape == tuple(g["shape"])
    e_img = rel_l2(img, g["img"])
    v = vol.ravel()[g["idx"]].astype(np.float64)
    e_smp = rel_l2(v, g["val"])
    e_abs = np.abs(v - g["val"]).max() / np.abs(g["val"]).max()
    say(f"  img rel_l2 {e_img:.2e}, sampled voxels rel_l2 {e_smp:.2e}, max abs/max {e_abs:.2e}")
    assert e_img < tol and e_smp < tol and e_abs < tol
    assert argmax_index(img) == argmax_index(g["img"])


@pytest.mark.parametrize("cname", ["c4", "c3"])
def test_fk_full_size(ctx, cname):
    cfg = scenes.CONFIGS[cname]
    tau = scenes.config_transient(cname)
    g = load_golden(f"fk_{cname}", tau)
    say(f"fk {cname} full size")
    plan = runtime.FkPlan(ctx, cfg.ny, cfg.nx, cfg.nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad)
    t = to_dev(tau)
    vol = torch.empty(cfg.shape, device="cuda")
    img = torch.empty((cfg.ny, cfg.nx), device="cuda")
    ws = plan.workspace()
    plan(t, vol, img, ws)
    torch.cuda.synchronize()
    check_against_golden(g, vol.cpu().numpy(), img.cpu().numpy())
    # the image is the max over depth of the volume, bit for bit
    assert torch.equal(vol.amax(dim=2), img)


# reduced-precision storage at full size: 10 unit roundoffs (see test_gpu_fk_prec)
@pytest.mark.parametrize("prec,tol", [("fp16", 10 * 2.0 ** -11), ("bf16", 10 * 2.0 ** -8)])
def test_fk_full_size_reduced(ctx, prec, tol):
    cfg = scenes.CONFIGS["c4"]
    tau = scenes.config_transient("c4")
    g = load_golden("fk_c4", tau)
    say(f"fk c4 full size {prec}")
    plan = runtime.FkPlan(ctx, cfg.ny, cfg.nx, cfg.nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad,
                          prec)
    vol = torch.empty(cfg.shape, device="cuda")
    img = torch.empty((cfg.ny, cfg.nx), device="cuda")
    plan(to_dev(tau), vol, img, plan.workspace())
    torch.cuda.synchronize()
    check_against_golden(g, vol.cpu().numpy(), img.cpu().numpy(), tol)
    assert torch.equal(vol.amax(dim=2), img)


def test_rsd_full_size_c3(ctx):
    cfg = scenes.CONFIGS["c3"]
    tau = scenes.config_transient("c3")
    g = load_golden("rsd_c3", tau)
    say("rsd c3 full size")
    plan, p = rsd_plan_for(ctx, cfg)
    vol = torch.empty((cfg.ny, cfg.nx, p.n_depth), device="cuda")
    img = torch.empty((cfg.ny, cfg.nx), device="cuda")
    plan(to_dev(tau), vol, img, plan.workspace())
    torch.cuda.synchronize()
    check_against_golden(g, np.moveaxis(vol.cpu().numpy(), 2, 0), img.cpu().numpy())
    assert torch.equal(vol.amax(dim=2), img)


def test_c2_raw_photons_bin_fk_rsd(ctx):
    cfg = scenes.CONFIGS["c2"]
    ev = scenes.config_events("c2", "shuffled")
    say(f"c2: {len(ev)} events -> bin -> f-k and RSD")
    d_ev = torch.from_numpy(np.frombuffer(ev.tobytes(), dtype=np.uint8).copy()).cuda()
    hist = torch.empty(cfg.shape, dtype=torch.int32, device="cuda")
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    runtime.bin_events(ctx, d_ev, len(ev), hist, int(cfg.bin_ps), 0, False, dropped)
    tau_d = torch.empty(cfg.shape, device="cuda")
    nlos.nlos_counts_to_float(ctx.handle, hist, tau_d)
    ref_h, ref_d = binning.bin_events(ev["pixel"], ev["t_ps"], cfg.nx, cfg.ny, cfg.nt, int(cfg.bin_ps))
    h = hist.cpu().numpy().view(np.uint32)
    assert np.array_equal(h.astype(np.uint64), ref_h) and int(dropped.item()) == ref_d
    tau = ref_h.astype(np.float64)
    assert np.array_equal(tau_d.cpu().numpy(), tau.astype(np.float32))

    fplan = runtime.FkPlan(ctx, cfg.ny, cfg.nx, cfg.nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad)
    vol = torch.empty(cfg.shape, device="cuda")
    img = torch.empty((cfg.ny, cfg.nx), device="cuda")
    fplan(tau_d, vol, img, fplan.workspace())
    rv, ri = ofk.fk(tau, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad)
    torch.cuda.synchronize()
    e = rel_l2(vol.cpu().numpy(), rv)
    say(f"  fk rel_l2 {e:.2e}")
    assert e < TOL and rel_l2(img.cpu().numpy(), ri) < TOL

    rplan, p = rsd_plan_for(ctx, cfg)
    rvol = torch.empty((cfg.ny, cfg.nx, p.n_depth), device="cuda")
    rimg = torch.empty((cfg.ny, cfg.nx), device="cuda")
    rplan(tau_d, rvol, rimg, rplan.workspace())
    depths = p.depth0 + p.depth_step * np.arange(p.n_depth)
    ov, oi = orsd.rsd(tau, cfg.dx, cfg.dy, cfg.bin_ps, cfg.pad, p.freq_bins, p.weights, depths)
    torch.cuda.synchronize()
    e2 = rel_l2(np.moveaxis(rvol.cpu().numpy(), 2, 0), ov)
    say(f"  rsd rel_l2 {e2:.2e}")
    assert e2 < TOL and rel_l2(rimg.cpu().numpy(), oi) < TOL
