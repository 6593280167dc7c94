"""GPU complex fields and coherence-weighted merging (Section 4.4, Eq. 8-9).

The complex f-k field Psi and RSD field I against the oracle (relative L2 <= 1e-4), then
a stream of frames (the same scene under independent Poisson noise) merged on the GPU
against the oracle merge of the same GPU frames (relative L2 <= 1e-5: FP32 sums of a
few frames)."""
import numpy as np
import pytest
import torch

import scenes
from oracle import fk as ofk, merge as omerge, rsd as orsd
from oracle.metrics import rel_l2
from paper_2608_28183_amd import nlos, runtime

from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return runtime.Context(0)


def as_complex(t):
    a = t.cpu().numpy().astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def fk_field(ctx, plan, tau):
    ny, nx, nt = tau.shape
    psi = torch.empty((ny, nx, nt, 2), device="cuda")
    nlos.nlos_fk_complex(ctx.handle, plan.handle, to_dev(tau.astype(np.float32)), psi, plan.workspace())
    return psi


def test_fk_complex_field(ctx):
    cfg = scenes.CONFIGS["c1"]
    tau = scenes.config_transient("c1")
    plan = runtime.FkPlan(ctx, cfg.ny, cfg.nx, cfg.nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, 2)
    psi = as_complex(fk_field(ctx, plan, tau))
    _, _, rpsi = ofk.fk(tau.astype(np.float64), cfg.wall_w, cfg.wall_h, cfg.bin_ps, 2, return_psi=True)
    say(f"  fk field rel_l2 {rel_l2(psi, rpsi):.2e}")
    assert rel_l2(psi, rpsi) < 1e-4


def test_rsd_complex_field(ctx):
    cfg = scenes.CONFIGS["c1"]
    tau = scenes.config_transient("c1")
    p = scenes.rsd_params(cfg)
    plan = runtime.RsdPlan(ctx, cfg.ny, cfg.nx, cfg.nt, cfg.dx, cfg.dy, cfg.bin_ps, 2, p.freq_bins, p.weights,
                           p.n_depth, p.depth0, p.depth_step)
    field = torch.empty((cfg.ny, cfg.nx, p.n_depth, 2), device="cuda")
    nlos.nlos_rsd_complex(ctx.handle, plan.handle, to_dev(tau), field, plan.workspace())
    depths = p.depth0 + p.depth_step * np.arange(p.n_depth)
    _, _, Ic = orsd.rsd(tau.astype(np.float64), cfg.dx, cfg.dy, cfg.bin_ps, 2, p.freq_bins, p.weights, depths,
                        return_complex=True)
    I = np.moveaxis(as_complex(field), 2, 0)
    say(f"  rsd field rel_l2 {rel_l2(I, Ic):.2e}")
    assert rel_l2(I, Ic) < 1e-4


@pytest.mark.parametrize("window", [1, 3, 4])
def test_merge_stream(ctx, window):
    cfg = scenes.CONFIGS["c1"]
    plan = runtime.FkPlan(ctx, cfg.ny, cfg.nx, cfg.nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, 2)
    frames = [fk_field(ctx, plan, scenes.transient(cfg, seed=500 + i)) for i in range(6)]
    n = frames[0].numel() // 2
    m = nlos.nlos_merge_create(ctx.handle, n, window, 1e-6)
    try:
        ref = omerge.merge_sequence([as_complex(f) for f in frames], window, 1e-6)
        for rep in range(2):  # the second pass after a reset starts a new stream
            for i, f in enumerate(frames):
                merged = torch.full(frames[0].shape[:-1], -1.0, device="cuda")
                coh = torch.full(frames[0].shape[:-1], -1.0, device="cuda")
                nlos.nlos_merge_push(ctx.handle, m, f, merged, coh)
                torch.cuda.synchronize()
                rm, rc = ref[i]
                em, ec = rel_l2(merged.cpu().numpy(), rm), rel_l2(coh.cpu().numpy(), rc)
                assert em < 1e-5 and ec < 1e-5, (rep, i, em, ec)
                c = coh.cpu().numpy()
                # 0 <= C < 1 in exact arithmetic; in FP32 C rounds to 1 where |S| >> eps
                assert c.min() >= 0 and c.max() <= 1
            nlos.nlos_merge_reset(m)
        say(f"  window {window}: last frame rel_l2 merged {em:.2e} coherence {ec:.2e}")
    finally:
        nlos.nlos_merge_destroy(m)
