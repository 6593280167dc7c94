"""GPU parity of nlos_bin against the oracle: bit-exact."""
import numpy as np
import pytest
import torch

import scenes
from oracle import binning
from paper_2608_28183_amd import runtime

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return runtime.Context(0)


def gpu_bin(ctx, ev, nx, ny, nt, bin_ps, t0=0, hist0=None):
    n = len(ev)
    raw = np.frombuffer(ev.tobytes(), dtype=np.uint8) if n else np.zeros(8, np.uint8)
    d_ev = torch.from_numpy(raw.copy()).cuda()
    if hist0 is None:
        hist = torch.full((ny, nx, nt), 12345, dtype=torch.int32, device="cuda")
        acc = False
    else:
        hist = torch.from_numpy(hist0.astype(np.int64).astype(np.int32)).cuda()
        acc = True
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda")
    runtime.bin_events(ctx, d_ev, n, hist, bin_ps, t0, acc, dropped)
    torch.cuda.synchronize()
    return hist.cpu().numpy().view(np.uint32), int(dropped.item())


@pytest.mark.parametrize("order", ["shuffled", "pixel"])
def test_bin_c2_bit_exact(ctx, order):
    cfg = scenes.CONFIGS["c2"]
    ev = scenes.config_events("c2", order)
    say(f"bin c2 {order} n={len(ev)}")
    h, d = gpu_bin(ctx, ev, cfg.nx, cfg.ny, cfg.nt, int(cfg.bin_ps))
    ref, rd = binning.bin_events(ev["pixel"], ev["t_ps"], cfg.nx, cfg.ny, cfg.nt, int(cfg.bin_ps))
    assert np.array_equal(h.astype(np.uint64), ref)
    assert d == rd
    assert int(h.sum(dtype=np.uint64)) + d == len(ev)


@pytest.mark.parametrize("n,inval,t0", [(0, 0.0, 0), (1, 0.0, 0), (1000003, 0.3, 0),
                                        (65, 1.0, 0), (50000, 0.1, 77)])
def test_bin_edges(ctx, n, inval, t0):
    say(f"bin edge n={n} invalid={inval} t0={t0}")
    ev = scenes.random_events(n, 5, 3, 7, 13, seed=n + 1, invalid_frac=inval)
    if n:
        ev["t_ps"] = ev["t_ps"] + np.uint32(t0)
    h, d = gpu_bin(ctx, ev, 5, 3, 7, 13, t0)
    ref, rd = binning.bin_events(ev["pixel"], ev["t_ps"], 5, 3, 7, 13, t0)
    assert np.array_equal(h.astype(np.uint64), ref) and d == rd


def test_bin_accumulate(ctx):
    ev = scenes.random_events(20000, 8, 8, 16, 10, seed=3, invalid_frac=0.05)
    h1, _ = gpu_bin(ctx, ev[:7000], 8, 8, 16, 10)
    h2, d2 = gpu_bin(ctx, ev[7000:], 8, 8, 16, 10, hist0=h1)
    ref, rd = binning.bin_events(ev["pixel"], ev["t_ps"], 8, 8, 16, 10)
    _, rd2 = binning.bin_events(ev["pixel"][7000:], ev["t_ps"][7000:], 8, 8, 16, 10)
    assert np.array_equal(h2.astype(np.uint64), ref) and d2 == rd2


def test_bin_hot_bin_aggregation(ctx):
    # every event in one bin: exercises the wave-merged atomics
    ev = np.zeros(300001, dtype=scenes.EVENT_DTYPE)
    ev["pixel"] = 5
    ev["t_ps"] = 33
    h, d = gpu_bin(ctx, ev, 4, 4, 8, 10)
    assert h[1, 1, 3] == 300001 and h.sum() == 300001 and d == 0
