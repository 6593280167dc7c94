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


# (nx, ny, nt, bin_ps, n events, invalid fraction, t0): the tile layouts of the tiled path
# (tp = 4096 // nt pixels per tile, at most 8192 tiles) and the per-event path beyond it
LAYOUTS = [
    (128, 128, 1024, 3, 3_000_000, 0.05, 0),        # 4096 tiles of 4 pixels
    (256, 256, 512, 7, 1_000_000, 0.02, 0),         # 8192 tiles of 8 pixels (the most), sparse runs
    (91, 90, 4096, 1, 400_000, 0.01, 0),            # 8190 tiles of one pixel
    (91, 90, 8192, 1, 400_000, 0.01, 0),            # nt above the tile size: per-event path
    (40, 30, 700, 4093, 2_000_000, 0.1, 12345),     # ragged last tile, odd bin width, t0
    (32, 32, 256, 5, 16_789_505, 0.01, 0),          # more than 2048 chunks: two gather rounds
    (8, 8, 64, 1, 100_000, 0.0, 0),                 # unit bin width
    (8, 8, 3, 1_431_655_765, 200_000, 0.0, 0),      # times over the whole u32 range
    (4, 4, 1, 2 ** 31 + 1, 50_000, 0.0, 0),         # bin width above 2^31
    (16, 16, 9000, 3, 500_000, 0.05, 0),            # nt > 8192: per-event atomic path
]


@pytest.mark.parametrize("nx,ny,nt,bin_ps,n,inval,t0", LAYOUTS)
def test_bin_tile_layouts(ctx, nx, ny, nt, bin_ps, n, inval, t0):
    say(f"bin layout {nx}x{ny}x{nt} bin_ps={bin_ps} n={n} invalid={inval} t0={t0}")
    ev = scenes.random_events(n, nx, ny, nt, bin_ps, seed=nx * 7 + nt, invalid_frac=inval)
    if t0:
        ev["t_ps"] = ev["t_ps"] + np.uint32(t0)
    h, d = gpu_bin(ctx, ev, nx, ny, nt, bin_ps, t0)
    ref, rd = binning.bin_events(ev["pixel"], ev["t_ps"], nx, ny, nt, bin_ps, t0)
    assert np.array_equal(h.astype(np.uint64), ref) and d == rd
