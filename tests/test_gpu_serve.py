"""Serving loop on the GPU: concurrent mixed requests give the same results as alone.

FP32 and FP16 requests of both methods are mixed; every path is deterministic (the FP16
storage scales come from a fixed-order reduction), so results are compared bit for bit."""
import numpy as np
import pytest
import torch

import scenes
from paper_2608_28183_amd import runtime
from paper_2608_28183_amd.serve import GpuExecutor, Request, Server

from gpu_util import say

pytestmark = pytest.mark.gpu


def test_results_alone_equal_results_in_the_mix(lib):
    shapes = [(64, 64, 512), (128, 128, 1024), (256, 256, 512)]
    combos = [(m, s, p) for m in ("fk", "rsd") for s in shapes for p in ("fp32", "fp16")]
    inputs = {(s, k): torch.from_numpy(scenes.serve_input(s, 100 + k)).cuda()
              for s in shapes for k in range(2)}
    torch.cuda.synchronize()
    ex = GpuExecutor(n_slots=4, geometry=scenes.serve_geometry)
    budget = 12 << 30
    srv = Server(ex, n_slots=4, hbm_budget=budget)
    reqs = []
    for rep in range(2):
        for (m, s, p) in combos:
            for k in range(2):
                reqs.append(Request(m, s, p, tau=inputs[(s, k)]))
    # plans first (resident), then the burst
    for r in reqs:
        ex.plan(r.method, r.shape, r.precision)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    srv.start()
    futs = [srv.submit(r) for r in reqs]
    outs = [f.result(timeout=300) for f in futs]
    srv.stop()
    torch.cuda.synchronize()
    st = srv.stats.summary()
    say(f"serve burst: {st}")
    assert st["completed"] == len(reqs)
    assert srv.stats.peak_bytes <= budget
    # device memory actually held: the in-flight workspaces and outputs stay within the
    # budget; the outputs of finished requests belong to the client on top of it
    handed_out = sum(v.numel() * 4 + i.numel() * 4 for v, i in outs)
    grown = torch.cuda.max_memory_allocated() - base
    say(f"device memory growth {grown / 2**30:.2f} GiB, budget {budget / 2**30:.0f} GiB, "
        f"results handed out {handed_out / 2**30:.2f} GiB")
    assert grown <= budget + handed_out + (64 << 20)
    assert srv.stats.peak_inflight >= 2          # work from several requests overlapped

    # each request alone on one stream, the same plan
    ctx = runtime.Context(0)
    for r, (vol, img) in zip(reqs, outs):
        p = ex.plan(r.method, r.shape, r.precision)
        v1 = torch.empty_like(vol)
        i1 = torch.empty_like(img)
        p.ctx = ctx
        if r.method == "fk":
            runtime.nlos.nlos_fk(ctx.handle, p.handle, r.tau, v1, i1, p.workspace())
        else:
            runtime.nlos.nlos_rsd(ctx.handle, p.handle, r.tau, v1, i1, p.workspace())
        torch.cuda.synchronize()
        assert torch.equal(v1, vol) and torch.equal(i1, img), (r.method, r.shape, r.precision)
