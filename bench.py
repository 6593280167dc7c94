#!/usr/bin/env python3
"""Benchmark of the NLOS hot path on one MI355X.

Default workload: f-k migration of a 256 x 256 x 512 confocal transient
(32 ps bins, 1 m wall, seeded scene of 5 planar patches and 3 spheres), zero
padded to 512 x 512 x 1024, FP32, input resident in HBM.  One step is one
complete nlos_fk call (5 kernel passes + the image clear).  Prints one JSON
line with volumes/s, the HBM roofline of the dominant kernel and the FP64
oracle's CPU throughput on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload fk_c4|fk_c3|fk_office|rsd_c3|rsd_c2|rsd_office|bin_c2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
F32_VALU_PEAK_TFLOPS = 157.3
MFMA_F16_PEAK_TFLOPS = 2500.0  # dense FP16 / BF16 matrix cores


def fk_pass_bytes(ny, nx, nt, pad, c=8, xfirst=True):
    """Algorithmic HBM bytes of each f-k pass of the schedule: every pruned intermediate
    written once and read once as c-byte complex values (8: FP32; 4: FP16 / BF16) -- half spectra
    kx <= Mx/2 up to the column pass, the z-IFFT last on the cropped ny x nx columns --
    tau read and vol written as float32.  The schedule (xfirst) runs the x-IFFT before the
    y-IFFT; the shared-spectrum mixture runs the y-IFFT first."""
    Mx, My = pad * nx, pad * ny
    Mh = Mx // 2 + 1
    nwork = (Mx // 2 - 1) * My + 2 * (My // 2 + 1)
    out = {
        "fk_x": 4 * ny * nx * nt + c * ny * Mh * nt,
        "fk_y": c * ny * Mh * nt + c * My * Mh * nt,
        "fk_column": c * nwork * nt + c * My * Mx * nt,
        "fk_zi": c * ny * nx * nt + 4 * ny * nx * nt + 4 * ny * nx,
        "fill": 4 * ny * nx,
    }
    if xfirst:
        out["fk_xi"] = c * My * Mx * nt + c * My * nx * nt
        out["fk_yi"] = c * My * nx * nt + c * ny * nx * nt
    else:
        out["fk_yi"] = c * My * Mx * nt + c * ny * Mx * nt
        out["fk_xi"] = c * ny * Mx * nt + c * ny * nx * nt
    return out


def fk_full_schedule_bytes(ny, nx, nt, pad):
    """The fixed per-volume byte count of the plain 5-pass schedule (full complex
    spectra, each pruned intermediate written and read once): 6.71 GB at 256x256x512."""
    Mx, My = pad * nx, pad * ny
    c = 8
    return (4 * ny * nx * nt + c * ny * Mx * nt) + (c * ny * Mx * nt + c * My * Mx * nt) + \
        2 * c * My * Mx * nt + (c * My * Mx * nt + c * ny * Mx * nt) + \
        (c * ny * Mx * nt + 4 * ny * nx * nt)


def rsd_pass_bytes(ny, nx, nt, pad, nf, nd, nrho, nchunks=0, kernel_bytes=8, data_bytes=8):
    """Algorithmic bytes of each RSD pass (frequency / depth contiguous layout)."""
    Mx, My = pad * nx, pad * ny
    c = data_bytes
    return {
        "rsd_phasor": 4 * ny * nx * nt + c * ny * nx * nf,
        "rsd_x": c * ny * nx * nf + c * ny * Mx * nf,
        "rsd_y": c * ny * Mx * nf + c * My * Mx * nf,
        # spectra, kernel rows (read at least once), pixel chunks and the propagated planes
        "rsd_propagate": c * My * Mx * nf + kernel_bytes * nrho * nf * nd + (4 + 12 * 64) * nchunks
        + c * My * Mx * nd,
        "rsd_yi": c * My * Mx * nd + c * ny * Mx * nd,
        "rsd_xi": c * ny * Mx * nd + 4 * ny * nx * nd + 4 * ny * nx,
        "fill": 4 * ny * nx,
    }


def moe_pass_bytes(ny, nx, nt, pad, nf, nd, nrho, shared=False):
    """Algorithmic bytes of the mixture-of-experts passes: the f-k passes (images only,
    no volume), the RSD phasors -- from the shared half spectrum (shared schedule) or the
    transient followed by the x and y passes (branches in sequence) -- the RSD
    propagation and inverse passes (image only) and the mixture."""
    Mx, My = pad * nx, pad * ny
    fk = fk_pass_bytes(ny, nx, nt, pad, xfirst=not shared)
    fk["fk_zi"] = 8 * ny * nx * nt + 4 * ny * nx
    rsd = rsd_pass_bytes(ny, nx, nt, pad, nf, nd, nrho)
    out = {k: fk[k] for k in ("fk_x", "fk_y", "fk_column", "fk_yi", "fk_xi", "fk_zi")}
    if shared:
        out["moe_phasor"] = 8 * My * (Mx // 2 + 1) * nt + 8 * My * Mx * nf
    else:
        for k in ("rsd_phasor", "rsd_x", "rsd_y"):
            out[k] = rsd[k]
    out["rsd_propagate"] = rsd["rsd_propagate"]
    out["rsd_yi"] = rsd["rsd_yi"]
    out["rsd_xi"] = 8 * ny * Mx * nd + 4 * ny * nx
    out["moe_mix"] = 4 * 4 * ny * nx
    out["fill"] = 8 * ny * nx
    return out


def cpu_baseline_fk(cfg, fraction=2):
    """The FP64 oracle, untuned, on a bounded sample of the f-k workload: each oracle
    step runs on 1/fraction of its independent slices of the full-size padded volume
    (random data of the same shape: the matrix-DFT cost does not depend on values),
    and the per-volume time is the sum of the steps scaled by `fraction`."""
    import numpy as np
    from oracle import fk as ofk
    from oracle.dft import dft
    ny, nx, nt, pad = cfg.ny, cfg.nx, cfg.nt, cfg.pad
    My, Mx, Mt = pad * ny, pad * nx, pad * nt
    rng = np.random.default_rng(0)
    t_total = 0.0
    tau = rng.poisson(2.0, size=(ny // fraction, nx, nt)).astype(np.float64)
    t = time.perf_counter(); G = ofk.scale_and_pad(tau, pad); t_total += time.perf_counter() - t
    sub = (My // fraction, Mx, Mt)
    X = rng.normal(size=sub) + 1j * rng.normal(size=sub)
    for ax in (2, 1):
        for inv in (False, True):
            t = time.perf_counter(); dft(X, ax, inverse=inv); t_total += time.perf_counter() - t
    suby = (My, Mx // fraction, Mt)
    Y = rng.normal(size=suby) + 1j * rng.normal(size=suby)
    for inv in (False, True):
        t = time.perf_counter(); dft(Y, 0, inverse=inv); t_total += time.perf_counter() - t
    sx, sy = ofk.stolt_constants(cfg.dx, cfg.dy, cfg.bin_ps)
    t = time.perf_counter(); out = ofk.stolt(X, sx, sy); t_total += time.perf_counter() - t
    t = time.perf_counter(); v = np.abs(out[:, :nx, :nt]) ** 2; v.max(axis=2); t_total += time.perf_counter() - t
    del G, X, Y, out, v
    return t_total * fraction, t_total


def serve_bench(n_requests=2000, rate_hz=50.0, n_slots=4, budget_gib=24, seed=5005, n_saturation=1000):
    """Poisson stream of mixed reconstructions through the continuous-batching loop:
    shapes uniform over {64x64x512, 128x128x1024, 256x256x512}, f-k / RSD 50/50; runs
    all FP32, all FP16 and 50/50 mixed (2000 requests each, about 40 s at 50/s), and a
    saturation run (1000 requests at 2000/s) under a 16 GiB budget."""
    import torch

    import scenes
    from paper_2608_28183_amd.serve import GpuExecutor, Request, Server, run_stream

    ex = GpuExecutor(n_slots=n_slots, geometry=scenes.serve_geometry)
    inputs = {}
    for s in scenes.SERVE_SHAPES:
        for k in range(2):
            inputs[(s, k)] = torch.from_numpy(scenes.serve_input(s, 200 + k)).cuda()
    for s in scenes.SERVE_SHAPES:
        for m in ("fk", "rsd"):
            for p in ("fp32", "fp16"):
                ex.plan(m, s, p)
    torch.cuda.synchronize()

    def one_run(precisions, rate, budget, n):
        stream = scenes.request_stream(n, rate, seed=seed, precisions=precisions)
        arr = []
        for r in stream:
            prec = r["precision"]
            arr.append((r["arrival_s"], Request(r["method"], tuple(r["shape"]), prec,
                                                tau=inputs[(tuple(r["shape"]), r["id"] % 2)])))
        srv = Server(ex, n_slots=n_slots, hbm_budget=budget << 30).start()
        run_stream(srv, arr)
        srv.stop()
        s = srv.stats.summary()
        return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in s.items()}

    one_run(("fp32",), 1000.0, budget_gib, 12)  # warm-up: allocator pools, code paths
    return {
        "arrival_rate_hz": rate_hz, "requests": n_requests, "slots": n_slots,
        "saturation_requests": n_saturation,
        "mix": "shapes uniform over 64x64x512, 128x128x1024, 256x256x512; f-k/RSD 50/50; "
               "fp16 = FP16 f-k intermediates, FP16 RSD intermediates and kernel",
        "fp32": one_run(("fp32",), rate_hz, budget_gib, n_requests),
        "fp16": one_run(("fp16",), rate_hz, budget_gib, n_requests),
        "fp32_fp16_mixed": one_run(("fp32", "fp16"), rate_hz, budget_gib, n_requests),
        "saturation_2000hz_16GiB": one_run(("fp32",), 2000.0, 16, n_saturation),
    }


def per_call_ms(step, n, stream):
    """Durations of n back-to-back calls, each bracketed by HIP events on the launch stream."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    import numpy as np
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return {"calls": n, "p50_ms": round(float(np.percentile(t, 50)), 4),
            "p99_ms": round(float(np.percentile(t, 99)), 4), "mean_ms": round(float(t.mean()), 4)}


def golden_accuracy(name, vol, img):
    """Error of a full-size output against the FP64 oracle values stored under tests/golden/
    (written by tests/golden/make_golden.py from the oracle): the whole max-over-depth
    image and 4096 sampled voxels (the 1024 largest and 3072 random), relative L2, max
    |error| / max |reference| and whether the image arg-max agrees."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{name}.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path, allow_pickle=False)
    im = img.detach().cpu().numpy().astype(np.float64)
    v = vol.detach().reshape(-1)[__import__("torch").from_numpy(g["idx"]).to(vol.device)].cpu().numpy()
    ri, rv = g["img"].astype(np.float64), g["val"]

    def rl2(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return {"img_rel_l2": rl2(im, ri), "img_max_rel": float(np.abs(im - ri).max() / np.abs(ri).max()),
            "sampled_voxels_rel_l2": rl2(v, rv), "sampled_voxels_max_rel": float(np.abs(v - rv).max() / np.abs(rv).max()),
            "img_argmax_equal": bool(np.argmax(im) == np.argmax(ri)), "reference": "FP64 oracle"}


def copy_calibration(args):
    """torch's device copy of 1 GiB (256 Mi float32): 1 GiB read + 1 GiB written per
    launch; prints its bandwidth.  Under rocprofv3 --pmc its FETCH_SIZE and WRITE_SIZE
    give the counter-to-bytes factor used for the other workloads."""
    import torch
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    print(json.dumps({"metric": "copy_GBps", "value": round(2 * 4 * n / sec / 1e9, 1), "unit": "GB/s",
                      "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                      "steps": args.steps, "ms_per_step": round(sec * 1e3, 4)}), flush=True)


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"]
        return max(n) if n else None
    except Exception:
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="fk_c4",
                    choices=["fk_c4", "fk_c3", "fk_c1", "fk_office", "rsd_c3", "rsd_c2", "rsd_office", "bin_c2", "phasor_c2", "moe_c4",
                             "moe_c3", "merge_c4", "dda_c3", "copy_1GiB"],
                    help="copy_1GiB: a plain device copy of 1 GiB, the reference that the HBM "
                         "byte counters of the other workloads are scaled by")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp16", "bf16"],
                    help="storage precision of the complex intermediates (RSD: and of the radial "
                         "kernel, FP16 / BF16 propagating on the matrix cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import scenes
    from paper_2608_28183_amd import nlos, runtime

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    kind, cname = args.workload.split("_")
    if kind == "copy":
        copy_calibration(args)
        return
    cfg = scenes.CONFIGS[cname]
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    ctx = runtime.Context(0, stream)
    ny, nx, nt = cfg.ny, cfg.nx, cfg.nt
    print(f"[bench] workload {args.workload}: generating input", file=sys.stderr, flush=True)

    if kind == "fk":
        tau = torch.from_numpy(scenes.config_transient(cname)).to(dev)
        plan = runtime.FkPlan(ctx, ny, nx, nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad, args.prec)
        ws = plan.workspace()
        vol = torch.empty((ny, nx, nt), device=dev)
        img = torch.empty((ny, nx), device=dev)
        step = lambda: plan(tau, vol, img, ws)  # noqa: E731
        pass_bytes = fk_pass_bytes(ny, nx, nt, cfg.pad, 8 if args.prec == "fp32" else 4)
        if args.prec == "fp16":
            pass_bytes["fk_scale"] = 4 * ny * nx * nt  # the bound's read of tau
        metric, unit = "fk_volumes_per_s", "volumes/s"
        units_per_step = 1
        workload = {"workload": f"f-k migration {ny}x{nx}x{nt} padded x{cfg.pad} "
                                f"to {cfg.pad*ny}x{cfg.pad*nx}x{cfg.pad*nt}",
                    "shape": [ny, nx, nt], "pad": cfg.pad, "bin_ps": cfg.bin_ps, "wall_m": cfg.wall_w,
                    "scene": cfg.scene, "precision": args.prec}
    elif kind == "rsd":
        tau = torch.from_numpy(scenes.config_transient(cname) if cname != "c2"
                               else scenes.transient(cfg)).to(dev)
        p = scenes.rsd_params(cfg)
        plan = runtime.RsdPlan(ctx, ny, nx, nt, cfg.dx, cfg.dy, cfg.bin_ps, cfg.pad, p.freq_bins,
                               p.weights, p.n_depth, p.depth0, p.depth_step, data_prec=args.prec,
                               kernel_prec=args.prec)
        ws = plan.workspace()
        vol = torch.empty((ny, nx, p.n_depth), device=dev)
        img = torch.empty((ny, nx), device=dev)
        step = lambda: plan(tau, vol, img, ws)  # noqa: E731
        g = nlos.nlos_rsd_geometry_get(plan.desc)
        pass_bytes = rsd_pass_bytes(ny, nx, nt, cfg.pad, len(p.freq_bins), p.n_depth, g["n_rho"],
                                    kernel_bytes=8 if args.prec == "fp32" else 4,
                                    data_bytes=8 if args.prec == "fp32" else 4)
        if args.prec == "fp16":
            pass_bytes["rsd_scale"] = 4 * ny * nx * nt  # the bound's read of tau
        # the propagation's arithmetic: per padded pixel, frequency, depth and radial tap one
        # complex multiply-add (8 flops)
        prop_flops = 16 * (cfg.pad * ny) * (cfg.pad * nx) * len(p.freq_bins) * p.n_depth
        metric, unit = "rsd_volumes_per_s", "volumes/s"
        units_per_step = 1
        workload = {"workload": f"radial RSD {ny}x{nx}x{nt} padded x{cfg.pad}, "
                                f"{len(p.freq_bins)} freqs, {p.n_depth} depths",
                    "shape": [ny, nx, nt], "pad": cfg.pad, "n_freq": len(p.freq_bins),
                    "n_depth": p.n_depth}
    elif kind == "moe":
        tau = torch.from_numpy(scenes.config_transient(cname)).to(dev)
        p = scenes.rsd_params(cfg)
        plan = runtime.MoePlan(ctx, ny, nx, nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad,
                               p.freq_bins, p.weights, p.n_depth, p.depth0, p.depth_step)
        ws = plan.workspace()
        img = torch.empty((ny, nx), device=dev)
        step = lambda: plan(tau, img, None, None, ws)  # noqa: E731
        g = nlos.nlos_rsd_geometry_get(plan.rsd_desc)
        nf = len(p.freq_bins)
        pass_bytes = moe_pass_bytes(ny, nx, nt, cfg.pad, nf, p.n_depth, g["n_rho"])
        metric, unit = "moe_images_per_s", "images/s"
        units_per_step = 1
        workload = {"workload": f"mixture of experts f-k x RSD (Eq. 10, beta 0.3) on {ny}x{nx}x{nt} "
                                f"padded x{cfg.pad}, RSD {nf} freqs x {p.n_depth} depths",
                    "shape": [ny, nx, nt], "pad": cfg.pad, "n_freq": nf, "n_depth": p.n_depth}
        # the same two reconstructions run separately, for comparison
        fkp = runtime.FkPlan(ctx, ny, nx, nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad)
        rsp = runtime.RsdPlan(ctx, ny, nx, nt, cfg.dx, cfg.dy, cfg.bin_ps, cfg.pad, p.freq_bins,
                              p.weights, p.n_depth, p.depth0, p.depth_step)
        ws2 = torch.empty(max(fkp.ws_bytes, rsp.ws_bytes), dtype=torch.uint8, device=dev)
        im2 = torch.empty((ny, nx), device=dev)

        def separate():
            fkp(tau, None, im2, ws2)
            rsp(tau, None, im2, ws2)

        shp = runtime.MoePlan(ctx, ny, nx, nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad,
                              p.freq_bins, p.weights, p.n_depth, p.depth0, p.depth_step,
                              shared_spectrum=True)

        def shared():
            shp(tau, im2, None, None, ws)
    elif kind == "merge":
        # one frame = the complex f-k field of a transient, then coherence merging over the
        # last 3 frames (Eq. 8-9); the input alternates between two noise draws
        taus = [torch.from_numpy(scenes.config_transient(cname)).to(dev),
                torch.from_numpy(scenes.transient(cfg, seed=cfg.seed + 1)).to(dev)]
        plan = runtime.FkPlan(ctx, ny, nx, nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad)
        ws = plan.workspace()
        psi = torch.empty((ny, nx, nt, 2), device=dev)
        merged = torch.empty((ny, nx, nt), device=dev)
        coh = torch.empty((ny, nx, nt), device=dev)
        window = 3
        mstate = nlos.nlos_merge_create(ctx.handle, ny * nx * nt, window, 1e-6)
        counter = [0]

        def step():
            nlos.nlos_fk_complex(ctx.handle, plan.handle, taus[counter[0] & 1], psi, ws)
            nlos.nlos_merge_push(ctx.handle, mstate, psi, merged, coh)
            counter[0] += 1
        pass_bytes = fk_pass_bytes(ny, nx, nt, cfg.pad)
        pass_bytes["fk_zi"] = 16 * ny * nx * nt
        pass_bytes["merge"] = (8 + 8 + 8 * (window - 1) + 8) * ny * nx * nt
        metric, unit = "merged_fk_volumes_per_s", "volumes/s"
        units_per_step = 1
        workload = {"workload": f"complex f-k field {ny}x{nx}x{nt} padded x{cfg.pad} + coherence merging "
                                f"over {window} frames", "shape": [ny, nx, nt], "window": window}
    elif kind == "dda":
        # one frame = a radial RSD volume, then the depth-dependent average over the last 3
        # volumes with the default table; the input alternates between two noise draws
        taus = [torch.from_numpy(scenes.config_transient(cname)).to(dev),
                torch.from_numpy(scenes.transient(cfg, seed=cfg.seed + 1)).to(dev)]
        p = scenes.rsd_params(cfg)
        plan = runtime.RsdPlan(ctx, ny, nx, nt, cfg.dx, cfg.dy, cfg.bin_ps, cfg.pad, p.freq_bins,
                               p.weights, p.n_depth, p.depth0, p.depth_step)
        ws = plan.workspace()
        vol = torch.empty((ny, nx, p.n_depth), device=dev)
        avg = torch.empty((ny, nx, p.n_depth), device=dev)
        img = torch.empty((ny, nx), device=dev)
        window = 3
        table = nlos.nlos_dda_default_weights(p.n_depth, window)
        dstate = nlos.nlos_dda_create(ctx.handle, ny * nx, p.n_depth, window, table)
        counter = [0]

        def step():
            plan(taus[counter[0] & 1], vol, None, ws)
            nlos.nlos_dda_push(ctx.handle, dstate, vol, avg, img)
            counter[0] += 1
        g = nlos.nlos_rsd_geometry_get(plan.desc)
        pass_bytes = rsd_pass_bytes(ny, nx, nt, cfg.pad, len(p.freq_bins), p.n_depth, g["n_rho"])
        # new volume read, ring slot and average written, the older frames of non-zero weight
        # read, the image written
        older = sum(sum(1 for w in row[1:] if w != 0.0) for row in table)
        pass_bytes["dda"] = 4 * ny * nx * (3 * p.n_depth + older + 1)
        metric, unit = "dda_rsd_volumes_per_s", "volumes/s"
        units_per_step = 1
        workload = {"workload": f"radial RSD {ny}x{nx}x{nt} padded x{cfg.pad}, {p.n_depth} depths, then the "
                                f"depth-dependent average over {window} volumes",
                    "shape": [ny, nx, nt], "n_depth": p.n_depth, "window": window}
    elif kind == "phasor":
        ev = scenes.config_events(cname, "shuffled")
        d_ev = torch.from_numpy(np.frombuffer(ev.tobytes(), dtype=np.uint8).copy()).to(dev)
        p = scenes.rsd_params(cfg)
        nf = len(p.freq_bins)
        pplan = nlos.nlos_phasor_plan_create(ctx.handle, nlos.bin_desc(nx, ny, nt, int(cfg.bin_ps), 0, False),
                                             p.freq_bins)
        P = torch.empty((ny, nx, nf, 2), device=dev)
        dropped = torch.zeros(1, dtype=torch.int64, device=dev)
        n = len(ev)
        step = lambda: nlos.nlos_phasor_bin(ctx.handle, pplan, d_ev, n, P, dropped)  # noqa: E731
        pass_bytes = {"phasor_bin": 8 * n + 8 * ny * nx * nf, "fill": 8 * ny * nx * nf}
        metric, unit = "phasor_events_per_s", "events/s"
        units_per_step = n
        workload = {"workload": f"phasor binning of {n} events into {ny}x{nx} pixels x {nf} frequencies "
                                f"(nt {nt})", "n_events": n, "shape": [ny, nx, nt], "n_freq": nf}
        # photons -> RSD volume both ways: direct phasors, or histogram then the phasor DFT
        rplan = runtime.RsdPlan(ctx, ny, nx, nt, cfg.dx, cfg.dy, cfg.bin_ps, cfg.pad, p.freq_bins,
                                p.weights, p.n_depth, p.depth0, p.depth_step)
        rws = rplan.workspace()
        rvol = torch.empty((ny, nx, p.n_depth), device=dev)
        rimg = torch.empty((ny, nx), device=dev)
        hist = torch.empty((ny, nx, nt), dtype=torch.int32, device=dev)
        tau_h = torch.empty((ny, nx, nt), device=dev)

        def via_phasors():
            nlos.nlos_phasor_bin(ctx.handle, pplan, d_ev, n, P, dropped)
            nlos.nlos_rsd_from_phasors(ctx.handle, rplan.handle, P, rvol, rimg, rws)

        def via_histogram():
            runtime.bin_events(ctx, d_ev, n, hist, int(cfg.bin_ps), 0, False, dropped)
            nlos.nlos_counts_to_float(ctx.handle, hist, tau_h)
            rplan(tau_h, rvol, rimg, rws)
    else:  # bin
        ev = scenes.config_events(cname, "shuffled")
        d_ev = torch.from_numpy(np.frombuffer(ev.tobytes(), dtype=np.uint8).copy()).to(dev)
        hist = torch.empty((ny, nx, nt), dtype=torch.int32, device=dev)
        dropped = torch.zeros(1, dtype=torch.int64, device=dev)
        n = len(ev)
        step = lambda: runtime.bin_events(ctx, d_ev, n, hist, int(cfg.bin_ps), 0, False, dropped)  # noqa
        pass_bytes = {"bin": 8 * n + 4 * ny * nx * nt, "fill": 4 * ny * nx * nt}
        metric, unit = "events_per_s", "events/s"
        units_per_step = n
        workload = {"workload": f"photon binning of {n} events into {ny}x{nx}x{nt}",
                    "n_events": n, "shape": [ny, nx, nt]}

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: K back-to-back steps on one stream
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / args.steps
    value = units_per_step / sec

    # per-pass kernel durations from HIP events on the launch stream, same K steps
    nlos.nlos_timing_enable(ctx.handle, True)
    for _ in range(args.steps):
        step()
    passes = nlos.nlos_timing_read(ctx.handle)
    nlos.nlos_timing_enable(ctx.handle, False)
    avg_ms = {k: v[0] / v[1] for k, v in passes.items()}
    dom = max((k for k in avg_ms if k in pass_bytes and k != "fill"), key=lambda k: avg_ms[k])
    achieved = pass_bytes[dom] / (avg_ms[dom] * 1e-3) / 1e9
    traffic = None
    prof_path = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(prof_path):
        try:
            from paper_2608_28183_amd import build as _b
            prof = json.load(open(prof_path))
            key = f"{args.workload}:{args.prec if kind == 'fk' else 'fp32'}:{dom}"
            rec = prof.get("entries", {}).get(key)
            # counters taken from other kernel code do not describe this one
            if rec and prof.get("source_sha") == _b.source_sha():
                traffic = rec["bytes_per_launch"]
        except Exception:
            traffic = None
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes": pass_bytes[dom], "avg_ms": round(avg_ms[dom], 4)}
    if kind == "rsd" and dom == "rsd_propagate":
        # the propagation is a contraction: priced against the arithmetic peak it runs on
        # (matrix cores for FP16 / BF16 kernels, FP32 FMAs otherwise), bytes kept beside
        tflops = prop_flops / (avg_ms[dom] * 1e-3) / 1e12
        on_fma = os.environ.get("NLOS_RSD_MFMA", "1") == "0"
        # FP32 matrix cores and FP32 vector FMAs share the published 157.3 TFLOP/s
        peak = MFMA_F16_PEAK_TFLOPS if args.prec != "fp32" else F32_VALU_PEAK_TFLOPS
        roofline = {"bound": "alu" if on_fma else "mfma", "kernel": dom,
                    "achieved": round(tflops, 2), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(tflops / peak, 4), "traffic": traffic, "algorithmic_flops": prop_flops,
                    "avg_ms": round(avg_ms[dom], 4), "hbm_GBps": round(achieved, 1),
                    "hbm_frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes": pass_bytes[dom]}
    total_alg = sum(v for k, v in pass_bytes.items())
    print(f"[bench] {args.steps} steps: {sec*1e3:.3f} ms/step; passes (avg ms): "
          + ", ".join(f"{k} {v:.3f}" for k, v in avg_ms.items()), file=sys.stderr, flush=True)

    # per-call latency of the step (HIP events around each call, back to back)
    per_call = per_call_ms(step, max(100, args.steps), stream)
    accuracy = None
    precision_path = None
    if kind == "fk":
        step()
        torch.cuda.synchronize()
        accuracy = golden_accuracy(f"fk_{cname}", vol, img)
        if args.prec == "fp32":
            # the reduced-precision storage forms of the same step (FP16 / BF16 intermediates,
            # DFT stages on the matrix cores): volumes/s, per-call latency and accuracy
            precision_path = {}
            for pr in ("fp16", "bf16"):
                try:
                    pp = runtime.FkPlan(ctx, ny, nx, nt, cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad, pr)
                except nlos.NlosError as e:  # e.g. mixed-radix grids: FP32 only
                    precision_path[pr] = {"unsupported": str(e)}
                    continue
                pws = pp.workspace()
                pstep = lambda: pp(tau, vol, img, pws)  # noqa: E731
                for _ in range(args.warmup):
                    pstep()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    pstep()
                torch.cuda.synchronize()
                psec = (time.perf_counter() - t0) / args.steps
                pc = per_call_ms(pstep, max(100, args.steps), stream)
                pstep()
                torch.cuda.synchronize()
                precision_path[pr] = {"value": round(1.0 / psec, 3), "unit": unit, "ms_per_step": round(psec * 1e3, 4),
                                      "speedup_vs_fp32": round(sec / psec, 3),
                                      "step_bytes": sum(fk_pass_bytes(ny, nx, nt, cfg.pad, 4).values()),
                                      "per_call": pc, "accuracy": golden_accuracy(f"fk_{cname}", vol, img)}
                del pws
            step()  # leave the FP32 result in vol / img
            torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline and kind == "fk":
        try:
            frac = 1
            est, spent = cpu_baseline_fk(cfg, frac)
            cpu = {"value": round(1.0 / est, 6), "unit": unit, "cores": blas_threads() or
                   len(os.sched_getaffinity(0)), "kind": "oracle",
                   "sample": f"every FP64 oracle step once on the full {cfg.pad*ny}x{cfg.pad*nx}x{cfg.pad*nt} "
                             f"padded volume (random data of the same shape) "
                             f"({spent:.1f} s of CPU time measured)",
                   "host_cpus": len(os.sched_getaffinity(0))}
        except MemoryError:
            cpu = None

    serving = None
    if not args.no_serve and kind == "fk":
        print("[bench] serving run", file=sys.stderr, flush=True)
        serving = serve_bench()

    moe_cmp = None
    if kind == "moe":
        def clock(fn):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / args.steps
        sep, sh = clock(separate), clock(shared)
        moe_cmp = {"moe_branches_in_sequence_ms": round(sec * 1e3, 4),
                   "moe_shared_spectrum_ms": round(sh * 1e3, 4),
                   "separate_fk_then_rsd_ms": round(sep * 1e3, 4), "speedup_vs_separate": round(sep / sec, 3)}

    phasor_cmp = None
    if kind == "phasor":
        def clock2(fn):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / args.steps
        phasor_cmp = {"photons_to_rsd_via_phasor_binning_ms": round(clock2(via_phasors) * 1e3, 4),
                      "photons_to_rsd_via_histogram_ms": round(clock2(via_histogram) * 1e3, 4)}

    # the same step as one replayed HIP graph (same buffers), against the eager launches
    graph_cmp = None
    if kind in ("fk", "rsd"):
        g = plan.graph(tau, vol, img, ws)
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        gsec = (time.perf_counter() - t0) / args.steps
        g.close()
        graph_cmp = {"eager_ms": round(sec * 1e3, 4), "graph_replay_ms": round(gsec * 1e3, 4),
                     "speedup": round(sec / gsec, 4)}

    line = {
        "metric": metric, "value": round(value, 3), "unit": unit, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.prec == "fp32" else args.prec, "data": "synthetic",
        "config": workload, "roofline": roofline, "cpu_baseline": cpu,
        "per_call": per_call, "accuracy": accuracy, "precision_path": precision_path,
        "passes_ms": {k: round(v, 4) for k, v in avg_ms.items()},
        "serving": serving,
        "moe_vs_separate": moe_cmp,
        "phasor_vs_histogram": phasor_cmp,
        "graph_vs_eager": graph_cmp,
        "step_frac_of_hbm": round(total_alg * value / units_per_step / (HBM_PEAK_GBS * 1e9), 4),
        "step_bytes": total_alg,
    }
    if kind == "fk":
        fixed = fk_full_schedule_bytes(ny, nx, nt, cfg.pad)
        line["fixed_schedule_bytes"] = fixed
        line["fixed_schedule_frac_of_hbm"] = round(fixed * value / (HBM_PEAK_GBS * 1e9), 4)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
