"""Tensor-level helpers over the C ABI: contexts, plans and workspace as torch
device memory.  Marshalling only -- every step runs in libnlos kernels."""
from __future__ import annotations

import torch

from . import nlos

EVENT_BYTES = 8


class Context:
    """An nlos context bound to one device and stream."""

    def __init__(self, device: int = 0, stream: "torch.cuda.Stream | None" = None):
        if not torch.cuda.is_available():
            raise RuntimeError("libnlos needs a HIP device")
        self.device = torch.device("cuda", device)
        self.stream = stream
        self.handle = nlos.nlos_create(device, stream)

    def set_stream(self, stream) -> None:
        self.stream = stream
        nlos.nlos_set_stream(self.handle, stream)

    def close(self) -> None:
        if self.handle:
            nlos.nlos_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """One reconstruction captured with fixed buffers (nlos_*_graph_create); replay()
    runs it on the context's stream.  The buffers are held for the graph's lifetime:
    write new inputs into ``tau`` and read results from ``vol`` / ``img`` between replays."""

    def __init__(self, ctx: Context, handle: int, tau, vol, img, ws, plan):
        self.ctx, self.handle = ctx, handle
        self.tau, self.vol, self.img, self.ws, self.plan = tau, vol, img, ws, plan

    def replay(self) -> None:
        nlos.nlos_graph_launch(self.ctx.handle, self.handle)

    def close(self) -> None:
        if self.handle:
            nlos.nlos_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FkPlan:
    def __init__(self, ctx: Context, ny: int, nx: int, nt: int, wall_w: float, wall_h: float,
                 bin_ps: float, pad: int = 2, prec: str = "fp32"):
        self.ctx = ctx
        self.shape = (ny, nx, nt)
        self.desc = nlos.fk_desc(nx, ny, nt, wall_w, wall_h, bin_ps, pad, prec)
        self.handle = nlos.nlos_fk_plan_create(ctx.handle, self.desc)
        self.ws_bytes = nlos.nlos_fk_workspace_bytes(self.handle)

    def workspace(self) -> torch.Tensor:
        return torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.ctx.device)

    def __call__(self, tau: torch.Tensor, vol=None, img=None, ws=None):
        ny, nx, nt = self.shape
        assert tau.shape == (ny, nx, nt) and tau.dtype == torch.float32 and tau.is_cuda
        nlos.nlos_fk(self.ctx.handle, self.handle, tau, vol, img, ws)
        return vol, img

    def graph(self, tau: torch.Tensor, vol=None, img=None, ws=None) -> Graph:
        """This plan's reconstruction of these buffers as a replayable graph."""
        ws = self.workspace() if ws is None else ws
        h = nlos.nlos_fk_graph_create(self.ctx.handle, self.handle, tau, vol, img, ws)
        return Graph(self.ctx, h, tau, vol, img, ws, self)

    def __del__(self):
        try:
            nlos.nlos_fk_plan_destroy(self.handle)
        except Exception:
            pass


class RsdPlan:
    def __init__(self, ctx: Context, ny: int, nx: int, nt: int, dx: float, dy: float, bin_ps: float,
                 pad: int, freq_bins, weights, n_depth: int, depth0: float, depth_step: float,
                 sigma_s: int = 2, sigma_t: int = 0, delta: float = 0.0, data_prec: str = "fp32",
                 kernel_prec: str = "fp32", vol_depth_major: bool = False):
        self.ctx = ctx
        self.shape = (ny, nx, nt)
        self.n_depth = n_depth
        self.depth_major = bool(vol_depth_major)
        self.desc = nlos.RsdDesc(nx, ny, nt, dx, dy, bin_ps, pad, freq_bins, weights, n_depth,
                                 depth0, depth_step, sigma_s, sigma_t, delta, data_prec,
                                 kernel_prec, vol_depth_major)
        self.handle = nlos.nlos_rsd_plan_create(ctx.handle, self.desc)
        self.ws_bytes = nlos.nlos_rsd_workspace_bytes(self.handle)

    def workspace(self) -> torch.Tensor:
        return torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.ctx.device)

    def __call__(self, tau: torch.Tensor, vol=None, img=None, ws=None):
        """vol: float32 [ny, nx, n_depth] (depth contiguous) or, for a depth-major plan,
        [n_depth, ny, nx]; img: float32 [ny, nx]."""
        ny, nx, nt = self.shape
        assert tau.shape == (ny, nx, nt) and tau.dtype == torch.float32 and tau.is_cuda
        want = (self.n_depth, ny, nx) if self.depth_major else (ny, nx, self.n_depth)
        assert vol is None or vol.shape == want
        nlos.nlos_rsd(self.ctx.handle, self.handle, tau, vol, img, ws)
        return vol, img

    def graph(self, tau: torch.Tensor, vol=None, img=None, ws=None) -> Graph:
        """This plan's reconstruction of these buffers as a replayable graph."""
        ws = self.workspace() if ws is None else ws
        h = nlos.nlos_rsd_graph_create(self.ctx.handle, self.handle, tau, vol, img, ws)
        return Graph(self.ctx, h, tau, vol, img, ws, self)

    def __del__(self):
        try:
            nlos.nlos_rsd_plan_destroy(self.handle)
        except Exception:
            pass


class MoePlan:
    """Mixture of experts (Section 4.4, Eq. 10) of f-k and radial RSD on one transient."""

    def __init__(self, ctx: Context, ny: int, nx: int, nt: int, wall_w: float, wall_h: float,
                 bin_ps: float, pad: int, freq_bins, weights, n_depth: int, depth0: float,
                 depth_step: float, beta: float = 0.3, eps: float = 1e-6, sigma_s: int = 2,
                 sigma_t: int = 0, delta: float = 0.0, kernel_prec: str = "fp32",
                 shared_spectrum: bool = False):
        self.ctx = ctx
        self.shape = (ny, nx, nt)
        self.fk_desc = nlos.fk_desc(nx, ny, nt, wall_w, wall_h, bin_ps, pad, "fp32")
        self.rsd_desc = nlos.RsdDesc(nx, ny, nt, wall_w / nx, wall_h / ny, bin_ps, pad, freq_bins,
                                     weights, n_depth, depth0, depth_step, sigma_s, sigma_t, delta,
                                     "fp32", kernel_prec)
        self.ws_bytes = nlos.nlos_moe_workspace_bytes(self.fk_desc, self.rsd_desc)
        self.handle = nlos.nlos_moe_plan_create(ctx.handle, self.fk_desc, self.rsd_desc, beta, eps,
                                                shared_spectrum)

    def workspace(self) -> torch.Tensor:
        return torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.ctx.device)

    def __call__(self, tau: torch.Tensor, img: torch.Tensor, img_fk=None, img_rsd=None, ws=None):
        ny, nx, nt = self.shape
        assert tau.shape == (ny, nx, nt) and tau.dtype == torch.float32 and tau.is_cuda
        assert img.shape == (ny, nx) and img.dtype == torch.float32
        nlos.nlos_moe(self.ctx.handle, self.handle, tau, img, img_fk, img_rsd, ws)
        return img, img_fk, img_rsd

    def __del__(self):
        try:
            nlos.nlos_moe_plan_destroy(self.handle)
        except Exception:
            pass


def bin_events(ctx: Context, events: torch.Tensor, n_events: int, hist: torch.Tensor, bin_ps: int,
               t0_ps: int = 0, accumulate: bool = False, dropped: "torch.Tensor | None" = None):
    """events: device tensor of n_events packed 8-byte records; hist: int32 [ny, nx, nt]."""
    ny, nx, nt = hist.shape
    desc = nlos.bin_desc(nx, ny, nt, bin_ps, t0_ps, accumulate)
    nlos.nlos_bin(ctx.handle, desc, events, n_events, hist, dropped)
    return hist, dropped
