"""Seeded synthetic inputs for the NLOS hot path.

This module is shared by the FP64 oracle (``oracle/``), the tests and the
benchmark.  It produces *inputs only*: confocal transient volumes, raw photon
events, the RSD frequency/weight/depth settings that the method takes as
parameters, and request streams for the serving loop.  It contains none of the
reconstruction arithmetic (no DFT, no Stolt remap, no propagation kernel).

Geometry follows the confocal setup of the paper's background section: the
relay wall is the plane z = 0, scan point (x, y) sits at
``((i + 1/2) * dx - W/2, (j + 1/2) * dy - H/2)`` and a time bin ``k`` covers
``[k * dt, (k + 1) * dt)`` of round-trip time measured from the wall point.

Transient recipe (configs with a volume input): every scene object is a set of
surface samples (position, normal, albedo * area).  Each (sample, scan point)
pair deposits ``a * cos(theta) / r**4`` at round-trip time ``2 r / c``, with
``theta`` the angle between the sample normal and the direction to the wall
point (point reflectors face the wall), linearly split between the two
nearest bins, then blurred along time with a Gaussian of sigma = 1 bin (normal
CDF mass per bin).  The expected volume is scaled so that the mean over objects
of each object's own peak bin is 50 photons, then Poisson-sampled.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

C_LIGHT = 299_792_458.0  # m/s

# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    nx: int
    ny: int
    nt: int
    bin_ps: float
    wall_w: float
    wall_h: float
    pad: int
    scene: str
    depth_range: Tuple[float, float]
    n_events: int = 0
    n_depth: int = 64
    seed: int = 0

    @property
    def dx(self) -> float:
        return self.wall_w / self.nx

    @property
    def dy(self) -> float:
        return self.wall_h / self.ny

    @property
    def c_dt(self) -> float:
        """Round-trip path length covered by one time bin (m)."""
        return C_LIGHT * self.bin_ps * 1e-12

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.ny, self.nx, self.nt)


CONFIGS: Dict[str, Config] = {
    # 32x32 scan on a 1 m wall, 256 bins of 32 ps, 3 point reflectors
    "c1": Config("c1", 32, 32, 256, 32.0, 1.0, 1.0, 2, "points3", (0.3, 0.8), seed=1001),
    # 64x64, 512 bins of 16 ps, 1e7 raw photon events from 2 planar patches
    "c2": Config("c2", 64, 64, 512, 16.0, 1.0, 1.0, 2, "patches2_events", (0.3, 0.9),
                 n_events=10_000_000, seed=1002),
    # 128x128x1024 of 16 ps, 5 patches + 3 spheres, padded to 256x256x2048
    "c3": Config("c3", 128, 128, 1024, 16.0, 1.0, 1.0, 2, "mix", (0.5, 1.5), seed=1003),
    # 256x256x512 of 32 ps, same generator, padded to 512x512x1024
    "c4": Config("c4", 256, 256, 512, 32.0, 1.0, 1.0, 2, "mix", (0.5, 1.5), seed=1004),
    # the office grid of Table 4 (360x260x512), 5 mm pitch on a 1.8 x 1.3 m wall, padded to
    # 720x520x1024 (factors 2, 3, 5, 13): a synthetic stand-in for the captured dataset
    "office": Config("office", 360, 260, 512, 32.0, 1.8, 1.3, 2, "mix", (0.5, 1.5), n_depth=51, seed=1005),
}


def small_config(nx: int, ny: int, nt: int, bin_ps: float = 32.0, pad: int = 2,
                 seed: int = 7, scene: str = "points3",
                 depth_range: Tuple[float, float] = (0.3, 0.8), n_depth: int = 16) -> Config:
    """A reduced geometry (1 m wall) for fast tests."""
    return Config(f"s{nx}x{ny}x{nt}", nx, ny, nt, bin_ps, 1.0, 1.0, pad, scene,
                  depth_range, n_depth=n_depth, seed=seed)


# ---------------------------------------------------------------------------
# scene objects as surface samples
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class SceneObject:
    kind: str
    pos: np.ndarray      # (n, 3) metres
    normal: np.ndarray   # (n, 3) unit, or None for wall-facing points
    weight: np.ndarray   # (n,) albedo * area


def _point_reflectors(rng, n, depth_range) -> List[SceneObject]:
    out = []
    for _ in range(n):
        x, y = rng.uniform(-0.4, 0.4, size=2)
        z = rng.uniform(*depth_range)
        out.append(SceneObject("point", np.array([[x, y, z]]), None, np.array([1.0])))
    return out


def _patch(rng, depth_range, spacing, max_side_pts, albedo_range=None) -> SceneObject:
    w, h = rng.uniform(0.1, 0.4, size=2)
    cx, cy = rng.uniform(-0.3, 0.3, size=2)
    z = rng.uniform(*depth_range)
    a = 1.0 if albedo_range is None else rng.uniform(*albedo_range)
    nu = int(min(max_side_pts, max(2, math.ceil(w / spacing) + 1)))
    nv = int(min(max_side_pts, max(2, math.ceil(h / spacing) + 1)))
    u = (np.arange(nu) + 0.5) / nu * w - w / 2
    v = (np.arange(nv) + 0.5) / nv * h - h / 2
    uu, vv = np.meshgrid(u, v, indexing="xy")
    pos = np.stack([cx + uu.ravel(), cy + vv.ravel(), np.full(uu.size, z)], axis=1)
    normal = np.tile(np.array([[0.0, 0.0, -1.0]]), (pos.shape[0], 1))
    weight = np.full(pos.shape[0], a * (w / nu) * (h / nv))
    return SceneObject("patch", pos, normal, weight)


def _sphere(rng, depth_range, n_pts, albedo_range) -> SceneObject:
    rad = rng.uniform(0.05, 0.2)
    cx, cy = rng.uniform(-0.3, 0.3, size=2)
    cz = rng.uniform(*depth_range)
    a = rng.uniform(*albedo_range)
    # Fibonacci points on the hemisphere facing the wall (normal.z < 0)
    k = np.arange(n_pts) + 0.5
    cos_pol = k / n_pts               # in (0, 1): angle from the -z axis
    sin_pol = np.sqrt(1.0 - cos_pol ** 2)
    az = math.pi * (1.0 + 5.0 ** 0.5) * k
    # scalar libm trig so that the samples do not depend on the host's SIMD dispatch
    ca = np.array([math.cos(x) for x in az])
    sa = np.array([math.sin(x) for x in az])
    normal = np.stack([sin_pol * ca, sin_pol * sa, -cos_pol], axis=1)
    pos = np.array([cx, cy, cz]) + rad * normal
    weight = np.full(n_pts, a * 2.0 * math.pi * rad * rad / n_pts)
    return SceneObject("sphere", pos, normal, weight)


def make_objects(cfg: Config, seed: Optional[int] = None,
                 max_side_pts: Optional[int] = None,
                 sphere_pts: Optional[int] = None) -> List[SceneObject]:
    """Scene of the config.  The mixed scene's sampling density is capped so that
    (scan points x surface samples) stays near 1.5e8 pairs: 32x32 samples per
    patch and 512 per sphere up to 128x128 scans, 16x16 and 256 at 256x256."""
    npix = cfg.nx * cfg.ny
    if max_side_pts is None:
        max_side_pts = 32 if npix <= 128 * 128 else 16
    if sphere_pts is None:
        sphere_pts = 512 if npix <= 128 * 128 else 256
    rng = np.random.Generator(np.random.PCG64(cfg.seed if seed is None else seed))
    if cfg.scene == "points3":
        return _point_reflectors(rng, 3, cfg.depth_range)
    if cfg.scene == "patches2_events":
        spacing = cfg.dx / 2
        return [_patch(rng, cfg.depth_range, spacing, 10 ** 6) for _ in range(2)]
    if cfg.scene == "mix":
        objs = [_patch(rng, cfg.depth_range, cfg.dx / 2, max_side_pts, (0.2, 1.0))
                for _ in range(5)]
        objs += [_sphere(rng, cfg.depth_range, sphere_pts, (0.2, 1.0)) for _ in range(3)]
        return objs
    raise ValueError(cfg.scene)


def point_object(x: float, y: float, z: float) -> SceneObject:
    return SceneObject("point", np.array([[x, y, z]], dtype=np.float64), None, np.array([1.0]))


# ---------------------------------------------------------------------------
# transient volumes
# ---------------------------------------------------------------------------


def scan_positions(cfg: Config) -> Tuple[np.ndarray, np.ndarray]:
    xs = (np.arange(cfg.nx) + 0.5) * cfg.dx - cfg.wall_w / 2
    ys = (np.arange(cfg.ny) + 0.5) * cfg.dy - cfg.wall_h / 2
    return xs, ys


def _gauss_bin_mass(sigma_bins: float = 1.0, half: int = 4) -> np.ndarray:
    """Mass of N(0, sigma) in each unit bin centred on -half..half."""
    edges = np.arange(-half, half + 2) - 0.5
    cdf = np.array([0.5 * (1.0 + math.erf(e / (sigma_bins * math.sqrt(2.0)))) for e in edges])
    m = np.diff(cdf)
    return m / m.sum()


def _object_transient(cfg: Config, obj: SceneObject, pairs_per_chunk: int = 1 << 22) -> np.ndarray:
    """Expected (noise-free, un-blurred) transient of one object, [ny*nx, nt]."""
    xs, ys = scan_positions(cfg)
    sx, sy = np.meshgrid(xs, ys, indexing="xy")  # (ny, nx)
    sx = sx.ravel()
    sy = sy.ravel()
    npix = sx.size
    nt = cfg.nt
    acc = np.zeros((npix, nt), dtype=np.float64)
    p = obj.pos
    npts = p.shape[0]
    step = max(1, pairs_per_chunk // npts)
    inv_cdt = 2.0 / cfg.c_dt
    for s in range(0, npix, step):
        e = min(npix, s + step)
        dxv = sx[s:e, None] - p[None, :, 0]
        dyv = sy[s:e, None] - p[None, :, 1]
        dzv = -p[None, :, 2]
        r2 = dxv * dxv + dyv * dyv + dzv * dzv
        r = np.sqrt(r2)
        if obj.normal is None:
            num = -dzv
        else:
            n = obj.normal
            num = dxv * n[None, :, 0] + dyv * n[None, :, 1] + dzv * n[None, :, 2]
            np.clip(num, 0.0, None, out=num)
        val = (obj.weight[None, :] * num) / (r2 * r2 * r)   # a cos / r^4
        tb = r * inv_cdt - 0.5  # bin-centre coordinate
        i0 = np.floor(tb)
        fr = tb - i0
        i0 = i0.astype(np.int64)
        idx = np.concatenate([i0.ravel(), (i0 + 1).ravel()])
        wv = np.concatenate([(val * (1.0 - fr)).ravel(), (val * fr).ravel()])
        row = np.tile(np.repeat(np.arange(e - s, dtype=np.int64) * nt, npts), 2)
        ok = (idx >= 0) & (idx < nt)
        acc[s:e] = np.bincount((row + idx)[ok], weights=wv[ok],
                               minlength=(e - s) * nt).reshape(e - s, nt)
    return acc


def _blur_time(vol: np.ndarray) -> np.ndarray:
    k = _gauss_bin_mass()
    half = (k.size - 1) // 2
    out = np.zeros_like(vol)
    nt = vol.shape[-1]
    for o, m in zip(range(-half, half + 1), k):
        if o >= 0:
            out[..., o:] += m * vol[..., :nt - o]
        else:
            out[..., :nt + o] += m * vol[..., -o:]
    return out


def expected_transient(cfg: Config, objects: List[SceneObject],
                       peak_photons: float = 50.0) -> np.ndarray:
    """Expected photon counts [ny][nx][nt] (float64), scaled to the peak target."""
    total = np.zeros((cfg.ny * cfg.nx, cfg.nt))
    peaks = []
    for obj in objects:
        e = _blur_time(_object_transient(cfg, obj))
        peaks.append(e.max())
        total += e
    scale = peak_photons / max(np.mean(peaks), 1e-300)
    return (total * scale).reshape(cfg.ny, cfg.nx, cfg.nt)


def transient(cfg: Config, seed: Optional[int] = None, noise: bool = True,
              objects: Optional[List[SceneObject]] = None) -> np.ndarray:
    """Poisson-sampled transient volume tau[ny][nx][nt] as float32 counts."""
    s = cfg.seed if seed is None else seed
    objs = make_objects(cfg, s) if objects is None else objects
    lam = expected_transient(cfg, objs)
    if not noise:
        return lam.astype(np.float32)
    rng = np.random.Generator(np.random.PCG64(s + 17))
    return rng.poisson(lam).astype(np.float32)


# ---------------------------------------------------------------------------
# raw photon events
# ---------------------------------------------------------------------------

EVENT_DTYPE = np.dtype([("pixel", "<i4"), ("t_ps", "<u4")])


def photon_events(cfg: Config, n_events: Optional[int] = None, seed: Optional[int] = None,
                  order: str = "shuffled", background: float = 0.05) -> np.ndarray:
    """Raw events (int32 pixel = y*nx + x, uint32 picosecond timestamp).

    A fraction ``1 - background`` is drawn from the expected transient of the
    config's scene ((pixel, surface sample) pairs chosen with probability
    proportional to ``a cos(theta) / r**4``; time ``2 r / c`` plus N(0, bin_ps)
    jitter, floored to whole picoseconds).  The rest is uniform over pixels and
    ``[0, nt * bin_ps)`` ps.  ``order`` is "shuffled" or "pixel" (sorted by
    pixel, stable).
    """
    n = cfg.n_events if n_events is None else n_events
    s = cfg.seed if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(s + 29))
    objs = make_objects(cfg, s)
    xs, ys = scan_positions(cfg)
    sx, sy = np.meshgrid(xs, ys, indexing="xy")
    sx = sx.ravel()
    sy = sy.ravel()
    pos = np.concatenate([o.pos for o in objs])
    wgt = np.concatenate([o.weight for o in objs])
    nrm = np.concatenate([o.normal if o.normal is not None else
                          np.tile([[0.0, 0.0, -1.0]], (o.pos.shape[0], 1)) for o in objs])
    dxv = sx[:, None] - pos[None, :, 0]
    dyv = sy[:, None] - pos[None, :, 1]
    dzv = -pos[None, :, 2]
    r = np.sqrt(dxv ** 2 + dyv ** 2 + dzv ** 2)
    cos = np.clip((dxv * nrm[None, :, 0] + dyv * nrm[None, :, 1] + dzv * nrm[None, :, 2]) / r,
                  0.0, None)
    p = (wgt[None, :] * cos / r ** 4).ravel()
    p /= p.sum()
    n_sig = int(round(n * (1.0 - background)))
    n_bg = n - n_sig
    pick = rng.choice(p.size, size=n_sig, p=p)
    pix_sig = (pick // pos.shape[0]).astype(np.int64)
    t_true_ps = 2.0 * r.ravel()[pick] / C_LIGHT * 1e12
    t_sig = np.floor(t_true_ps + rng.normal(0.0, cfg.bin_ps, size=n_sig))
    t_sig = np.clip(t_sig, 0, 2 ** 32 - 1)
    pix_bg = rng.integers(0, cfg.nx * cfg.ny, size=n_bg)
    t_bg = rng.integers(0, int(cfg.nt * cfg.bin_ps), size=n_bg)
    ev = np.empty(n, dtype=EVENT_DTYPE)
    ev["pixel"][:n_sig] = pix_sig
    ev["t_ps"][:n_sig] = t_sig.astype(np.uint32)
    ev["pixel"][n_sig:] = pix_bg
    ev["t_ps"][n_sig:] = t_bg.astype(np.uint32)
    if order == "shuffled":
        ev = ev[rng.permutation(n)]
    elif order == "pixel":
        ev = ev[np.argsort(ev["pixel"], kind="stable")]
    else:
        raise ValueError(order)
    return ev


def random_events(n: int, nx: int, ny: int, nt: int, bin_ps: int, seed: int,
                  invalid_frac: float = 0.0) -> np.ndarray:
    """Uniform events, a fraction of them out of range (bad pixel or late time)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ev = np.empty(n, dtype=EVENT_DTYPE)
    ev["pixel"] = rng.integers(0, nx * ny, size=n)
    ev["t_ps"] = rng.integers(0, nt * bin_ps, size=n).astype(np.uint32)
    nbad = int(n * invalid_frac)
    if nbad:
        which = rng.choice(n, size=nbad, replace=False)
        kind = rng.integers(0, 3, size=nbad)
        ev["pixel"][which[kind == 0]] = -1 - rng.integers(0, 1000, size=int((kind == 0).sum()))
        ev["pixel"][which[kind == 1]] = nx * ny + rng.integers(0, 1000, size=int((kind == 1).sum()))
        ev["t_ps"][which[kind == 2]] = (nt * bin_ps + rng.integers(0, 10 ** 6, size=int((kind == 2).sum()))).astype(np.uint32)
    return ev


# ---------------------------------------------------------------------------
# RSD parameters (frequency set, weights, depth grid)
# ---------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class RsdParams:
    freq_bins: np.ndarray   # int32 DFT bins of nt
    weights: np.ndarray     # complex128 per frequency
    depth0: float
    depth_step: float
    n_depth: int
    sigma_s: int = 2
    sigma_t: int = 0
    delta: float = 0.0


def rsd_params(cfg: Config, n_depth: Optional[int] = None) -> RsdParams:
    """Gaussian band around the virtual wavelength, capped at Nyquist.

    lambda_c = max(4 dx, 8 c dt); k_c = round(nt c dt / lambda_c);
    sigma_k = max(2, k_c / 6); keep |k - k_c| <= 3 sigma_k within [1, nt/2 - 1];
    w = exp(-(k - k_c)^2 / (2 sigma_k^2)).  Depths span the scene range +- 0.1 m.
    """
    lam_c = max(4.0 * cfg.dx, 8.0 * cfg.c_dt)
    k_c = int(round(cfg.nt * cfg.c_dt / lam_c))
    k_c = max(1, min(k_c, cfg.nt // 2 - 1))
    ks = np.arange(1, cfg.nt // 2)
    if k_c >= 12:
        sigma = k_c / 6.0
        keep = 2 * np.abs(ks - k_c) <= k_c          # |k - k_c| <= 3 sigma, exact
    else:
        sigma = 2.0
        keep = np.abs(ks - k_c) <= 6
    kb = ks[keep].astype(np.int32)
    w = np.exp(-((kb - k_c) ** 2) / (2.0 * sigma ** 2)).astype(np.complex128)
    nd = cfg.n_depth if n_depth is None else n_depth
    z0, z1 = cfg.depth_range
    d0 = z0 - 0.1
    step = (z1 - z0 + 0.2) / max(nd - 1, 1)
    return RsdParams(kb, w, d0, step, nd)


# ---------------------------------------------------------------------------
# serving request stream
# ---------------------------------------------------------------------------

SERVE_SHAPES = [(64, 64, 512), (128, 128, 1024), (256, 256, 512)]


def request_stream(n: int, rate_hz: float, seed: int = 5005,
                   precisions=("fp32",)) -> List[dict]:
    """Poisson arrivals; size uniform over SERVE_SHAPES, method 50/50 fk/rsd."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, size=n)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        ny, nx, nt = SERVE_SHAPES[int(rng.integers(0, len(SERVE_SHAPES)))]
        method = "fk" if rng.random() < 0.5 else "rsd"
        prec = precisions[int(rng.integers(0, len(precisions)))]
        out.append(dict(id=i, arrival_s=float(t[i]), shape=(ny, nx, nt), method=method,
                        precision=prec, seed=int(rng.integers(0, 2 ** 31 - 1))))
    return out


# ---------------------------------------------------------------------------
# on-disk cache for the slow, large inputs (plain .npy, no pickle)
# ---------------------------------------------------------------------------

GENERATOR_VERSION = 2


def _cache_path(tag: str) -> str:
    import os
    d = os.environ.get("NLOS_SCENE_CACHE", "/tmp/nlos_scene_cache")
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, f"v{GENERATOR_VERSION}_{tag}.npy")


def cached(tag: str, make):
    """Load ``tag`` from the cache or build it with ``make()`` and store it."""
    import os
    path = _cache_path(tag)
    if os.path.exists(path):
        try:
            return np.load(path, allow_pickle=False)
        except (OSError, ValueError):
            pass
    arr = make()
    tmp = path + f".tmp{os.getpid()}.npy"
    np.save(tmp, arr, allow_pickle=False)
    os.replace(tmp, path)
    return arr


def config_transient(name: str) -> np.ndarray:
    """The seeded transient of a named config (c1, c3, c4), cached on disk."""
    cfg = CONFIGS[name]
    return cached(f"{name}_tau_{cfg.seed}", lambda: transient(cfg))


def checksum(a: np.ndarray) -> str:
    """sha256 of an array's bytes (identifies a generated input)."""
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def config_events(name: str = "c2", order: str = "shuffled") -> np.ndarray:
    cfg = CONFIGS[name]
    return cached(f"{name}_events_{order}_{cfg.seed}", lambda: photon_events(cfg, order=order))


# ---------------------------------------------------------------------------
# serving mix: geometry and inputs per request shape
# ---------------------------------------------------------------------------

SERVE_CONFIG_OF_SHAPE = {(64, 64, 512): "c2", (128, 128, 1024): "c3", (256, 256, 512): "c4"}


def serve_config(shape) -> Config:
    """The config whose geometry a serving request of this shape uses."""
    return CONFIGS[SERVE_CONFIG_OF_SHAPE[tuple(shape)]]


def serve_geometry(shape) -> dict:
    cfg = serve_config(shape)
    return dict(wall_w=cfg.wall_w, wall_h=cfg.wall_h, bin_ps=cfg.bin_ps, pad=cfg.pad,
                dx=cfg.dx, dy=cfg.dy, rsd=rsd_params(cfg))


def serve_input(shape, seed: int) -> np.ndarray:
    """A fast seeded input of a serving shape: three point reflectors in the config's
    depth range, Poisson counts (content does not affect the work)."""
    base = serve_config(shape)
    cfg = dataclasses.replace(base, scene="points3", seed=seed)
    return transient(cfg, seed=seed)
