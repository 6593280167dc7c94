"""Writes the oracle's expected values for the full-size parity cases.

Calls only oracle/ and scenes/ (the seeded input generators).  For each case it
stores the sha256 of the generated input, the full max-over-depth image (FP64
oracle values rounded to float32 for storage) and a seeded sample of volume
voxels (the 1024 largest plus 3072 uniformly drawn) with their FP64 values.  Run from the repository root:

    python tests/golden/make_golden.py [fk_c4 fk_c3 rsd_c3]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import scenes  # noqa: E402
from oracle import fk as ofk  # noqa: E402
from oracle import rsd as orsd  # noqa: E402


def sample_indices(vol: np.ndarray, n_top: int = 1024, n_rand: int = 3072, seed: int = 11):
    flat = vol.ravel()
    top = np.argpartition(flat, -n_top)[-n_top:]
    rng = np.random.default_rng(seed)
    rnd = rng.choice(flat.size, size=n_rand, replace=False)
    return np.unique(np.concatenate([top, rnd]))


def save(name: str, tau: np.ndarray, vol: np.ndarray, img: np.ndarray, extra=None):
    idx = sample_indices(vol)
    out = dict(tau_sha256=np.array(scenes.checksum(tau)), img=img.astype(np.float32),
               idx=idx.astype(np.int64), val=vol.ravel()[idx].astype(np.float64),
               vol_l2=np.array(np.linalg.norm(vol.ravel())), shape=np.array(vol.shape))
    if extra:
        out.update(extra)
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path} ({os.path.getsize(path) / 1024:.0f} KiB)", flush=True)


def fk_case(cname: str):
    cfg = scenes.CONFIGS[cname]
    tau = scenes.config_transient(cname)
    t = time.time()
    vol, img = ofk.fk(tau.astype(np.float64), cfg.wall_w, cfg.wall_h, cfg.bin_ps, cfg.pad)
    print(f"fk {cname}: oracle {time.time() - t:.1f} s", flush=True)
    save(f"fk_{cname}", tau, vol, img)


def rsd_case(cname: str):
    cfg = scenes.CONFIGS[cname]
    tau = scenes.config_transient(cname)
    p = scenes.rsd_params(cfg)
    depths = p.depth0 + p.depth_step * np.arange(p.n_depth)
    t = time.time()
    vol, img = orsd.rsd(tau.astype(np.float64), cfg.dx, cfg.dy, cfg.bin_ps, cfg.pad, p.freq_bins,
                        p.weights, depths, p.sigma_s, p.sigma_t, p.delta)
    print(f"rsd {cname}: oracle {time.time() - t:.1f} s", flush=True)
    save(f"rsd_{cname}", tau, vol, img)


CASES = {"fk_c4": lambda: fk_case("c4"), "fk_c3": lambda: fk_case("c3"),
         "rsd_c3": lambda: rsd_case("c3")}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        CASES[name]()
