"""Shared helpers of the GPU parity tests: problem construction and error
reports.  Comparisons always take the oracle's float64 result as reference."""
from __future__ import annotations

import functools
import os

import numpy as np

import lmsynth

CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), ".cache")


def proj_err(gpu: np.ndarray, orc: np.ndarray):
    """Per-event projection error normalised as
    |gpu - orc| / max(|orc|, 1e-3 mean|orc|); returns (max, mean)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    orc = np.asarray(orc, dtype=np.float64)
    floor = 1e-3 * np.abs(orc).mean() if orc.size else 0.0
    den = np.maximum(np.abs(orc), floor)
    den = np.where(den > 0, den, 1.0)
    e = np.abs(gpu - orc) / den
    return (float(e.max()) if e.size else 0.0, float(e.mean()) if e.size else 0.0)


def img_err(gpu: np.ndarray, orc: np.ndarray) -> float:
    """||gpu - orc||_inf / ||orc||_inf."""
    gpu = np.asarray(gpu, dtype=np.float64)
    orc = np.asarray(orc, dtype=np.float64)
    den = np.abs(orc).max()
    return float(np.abs(gpu - orc).max() / (den if den > 0 else 1.0))


def report(name: str, **vals):
    print(f"[parity] {name}: " + ", ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}"
                                           for k, v in vals.items()), flush=True)


@functools.lru_cache(maxsize=None)
def problem_2d(n_prompts: int = 100_000, seed: int = 1000):
    """The 2D ring workload (360 crystals, 128x128, 25 TOF bins)."""
    return lmsynth.simulate_2d(lmsynth.config_2d(), n_prompts=n_prompts, seed=seed)


@functools.lru_cache(maxsize=None)
def problem_3d(n_prompts: int, seed: int = 1001, large: bool = False):
    """The 3D cylinder workload (672 x 96 crystals, 200x200x96 or 300x300x96).
    Cached on disk: the Monte Carlo takes ~3 s per 1e6 prompts."""
    cfg = lmsynth.config_3d_large() if large else lmsynth.config_3d()
    os.makedirs(CACHE, exist_ok=True)
    path = os.path.join(CACHE, f"{cfg.name}_{n_prompts}_{seed}.npz")
    if os.path.exists(path):
        d = np.load(path)
        cfg.events, cfg.s, cfg.x0 = d["events"], d["s"], d["x0"]
        cfg.seed = seed
        return cfg
    p = lmsynth.simulate_3d(cfg, n_prompts=n_prompts, seed=seed)
    tmp = path + f".tmp{os.getpid()}.npz"
    np.savez(tmp, events=p.events, s=p.s, x0=p.x0)
    os.replace(tmp, path)
    return p


def smooth_image(shape, seed: int, base: float = 1.0) -> np.ndarray:
    """A positive, smooth random image with a few sharp steps (phantom-like)."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.linspace(-1, 1, nz), np.linspace(-1, 1, ny), np.linspace(-1, 1, nx), indexing="ij")
    img = base * (1.0 + 0.3 * np.sin(2.1 * x + rng.uniform(0, 6)) * np.cos(1.7 * y + rng.uniform(0, 6)))
    for _ in range(4):
        c = rng.uniform(-0.6, 0.6, size=3)
        r = rng.uniform(0.1, 0.3)
        img = np.where((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 < r * r, img * 3.0, img)
    return img.astype(np.float32)


@functools.lru_cache(maxsize=None)
def sens_3d_input(large: bool = False) -> np.ndarray:
    """A dense sensitivity-like input image for the 3D workloads (the
    200x200x96 grid, or the 300x300x96 one with `large`): the oracle's
    non-TOF P^T 1 of a decimated scanner (every 16th crystal, every 8th
    ring, same cylinder and axial span), rescaled to the number of crystal
    pairs of the full one and floored at 1e-3 of its maximum so that no
    voxel is left without a penalty on x.  It is an input of the plan like
    any other, so both sides receive it (the full scanner's P^T 1 would take
    the oracle hours)."""
    import oracle
    p = lmsynth.config_3d_large() if large else lmsynth.config_3d()
    sc = p.scanner
    nr = sc.n_ring // 8
    dec = lmsynth.Scanner(sc.n_cry // 16, nr, sc.radius, sc.pitch * (sc.n_ring - 1) / (nr - 1))
    q = lmsynth.Problem("dec", dec, p.image, p.tof, 1, 1, 0.0)
    g = oracle.sens(oracle.Geometry.from_problem(q, tof_on=False))
    full = sc.n_det * (sc.n_det - 1) / 2.0
    part = dec.n_det * (dec.n_det - 1) / 2.0
    g = g * (full / part)
    return np.maximum(g, 1e-3 * g.max())
