"""Seeded synthetic inputs for listmode TOF-PET reconstruction.

This module produces the *inputs* of the problem: the crystal coordinate
table of a cylindrical scanner, phantoms, Monte-Carlo prompt events with
their contamination estimates, a starting image and the random subset
sequence of the stochastic algorithm.  It contains none of the method's
arithmetic (no projector, no step size, no prox): both the FP64 oracle and
the HIP library consume what it returns, and neither is imported here.

Geometry conventions (used identically by every consumer):

* crystal ``(c, r)`` has id ``c + n_cry * r`` and sits at
  ``(R cos(2 pi c / n_cry), R sin(2 pi c / n_cry), (r - (n_ring-1)/2) * pitch)``;
  the table is computed in float64 and rounded once to float32, and that
  float32 table is the scanner description both sides read;
* an event is ``int16[5] = (c1, r1, c2, r2, k)``: the two crystals of the
  line of response and the signed TOF bin ``k`` (``|k| <= (n_tof-1)/2``);
  a positive TOF coordinate points from crystal 1 towards crystal 2;
* an image is float32, C-order ``[z][y][x]``, voxel ``(i, j, k)`` centred at
  ``((i-(nx-1)/2) hx, (j-(ny-1)/2) hy, (k-(nz-1)/2) hz)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Tuple

import numpy as np

__all__ = [
    "Scanner", "ImageGeom", "TOF", "Problem",
    "config_2d", "config_3d", "config_3d_large", "config_serving_small",
    "tiny_2d", "tiny_3d",
    "det_table", "phantom_2d_discs", "phantom_3d_ellipsoid",
    "simulate_2d", "simulate_3d", "uniform_x0", "splitmix64", "subset_sequence",
    "random_events",
]



@dataclasses.dataclass(frozen=True)
class Scanner:
    n_cry: int          # crystals per ring
    n_ring: int         # rings
    radius: float       # mm
    pitch: float = 0.0  # axial ring spacing, mm (0 for a single ring)

    @property
    def n_det(self) -> int:
        return self.n_cry * self.n_ring

    @property
    def axial_half(self) -> float:
        """Half axial extent covered by the crystals (edge to edge), mm."""
        return 0.5 * self.n_ring * self.pitch


@dataclasses.dataclass(frozen=True)
class ImageGeom:
    n: Tuple[int, int, int]        # (nx, ny, nz)
    h: Tuple[float, float, float]  # voxel size (hx, hy, hz), mm

    @property
    def shape_zyx(self) -> Tuple[int, int, int]:
        return (self.n[2], self.n[1], self.n[0])

    @property
    def nvox(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def centres(self, axis: int) -> np.ndarray:
        n, h = self.n[axis], self.h[axis]
        return (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * h


@dataclasses.dataclass(frozen=True)
class TOF:
    n_tof: int          # odd number of TOF bins
    bin: float          # bin width, mm
    fwhm: float         # Gaussian TOF kernel FWHM, mm
    nsigma: float = 3.0 # truncation of the kernel in units of sigma
    on: bool = True

    @property
    def sigma(self) -> float:
        return self.fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))

    @property
    def kmax(self) -> int:
        return (self.n_tof - 1) // 2


@dataclasses.dataclass
class Problem:
    """A complete synthetic listmode reconstruction problem."""
    name: str
    scanner: Scanner
    image: ImageGeom
    tof: TOF
    n_subsets: int
    epochs: int
    beta: float
    events: np.ndarray | None = None   # int16 [N, 5], chronological order
    s: np.ndarray | None = None        # float32 [N], contamination per event
    x0: np.ndarray | None = None       # float32 [nz, ny, nx]
    x_true: np.ndarray | None = None   # float32 phantom (activity units)
    seed: int = 0

    @property
    def det(self) -> np.ndarray:
        return det_table(self.scanner)


# --------------------------------------------------------------------------
# scanner table


def det_table(sc: Scanner) -> np.ndarray:
    """float32 [n_cry * n_ring, 3] crystal centres (computed in float64)."""
    c = np.arange(sc.n_cry, dtype=np.float64)
    phi = 2.0 * np.pi * c / sc.n_cry
    r = np.arange(sc.n_ring, dtype=np.float64)
    z = (r - (sc.n_ring - 1) / 2.0) * sc.pitch
    tab = np.empty((sc.n_ring, sc.n_cry, 3), dtype=np.float64)
    tab[:, :, 0] = sc.radius * np.cos(phi)[None, :]
    tab[:, :, 1] = sc.radius * np.sin(phi)[None, :]
    tab[:, :, 2] = z[:, None]
    return np.ascontiguousarray(tab.reshape(-1, 3).astype(np.float32))


# --------------------------------------------------------------------------
# workload presets


def config_2d() -> Problem:
    """2D TOF ring: 360 crystals on R = 300 mm, 128x128 image of 2 mm pixels,
    TOF FWHM 60 mm (400 ps) over 25 bins of 24 mm truncated at 3 sigma,
    28 subsets, 10 epochs, TV beta = 0.03."""
    return Problem(
        name="2d_ring360_128x128",
        scanner=Scanner(360, 1, 300.0, 0.0),
        image=ImageGeom((128, 128, 1), (2.0, 2.0, 2.0)),
        tof=TOF(25, 24.0, 60.0, 3.0, True),
        n_subsets=28, epochs=10, beta=0.03)


def config_3d() -> Problem:
    """3D TOF cylinder: 672 crystals x 96 rings on R = 380 mm with 2.6 mm ring
    pitch (249.6 mm axial), 200x200x96 image of 2.6 mm voxels, TOF FWHM 400 ps
    (60 mm) over 33 bins of 24 mm, 224 subsets, 5 epochs, TV beta = 0.03."""
    return Problem(
        name="3d_672x96_200x200x96",
        scanner=Scanner(672, 96, 380.0, 2.6),
        image=ImageGeom((200, 200, 96), (2.6, 2.6, 2.6)),
        tof=TOF(33, 24.0, 60.0, 3.0, True),
        n_subsets=224, epochs=5, beta=0.03)


def config_3d_large() -> Problem:
    """Same scanner, 300x300x96 image of 1.75 x 1.75 x 2.6 mm voxels (the box
    stays inside the bore)."""
    p = config_3d()
    return dataclasses.replace(p, name="3d_672x96_300x300x96",
                               image=ImageGeom((300, 300, 96), (1.75, 1.75, 2.6)),
                               epochs=1)


def config_serving_small() -> Problem:
    """Dynamic-frame image: 128x128x48 over the same 520 x 249.6 mm field."""
    p = config_3d()
    return dataclasses.replace(p, name="3d_672x96_128x128x48",
                               image=ImageGeom((128, 128, 48), (4.0625, 4.0625, 5.2)),
                               n_subsets=28, epochs=3)


def tiny_2d(n_det: int = 16, nxy: int = 8, h: float = 2.0, radius: float = 20.0,
            n_tof: int = 5, tof_bin: float = 6.0, fwhm: float = 9.0,
            tof_on: bool = True) -> Problem:
    """A brute-force sized 2D ring for operator tests."""
    return Problem(
        name=f"tiny2d_{n_det}_{nxy}",
        scanner=Scanner(n_det, 1, radius, 0.0),
        image=ImageGeom((nxy, nxy, 1), (h, h, h)),
        tof=TOF(n_tof, tof_bin, fwhm, 3.0, tof_on),
        n_subsets=1, epochs=1, beta=0.03)


def tiny_3d(n_cry: int = 24, n_ring: int = 4, nxy: int = 10, nz: int = 4,
            h: float = 2.0, radius: float = 24.0, pitch: float = 2.0,
            n_tof: int = 7, tof_bin: float = 6.0, fwhm: float = 9.0,
            tof_on: bool = True) -> Problem:
    """A brute-force sized 3D cylinder for operator tests."""
    return Problem(
        name=f"tiny3d_{n_cry}x{n_ring}_{nxy}x{nz}",
        scanner=Scanner(n_cry, n_ring, radius, pitch),
        image=ImageGeom((nxy, nxy, nz), (h, h, h)),
        tof=TOF(n_tof, tof_bin, fwhm, 3.0, tof_on),
        n_subsets=1, epochs=1, beta=0.03)


# --------------------------------------------------------------------------
# phantoms


def _supersampled(img: ImageGeom, inside, ss: int = 3) -> np.ndarray:
    """Mean of an indicator-like function over ss^d sub-samples per voxel."""
    nx, ny, nz = img.n
    hx, hy, hz = img.h
    off = (np.arange(ss) + 0.5) / ss - 0.5
    zs = img.centres(2)
    out = np.zeros(img.shape_zyx, dtype=np.float64)
    xs, ys = img.centres(0), img.centres(1)
    oz = off if nz > 1 else np.zeros(1)
    for dz in oz:
        for dy in off:
            for dx in off:
                X = (xs + dx * hx)[None, None, :]
                Y = (ys + dy * hy)[None, :, None]
                Z = (zs + dz * hz)[:, None, None]
                out += inside(X, Y, Z)
    return out / (len(oz) * ss * ss)


HOT_DISCS_2D = ((50.0, 0.0, 12.0), (-25.0, 43.3, 16.0), (-25.0, -43.3, 20.0))


def phantom_2d_discs(img: ImageGeom) -> np.ndarray:
    """Disc r = 100 mm (activity 1) with three hot discs (activity 4)."""
    def act(X, Y, Z):
        a = ((X ** 2 + Y ** 2) <= 100.0 ** 2).astype(np.float64)
        for cx, cy, r in HOT_DISCS_2D:
            a = np.where((X - cx) ** 2 + (Y - cy) ** 2 <= r ** 2, 4.0, a)
        return a + 0 * Z
    return _supersampled(img, act).astype(np.float32)


ELLIPSOID = (200.0, 150.0, 100.0)
SPHERE_R = (5.0, 7.5, 10.0, 12.5, 15.0)


def _spheres_3d():
    return [(80.0 * math.cos(2 * math.pi * j / 5), 80.0 * math.sin(2 * math.pi * j / 5), 0.0, r)
            for j, r in enumerate(SPHERE_R)]


def phantom_3d_ellipsoid(img: ImageGeom) -> np.ndarray:
    """Ellipsoid (200, 150, 100) mm, activity 1, five hot spheres (activity 4)
    of radius 5..15 mm on a circle of 80 mm in the central plane."""
    a0, b0, c0 = ELLIPSOID

    def act(X, Y, Z):
        a = (((X / a0) ** 2 + (Y / b0) ** 2 + (Z / c0) ** 2) <= 1.0).astype(np.float64)
        for cx, cy, cz, r in _spheres_3d():
            a = np.where((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2 <= r ** 2, 4.0, a)
        return a
    return _supersampled(img, act, ss=2).astype(np.float32)


# --------------------------------------------------------------------------
# Monte-Carlo events


def _ring_hits(P: np.ndarray, U: np.ndarray, R: float):
    """Both intersections of lines P + s U with the cylinder x^2 + y^2 = R^2."""
    ux, uy = U[:, 0], U[:, 1]
    a = ux * ux + uy * uy
    b = P[:, 0] * ux + P[:, 1] * uy
    c = P[:, 0] ** 2 + P[:, 1] ** 2 - R * R
    disc = np.sqrt(np.maximum(b * b - a * c, 0.0))
    s_p = (-b + disc) / a
    s_m = (-b - disc) / a
    return P + s_p[:, None] * U, P + s_m[:, None] * U


def _nearest_crystal(Q: np.ndarray, sc: Scanner):
    phi = np.arctan2(Q[:, 1], Q[:, 0])
    c = np.rint(phi * sc.n_cry / (2 * np.pi)).astype(np.int64) % sc.n_cry
    if sc.n_ring > 1:
        r = np.rint(Q[:, 2] / sc.pitch + (sc.n_ring - 1) / 2.0).astype(np.int64)
        r = np.clip(r, 0, sc.n_ring - 1)
    else:
        r = np.zeros_like(c)
    return c, r


def _tof_bins(P, det64, c1, r1, c2, r2, sc: Scanner, tof: TOF, rng):
    """Signed TOF bin of emission points P on the detected LORs."""
    i1 = c1 + sc.n_cry * r1
    i2 = c2 + sc.n_cry * r2
    p1, p2 = det64[i1], det64[i2]
    d = p2 - p1
    nrm = np.linalg.norm(d, axis=1)
    nrm = np.where(nrm > 0.0, nrm, 1.0)  # same-crystal pairs: dropped by the caller
    t = np.einsum("ij,ij->i", P - 0.5 * (p1 + p2), d) / nrm
    t = t + rng.normal(0.0, tof.sigma, size=t.shape)
    return np.rint(t / tof.bin).astype(np.int64)


def _sample_2d_points(rng, n):
    """Emission points proportional to the 2D disc phantom."""
    out = np.empty((0, 2))
    while len(out) < n:
        m = 2 * (n - len(out)) + 1024
        xy = rng.uniform(-100.0, 100.0, size=(m, 2))
        rr = (xy ** 2).sum(1)
        act = np.where(rr <= 100.0 ** 2, 1.0, 0.0)
        for cx, cy, r in HOT_DISCS_2D:
            act = np.where(((xy[:, 0] - cx) ** 2 + (xy[:, 1] - cy) ** 2) <= r * r, 4.0, act)
        keep = rng.uniform(0.0, 4.0, size=m) < act
        out = np.concatenate([out, xy[keep]])
    return out[:n]


def _sample_3d_points(rng, n):
    """Emission points proportional to the 3D ellipsoid phantom (mixture of
    the uniform ellipsoid and the spheres' excess activity)."""
    a0, b0, c0 = ELLIPSOID
    vol_e = 4.0 / 3.0 * math.pi * a0 * b0 * c0
    sph = _spheres_3d()
    w = np.array([vol_e] + [3.0 * 4.0 / 3.0 * math.pi * r ** 3 for *_c, r in sph])
    comp = rng.choice(len(w), size=n, p=w / w.sum())
    out = np.empty((n, 3))
    cnt = np.bincount(comp, minlength=len(w))
    for j in range(len(w)):
        m = int(cnt[j])
        if m == 0:
            continue
        pts = np.empty((0, 3))
        while len(pts) < m:
            q = rng.uniform(-1.0, 1.0, size=(2 * (m - len(pts)) + 256, 3))
            pts = np.concatenate([pts, q[(q ** 2).sum(1) <= 1.0]])
        pts = pts[:m]
        if j == 0:
            pts = pts * np.array([a0, b0, c0])
        else:
            cx, cy, cz, r = sph[j - 1]
            pts = pts * r + np.array([cx, cy, cz])
        out[comp == j] = pts
    return out


def _trues(rng, n, sc: Scanner, tof: TOF, dim: int):
    det64 = det_table(sc).astype(np.float64)
    blocks, have, acc = [], 0, 0.5
    zmax = sc.axial_half
    while have < n:
        m = min(int(1.1 * (n - have) / acc) + 1024, 4_000_000)
        if dim == 2:
            P2 = _sample_2d_points(rng, m)
            P = np.concatenate([P2, np.zeros((m, 1))], axis=1)
            phi = rng.uniform(0.0, np.pi, size=m)
            U = np.stack([np.cos(phi), np.sin(phi), np.zeros(m)], axis=1)
        else:
            P = _sample_3d_points(rng, m)
            U = rng.normal(size=(m, 3))
            U /= np.linalg.norm(U, axis=1)[:, None]
        A, B = _ring_hits(P, U, sc.radius)
        ok = np.ones(m, dtype=bool)
        if dim == 3:
            ok &= (np.abs(A[:, 2]) <= zmax) & (np.abs(B[:, 2]) <= zmax)
        swap = rng.uniform(size=m) < 0.5
        A2 = np.where(swap[:, None], B, A)
        B2 = np.where(swap[:, None], A, B)
        c1, r1 = _nearest_crystal(A2, sc)
        c2, r2 = _nearest_crystal(B2, sc)
        ok &= c1 != c2
        k = _tof_bins(P, det64, c1, r1, c2, r2, sc, tof, rng)
        ok &= np.abs(k) <= tof.kmax
        blk = np.stack([c1, r1, c2, r2, k], axis=1)[ok]
        acc = max(len(blk) / m, 0.02)
        blocks.append(blk)
        have += len(blk)
    return np.concatenate(blocks)[:n]


def _random_pairs(rng, m, sc: Scanner):
    """Uniform unordered crystal pairs with different transaxial index, in a
    random order."""
    c1 = rng.integers(0, sc.n_cry, size=m)
    c2 = (c1 + rng.integers(1, sc.n_cry, size=m)) % sc.n_cry
    r1 = rng.integers(0, sc.n_ring, size=m)
    r2 = rng.integers(0, sc.n_ring, size=m)
    return c1, r1, c2, r2


def _lor_axis_distance(det64, c1, r1, c2, r2, sc: Scanner):
    """Transaxial distance of the LOR from the scanner axis."""
    p1 = det64[c1 + sc.n_cry * r1][:, :2]
    p2 = det64[c2 + sc.n_cry * r2][:, :2]
    d = p2 - p1
    cross = np.abs(p1[:, 0] * d[:, 1] - p1[:, 1] * d[:, 0])
    return cross / np.linalg.norm(d, axis=1)


SCATTER_WIDTH = 200.0  # mm, width of the smooth contamination profile


def _contamination(rng, n, sc: Scanner, tof: TOF, smooth: bool):
    det64 = det_table(sc).astype(np.float64)
    ev = np.empty((0, 5), dtype=np.int64)
    while len(ev) < n:
        m = 2 * (n - len(ev)) + 1024
        c1, r1, c2, r2 = _random_pairs(rng, m, sc)
        k = rng.integers(-tof.kmax, tof.kmax + 1, size=m)
        if smooth:
            b = _lor_axis_distance(det64, c1, r1, c2, r2, sc)
            keep = rng.uniform(size=m) < np.exp(-b * b / (2 * SCATTER_WIDTH ** 2))
        else:
            keep = np.ones(m, dtype=bool)
        ev = np.concatenate([ev, np.stack([c1, r1, c2, r2, k], axis=1)[keep]])
    return ev[:n]


def _n_pairs(sc: Scanner) -> float:
    return sc.n_cry * (sc.n_cry - 1) / 2.0 * sc.n_ring * sc.n_ring


def _contamination_level(rng, sc: Scanner, tof: TOF, n_contam: int, smooth: bool,
                         n_mc: int = 400_000) -> float:
    """Per-bin contamination scale s0 such that the expected number of
    contamination prompts over all (LOR, TOF bin) pairs is n_contam."""
    if not smooth:
        return n_contam / (_n_pairs(sc) * tof.n_tof)
    det64 = det_table(sc).astype(np.float64)
    c1, r1, c2, r2 = _random_pairs(rng, n_mc, sc)
    b = _lor_axis_distance(det64, c1, r1, c2, r2, sc)
    mean_prof = float(np.exp(-b * b / (2 * SCATTER_WIDTH ** 2)).mean())
    return n_contam / (_n_pairs(sc) * tof.n_tof * mean_prof)


def _finish(rng, trues, contam, s_true_level, s_contam, p: Problem, seed: int):
    ev = np.concatenate([trues, contam])
    s_all = np.concatenate([s_true_level, s_contam])
    order = rng.permutation(len(ev))
    p.events = np.ascontiguousarray(ev[order].astype(np.int16))
    p.s = np.ascontiguousarray(s_all[order].astype(np.float32))
    p.seed = seed
    return p


def simulate_2d(p: Problem, n_prompts: int = 100_000, contam_frac: float = 0.2,
                seed: int = 1000) -> Problem:
    """Prompts of the 2D disc phantom: trues by Monte Carlo (emission point,
    uniform in-plane direction, nearest crystals, Gaussian TOF blur), plus a
    flat contamination spread uniformly over every (LOR, TOF bin)."""
    rng = np.random.default_rng(seed)
    n_c = int(round(contam_frac * n_prompts))
    n_t = n_prompts - n_c
    trues = _trues(rng, n_t, p.scanner, p.tof, 2)
    contam = _contamination(rng, n_c, p.scanner, p.tof, smooth=False)
    s0 = _contamination_level(rng, p.scanner, p.tof, n_c, smooth=False)
    s = np.full(n_prompts, s0)
    p.x_true = phantom_2d_discs(p.image)
    p.x0 = uniform_x0(p, n_t, radius=110.0, rng=rng)
    return _finish(rng, trues, contam, s[:n_t], s[n_t:], p, seed)


CHUNK = 500_000  # events per independently seeded generation chunk


def _chunk(task):
    """One chunk of 3D events: (int16 [m, 5] events, float64 [m] distance
    of each LOR from the scanner axis)."""
    kind, count, seed_seq, sc, tof = task
    rng = np.random.default_rng(seed_seq)
    if kind == "t":
        ev = _trues(rng, count, sc, tof, 3)
    else:
        ev = _contamination(rng, count, sc, tof, smooth=True)
    det64 = det_table(sc).astype(np.float64)
    b = _lor_axis_distance(det64, ev[:, 0], ev[:, 1], ev[:, 2], ev[:, 3], sc)
    return ev.astype(np.int16), b


def _chunked(kind: str, n: int, seed_seq, sc: Scanner, tof: TOF):
    counts = [CHUNK] * (n // CHUNK) + ([n % CHUNK] if n % CHUNK else [])
    return [(kind, c, ss, sc, tof) for c, ss in zip(counts, seed_seq.spawn(len(counts)))]


def simulate_3d(p: Problem, n_prompts: int = 10_000_000, contam_frac: float = 0.3,
                seed: int = 1001, workers: int | None = None, progress=None) -> Problem:
    """Prompts of the 3D ellipsoid phantom: trues by Monte Carlo (isotropic
    directions accepted when both ends hit the crystal cylinder), plus
    contamination whose per-bin expectation is a smooth Gaussian profile in
    the LOR's distance from the axis; s_e is that expectation.  Generated in
    chunks of CHUNK events with seeds spawned from `seed`, so the result does
    not depend on the number of worker processes.  `progress(msg)`, if given,
    is called about every tenth of the chunks."""
    import os
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    root = np.random.SeedSequence(seed)
    s_main, s_t, s_c = root.spawn(3)
    rng = np.random.default_rng(s_main)
    n_c = int(round(contam_frac * n_prompts))
    n_t = n_prompts - n_c
    tasks = _chunked("t", n_t, s_t, p.scanner, p.tof) + _chunked("c", n_c, s_c, p.scanner, p.tof)
    if workers is None:
        workers = min(len(tasks), os.cpu_count() or 1, 16)
    every = max(1, len(tasks) // 10)

    def collect(it):
        out = []
        for i, r in enumerate(it):
            out.append(r)
            if progress is not None and ((i + 1) % every == 0 or i + 1 == len(tasks)):
                progress(f"generated {i + 1} of {len(tasks)} chunks of {CHUNK} events")
        return out

    res = None
    if workers > 1 and len(tasks) > 1:
        try:
            with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
                res = collect(ex.map(_chunk, tasks))
        except (RuntimeError, OSError):
            # e.g. a calling script without a __main__ guard: generate serially
            res = None
    if res is None:
        res = collect(map(_chunk, tasks))
    nt_chunks = len(_chunked("t", n_t, s_t, p.scanner, p.tof))

    def cat(parts, j, shape, dtype):
        return np.concatenate([r[j] for r in parts]) if parts else np.empty(shape, dtype)

    trues = cat(res[:nt_chunks], 0, (0, 5), np.int16)
    contam = cat(res[nt_chunks:], 0, (0, 5), np.int16)
    b = np.concatenate([cat(res[:nt_chunks], 1, (0,), np.float64), cat(res[nt_chunks:], 1, (0,), np.float64)])
    del res
    s0 = _contamination_level(rng, p.scanner, p.tof, n_c, smooth=True)
    s = s0 * np.exp(-b * b / (2 * SCATTER_WIDTH ** 2))
    del b
    p.x0 = uniform_x0(p, n_t, radius=0.9 * 0.5 * p.image.n[0] * p.image.h[0], rng=rng)
    return _finish(rng, trues, contam, s[:n_t], s[n_t:], p, seed)


def sort_by_dominant_axis(p: Problem, chunk: int = 10_000_000) -> Problem:
    """Reorders the events (and s) of `p` in place, stably, by the dominant
    axis of each event's line of response: the coordinate along which its
    two crystals differ most (the lower axis on ties).  This is the input
    order of the long static frame, whose events come grouped by dominant
    axis; inside a group the chronological order is kept.  Returns `p`."""
    det = p.det
    n = len(p.events)
    axis = np.empty(n, dtype=np.uint8)
    for a in range(0, n, chunk):
        ev = p.events[a:a + chunk].astype(np.int64)
        d = np.abs(det[ev[:, 2] + p.scanner.n_cry * ev[:, 3]] - det[ev[:, 0] + p.scanner.n_cry * ev[:, 1]])
        axis[a:a + chunk] = np.argmax(d, axis=1)  # first maximum: the lower axis
    order = np.argsort(axis, kind="stable")
    del axis
    p.events = np.ascontiguousarray(p.events[order])
    p.s = np.ascontiguousarray(p.s[order])
    return p


def uniform_x0(p: Problem, n_trues: int, radius: float, rng, n_mc: int = 200_000) -> np.ndarray:
    """Uniform starting image inside a cylinder of the given radius, scaled so
    that the summed line integrals over all LORs match the number of trues:
    the level is n_trues / sum over LORs of the chord length through that
    cylinder (exact chord geometry, Monte-Carlo over crystal pairs in 3D)."""
    sc, img = p.scanner, p.image
    det64 = det_table(sc).astype(np.float64)
    if sc.n_ring == 1:
        c1, c2 = np.triu_indices(sc.n_cry, 1)
        r1 = r2 = np.zeros_like(c1)
        scale = 1.0
    else:
        c1, r1, c2, r2 = _random_pairs(rng, n_mc, sc)
        scale = _n_pairs(sc) / n_mc
    b = _lor_axis_distance(det64, c1, r1, c2, r2, sc)
    half = np.sqrt(np.maximum(radius * radius - b * b, 0.0))
    p1 = det64[c1 + sc.n_cry * r1]
    p2 = det64[c2 + sc.n_cry * r2]
    d = p2 - p1
    sec = np.linalg.norm(d, axis=1) / np.maximum(np.linalg.norm(d[:, :2], axis=1), 1e-9)
    zlim = 0.5 * img.n[2] * img.h[2] if img.n[2] > 1 else np.inf
    # chord length through the finite cylinder: transaxial chord times the
    # obliqueness, clipped by the axial extent of the image
    chord = 2.0 * half * sec
    if np.isfinite(zlim):
        dz = np.abs(d[:, 2]) / np.linalg.norm(d, axis=1)
        zl = np.where(dz > 1e-12, 2.0 * zlim / np.maximum(dz, 1e-12), np.inf)
        chord = np.minimum(chord, zl)
    total = float(chord.sum()) * scale
    level = n_trues / total
    xs, ys = img.centres(0), img.centres(1)
    inside = (xs[None, :] ** 2 + ys[:, None] ** 2) <= radius * radius
    x0 = np.broadcast_to(inside[None, :, :], img.shape_zyx).astype(np.float32) * np.float32(level)
    return np.ascontiguousarray(x0)


def random_events(p: Problem, n: int, seed: int, min_sep: int = 1) -> np.ndarray:
    """Uniformly random events (any crystal pair with transaxial separation
    >= min_sep, any TOF bin), for operator tests."""
    rng = np.random.default_rng(seed)
    sc = p.scanner
    c1 = rng.integers(0, sc.n_cry, size=n)
    c2 = (c1 + rng.integers(min_sep, sc.n_cry - min_sep + 1, size=n)) % sc.n_cry
    r1 = rng.integers(0, sc.n_ring, size=n)
    r2 = rng.integers(0, sc.n_ring, size=n)
    k = rng.integers(-p.tof.kmax, p.tof.kmax + 1, size=n)
    return np.ascontiguousarray(np.stack([c1, r1, c2, r2, k], axis=1).astype(np.int16))


def random_events_many(p: Problem, n: int, seed: int, chunk: int = 1 << 23, workers: int = 8) -> np.ndarray:
    """Uniformly random events (two distinct crystals, any rings, any TOF
    bin) for lists of 1e8 events and more: int16 draws straight into the
    output, in chunks seeded from `seed` by SeedSequence.spawn and filled by
    a pool of threads, so the result does not depend on `workers`."""
    from concurrent.futures import ThreadPoolExecutor
    sc, kmax = p.scanner, p.tof.kmax
    out = np.empty((n, 5), dtype=np.int16)
    seeds = np.random.SeedSequence(seed).spawn((n + chunk - 1) // chunk)

    def fill(i):
        o = i * chunk
        m = min(chunk, n - o)
        rng = np.random.default_rng(seeds[i])
        e = out[o:o + m]
        c1 = rng.integers(0, sc.n_cry, m, dtype=np.int16)
        c2 = c1.astype(np.int32) + rng.integers(1, sc.n_cry, m, dtype=np.int16)
        c2[c2 >= sc.n_cry] -= sc.n_cry
        e[:, 0] = c1
        e[:, 2] = c2
        e[:, 1] = rng.integers(0, sc.n_ring, m, dtype=np.int16)
        e[:, 3] = rng.integers(0, sc.n_ring, m, dtype=np.int16)
        e[:, 4] = rng.integers(-kmax, kmax + 1, m, dtype=np.int16)

    with ThreadPoolExecutor(max(1, workers)) as ex:
        list(ex.map(fill, range(len(seeds))))
    return out


# --------------------------------------------------------------------------
# subset sequence (SplitMix64, Steele, Lea & Flood, OOPSLA 2014)

_M64 = (1 << 64) - 1


def splitmix64(seed: int, u: int) -> int:
    """Output number u (0-based) of the SplitMix64 stream started at seed."""
    x = (seed + (u + 1) * 0x9E3779B97F4A7C15) & _M64
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & _M64
    return x ^ (x >> 31)


def subset_sequence(seed: int, u0: int, count: int, n_subsets: int) -> np.ndarray:
    """Random choices for updates u0 .. u0+count-1: the prior block (index
    n_subsets) when the top bit is set (probability 1/2), otherwise data
    subset (low 63 bits) mod n_subsets (probability 1/(2 n_subsets) each)."""
    out = np.empty(count, dtype=np.int32)
    for j in range(count):
        x = splitmix64(seed, u0 + j)
        out[j] = n_subsets if (x >> 63) else (x & ((1 << 63) - 1)) % n_subsets
    return out
