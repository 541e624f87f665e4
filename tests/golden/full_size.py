"""Expected values of the full-size parity tests, computed by the FP64
oracle alone (it imports only ``oracle``, ``lmsynth`` and the test helpers
that call them; nothing here touches the HIP library).

Three cases:

* ``c2``: the 3D workload exactly as the benchmark runs it: 1e7 prompts of
  the ellipsoid phantom (seed 1001), 224 interleaved subsets, TV beta 0.03,
  rho 0.999, gamma = 3 / max(x0) rounded to float32, the subset sequence of
  SplitMix64 seed 2001 with the update counter running across epochs
  (Algorithm 2, five epochs of 2n updates).  The sensitivity image is the
  decimated-scanner input of ``tests.helpers.sens_3d_input`` (the full
  scanner's P^T 1 would take the oracle hours); both sides receive it.
  Stored: x after every epoch, z and zbar at the end, the dual complement
  c = 1 - y on every 32nd event and the TV dual w on three z slices.
* ``c3``: updates at the shape of the long static frame: the 300x300x96
  image of 1.75 x 1.75 x 2.6 mm, 8.9e6 prompts (seed 1012) presented sorted
  by dominant axis, 4 interleaved subsets (2.2e6 events per data update,
  the subset size of 5e8 events in 224 subsets), from a seeded state
  (``c3_inputs``): three data and three prior updates in one call.
  Stored: x, z, zbar and w on three z slices, c on every 17th event.
* ``sens``: P^T 1 over every crystal pair and TOF bin of a scanner with the
  full 672-crystal ring and 3 rings (Section 2 after Eq. lm_stepsizes: the
  back projection of a sinogram of ones), on a 200x200x5 grid of 2.6 mm.

Usage: ``python -m tests.golden.full_size compute c2|c3|sens`` (minutes to
about half an hour of one core each; raw results go to ``.cache/``), then
``python -m tests.golden.full_size pack`` writes the ``.npz`` files of this
directory from them.  ``python -m tests.golden.full_size sensitivity``
(after ``compute c2``; about an hour) writes ``c2_sensitivity.json``, the
oracle's own sensitivity of c2 to float32 rounding of its state.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import lmsynth  # noqa: E402

RAW = os.path.join(ROOT, ".cache", "golden_raw")

C2 = dict(n_events=10_000_000, seed=1001, n_sub=224, epochs=5, seq_seed=2001, beta=0.03, rho=0.999,
          c_stride=32, w_slices=(0, 48, 95))
C3 = dict(n_events=8_900_000, seed=1012, state_seed=1013, n_sub=4, seq=(0, 4, 1, 4, 4, 2), beta=0.03, rho=0.999,
          c_stride=17, slices=(0, 47, 95))
SENS = dict(n_cry=672, n_ring=3, radius=380.0, pitch=2.6, n=(200, 200, 5), h=(2.6, 2.6, 2.6))


def gamma_of(x0) -> float:
    """gamma = 3 / max(x0) (Section 3), rounded to float32 so that both
    sides use the same number."""
    return float(np.float32(3.0 / float(np.max(x0))))


# ----------------------------------------------------------------- inputs


def c2_inputs():
    """(problem, g) of the 3D workload as benchmarked."""
    from tests.helpers import problem_3d, sens_3d_input
    p = problem_3d(C2["n_events"], seed=C2["seed"])
    return p, sens_3d_input().astype(np.float32)


def c2_sequence(epoch: int) -> np.ndarray:
    n = C2["n_sub"]
    return lmsynth.subset_sequence(C2["seq_seed"], epoch * 2 * n, 2 * n, n)


def c3_inputs():
    """(problem, g, state) of the long-frame-shaped update case.  The state
    (x, z, zbar, w, c) is seeded: z and zbar around g, w inside the beta
    ball, c = 1 - y in [0.2, 0.8]."""
    from tests.helpers import sens_3d_input
    cfg = lmsynth.config_3d_large()
    p = lmsynth.simulate_3d(cfg, n_prompts=C3["n_events"], seed=C3["seed"])
    lmsynth.sort_by_dominant_axis(p)
    g = sens_3d_input(large=True).astype(np.float32)
    rng = np.random.default_rng(C3["state_seed"])
    zyx = g.shape
    beta = C3["beta"]
    gm = float(g.mean())
    z0 = (g + gm * rng.uniform(-0.05, 0.05, zyx)).astype(np.float32)
    zb0 = (g + gm * rng.uniform(-0.05, 0.05, zyx)).astype(np.float32)
    w0 = rng.normal(0.0, beta / 3, (3,) + zyx).astype(np.float32)
    nrm = np.sqrt((w0.astype(np.float64) ** 2).sum(0))
    w0 *= np.minimum(1.0, beta / np.maximum(nrm, 1e-30)).astype(np.float32)
    c0 = rng.uniform(0.2, 0.8, len(p.events)).astype(np.float32)
    state = {"x": p.x0.astype(np.float32), "z": z0, "zbar": zb0, "w": w0, "c": c0}
    return p, g, state


def sens_problem():
    sc = lmsynth.Scanner(SENS["n_cry"], SENS["n_ring"], SENS["radius"], SENS["pitch"])
    img = lmsynth.ImageGeom(SENS["n"], SENS["h"])
    tof = lmsynth.config_3d().tof
    return lmsynth.Problem("sens_672x3", sc, img, tof, 1, 1, 0.0)


# ----------------------------------------------------------------- compute


def _log(msg):
    print(f"[golden {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def compute_c2():
    import oracle
    p, g = c2_inputs()
    G = oracle.Geometry.from_problem(p)
    n = C2["n_sub"]
    t0 = time.time()
    su = oracle.lm_setup(G, p.events, n, g.astype(np.float64), gamma_of(p.x0), C2["rho"])
    _log(f"c2 setup {time.time() - t0:.0f} s")
    s = p.s.astype(np.float64)
    st = oracle.lm_init(G, p.events, s, su, p.x0)
    _log(f"c2 init {time.time() - t0:.0f} s")
    out = {}
    for ep in range(C2["epochs"]):
        seq = c2_sequence(ep)
        for i in seq:
            oracle.lm_update(G, p.events, s, su, st, int(i), n, C2["beta"])
        out[f"x{ep + 1}"] = st.x.astype(np.float32)
        _log(f"c2 epoch {ep + 1} {time.time() - t0:.0f} s")
    out["z"] = st.z.astype(np.float32)
    out["zbar"] = st.zbar.astype(np.float32)
    out["c"] = (1.0 - st.y[::C2["c_stride"]]).astype(np.float32)
    out["w"] = st.w[:, list(C2["w_slices"])].astype(np.float32)
    out["u"] = np.int64(st.u)
    os.makedirs(RAW, exist_ok=True)
    np.savez(os.path.join(RAW, "c2.npz"), **out)


def compute_c3():
    import oracle
    p, g, s0 = c3_inputs()
    G = oracle.Geometry.from_problem(p)
    n = C3["n_sub"]
    t0 = time.time()
    su = oracle.lm_setup(G, p.events, n, g.astype(np.float64), gamma_of(p.x0), C3["rho"])
    _log(f"c3 setup {time.time() - t0:.0f} s")
    st = oracle.LMState(x=s0["x"].astype(np.float64), z=s0["z"].astype(np.float64),
                        zbar=s0["zbar"].astype(np.float64), w=s0["w"].astype(np.float64),
                        y=1.0 - s0["c"].astype(np.float64), u=0)
    s = p.s.astype(np.float64)
    for i in C3["seq"]:
        oracle.lm_update(G, p.events, s, su, st, int(i), n, C3["beta"])
        _log(f"c3 update {i} {time.time() - t0:.0f} s")
    sl = list(C3["slices"])
    out = {"x": st.x[sl].astype(np.float32), "z": st.z[sl].astype(np.float32),
           "zbar": st.zbar[sl].astype(np.float32), "w": st.w[:, sl].astype(np.float32),
           "c": (1.0 - st.y[::C3["c_stride"]]).astype(np.float32), "u": np.int64(st.u)}
    os.makedirs(RAW, exist_ok=True)
    np.savez(os.path.join(RAW, "c3.npz"), **out)


def compute_sens():
    import oracle
    p = sens_problem()
    t0 = time.time()
    g = oracle.sens(oracle.Geometry.from_problem(p))
    _log(f"sens {time.time() - t0:.0f} s")
    os.makedirs(RAW, exist_ok=True)
    np.savez(os.path.join(RAW, "sens.npz"), g=g)


def compute_c2_sensitivity():
    """The oracle's own sensitivity on c2: the same five epochs with its
    state (x, z, zbar, w and y) rounded to float32 after every update,
    against the stored FP64 run (``compute c2`` first).  Writes
    ``c2_sensitivity.json``: the sup-norm differences of x (after the last
    epoch), z, and of the TV dual w over the stored slices (relative L2 and
    sup norm over beta).  The TV dual is the ill-conditioned quantity: where
    K x is nearly zero its direction follows tiny gradients."""
    import json
    import oracle
    raw = np.load(os.path.join(RAW, "c2.npz"))
    p, g = c2_inputs()
    G = oracle.Geometry.from_problem(p)
    n = C2["n_sub"]
    t0 = time.time()
    su = oracle.lm_setup(G, p.events, n, g.astype(np.float64), gamma_of(p.x0), C2["rho"])
    s = p.s.astype(np.float64)
    st = oracle.lm_init(G, p.events, s, su, p.x0)

    def f32(v):
        return v.astype(np.float32).astype(np.float64)

    for ep in range(C2["epochs"]):
        for i in c2_sequence(ep):
            oracle.lm_update(G, p.events, s, su, st, int(i), n, C2["beta"])
            st.x, st.z, st.zbar, st.w = f32(st.x), f32(st.z), f32(st.zbar), f32(st.w)
            st.y = 1.0 - f32(1.0 - st.y)
        _log(f"c2 sensitivity epoch {ep + 1} {time.time() - t0:.0f} s")
    x5 = raw[f"x{C2['epochs']}"].astype(np.float64)
    zr = raw["z"].astype(np.float64)
    wr = raw["w"].astype(np.float64)
    wp = st.w[:, list(C2["w_slices"])]
    out = {"x_inf": float(np.abs(st.x - x5).max() / np.abs(x5).max()),
           "z_inf": float(np.abs(st.z - zr).max() / np.abs(zr).max()),
           "w_l2": float(np.linalg.norm(wp - wr) / np.linalg.norm(wr)),
           "w_inf_over_beta": float(np.abs(wp - wr).max() / C2["beta"])}
    with open(os.path.join(HERE, "c2_sensitivity.json"), "w") as f:
        json.dump(out, f, indent=1)
    _log(f"c2 sensitivity {out}")


# ----------------------------------------------------------------- storage
#
# Images are stored as integers on a grid of 2^-18 of their largest
# magnitude (rounding error at most 1.9e-6 of the maximum, 2 % of the 1e-4
# parity bound), differenced along x so that smooth regions compress, and
# packed with lzma; zbar is stored as its difference from z (the last
# update's z increment over p), on a grid of its own; per-event lists stay
# float32.

QBITS = 18


def _pack_image(a: np.ndarray):
    import lzma
    a = np.asarray(a, dtype=np.float64)
    scale = float(np.abs(a).max()) * 2.0 ** -QBITS
    if scale == 0.0:
        scale = 1.0
    q = np.rint(a / scale).astype(np.int64)
    d = np.diff(q, axis=-1, prepend=0)
    assert np.abs(d).max() < 2 ** 31
    blob = lzma.compress(d.astype("<i4").tobytes(), preset=9)
    return np.frombuffer(blob, dtype=np.uint8), np.asarray(a.shape, dtype=np.int64), scale


def _unpack_image(blob: np.ndarray, shape, scale: float) -> np.ndarray:
    import lzma
    d = np.frombuffer(lzma.decompress(blob.tobytes()), dtype="<i4").reshape(tuple(int(v) for v in shape))
    return np.cumsum(d.astype(np.int64), axis=-1).astype(np.float64) * scale


def pack() -> None:
    for name in ("c2", "c3", "sens"):
        src = os.path.join(RAW, f"{name}.npz")
        if not os.path.exists(src):
            print(f"{src} missing: run compute {name} first")
            continue
        raw = np.load(src)
        out = {}
        for k in raw.files:
            a = raw[k]
            if k == "zbar" and "z" in raw.files:
                # against z as it will be read back
                zq, zs, zsc = _pack_image(raw["z"])
                blob, shape, sc = _pack_image(a.astype(np.float64) - _unpack_image(zq, zs, zsc))
                out["dq_zbar"] = blob
                out["shape_zbar"] = shape
                out["s_zbar"] = np.float64(sc)
            elif a.ndim >= 2:
                blob, shape, sc = _pack_image(a)
                out[f"q_{k}"] = blob
                out[f"shape_{k}"] = shape
                out[f"s_{k}"] = np.float64(sc)
            else:
                out[k] = a
        dst = os.path.join(HERE, f"{name}.npz")
        np.savez(dst, **out)
        print(f"{dst}: {os.path.getsize(dst) / 1e6:.1f} MB")


def load(name: str) -> dict:
    """The stored expected values of a case: image keys as float64 arrays,
    lists as stored."""
    d = np.load(os.path.join(HERE, f"{name}.npz"))
    out = {}
    for k in d.files:
        if k.startswith("q_"):
            b = k[2:]
            out[b] = _unpack_image(d[k], d["shape_" + b], float(d["s_" + b]))
        elif not (k.startswith("s_") or k.startswith("shape_") or k.startswith("dq_")):
            out[k] = d[k]
    for k in d.files:
        if k.startswith("dq_"):  # stored as a difference from z
            b = k[3:]
            out[b] = out["z"] + _unpack_image(d[k], d["shape_" + b], float(d["s_" + b]))
    return out


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else ""
    if what == "compute":
        {"c2": compute_c2, "c3": compute_c3, "sens": compute_sens}[sys.argv[2]]()
    elif what == "pack":
        pack()
    elif what == "sensitivity":
        compute_c2_sensitivity()
    else:
        sys.exit(__doc__)
