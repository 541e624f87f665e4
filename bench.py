"""Benchmark of the LM-SPDHG hot path on one MI355X.

Default workload (``--workload epoch``): the 3D TOF listmode problem
(cylinder of 672 crystals x 96 rings, R = 380 mm, 200x200x96 image of 2.6
mm voxels, 33 TOF bins of 24 mm, FWHM 60 mm), 1e7 Monte-Carlo prompts with
30 % smooth contamination, 224 subsets, TV beta = 0.03.  One step = one
LM-SPDHG epoch (448 updates: data subsets and prior updates drawn with p =
1/(2n) and 1/2), continuing the reconstruction from the previous step.
Inputs are resident in HBM before the timed region; the plan (event counts,
subsets, step sizes, the sensitivity image from lm_sens) is built before it.
Per-kernel durations come from HIP events that the library records around
every 8th launch of each kernel class on its own stream, inside the timed
region.

It prints one JSON line: value = events forward- and back-projected per
second over the timed epochs, the roofline of the dominant kernel (the
data update by image tile with the z / zbar / primal step fused into it,
on its algorithmic bytes, next to its HBM traffic measured with rocprofv3)
and its binding resource (its VALU instructions per second, from counts
measured with rocprofv3, against the chip's issue rate: 256 CUs x 4 SIMDs
x 2.4 GHz / 4 cycles per wavefront instruction), the FP64 oracle timed on
a bounded sample of the same workload on the
host (cpu_baseline), the same reconstruction continued with the DTV prior
(ms per epoch and per prior update), ms per epoch with the full forward
model (per-LOR factors and a Gaussian resolution model), the warm start of the same workload (one listmode
EM-TV iteration, 28 subsets, 20 accelerated PDHG steps per denoising, with
the time and bandwidth of one denoising step), seconds per epoch of the 2D
workload (1e5 events,
128x128, 28 subsets), the time of one LMProject forward + backward of the
Poisson likelihood over 16 frames of 1e6 events and, unless --no-serve, the
serving measurement: 64 dynamic-frame requests (event counts log-uniform in
1e5..5e7, half on a 128x128x48 grid and half on the 200x200x96 one, 28
subsets, 3 epochs each) arriving as a Poisson stream at 0.7 of the
sequential solver's throughput, served by the continuous-batching Server,
with p50/p99 latency and events/s next to the one-frame-at-a-time solver on
the same arrivals, and the same 64 requests submitted at once (burst
makespan against the solver's total).

The default run ends with the long frame (below); ``--only-epoch`` runs
the 1e7-event epoch leg alone (profiler runs).

``--workload large``: the same scanner with a 300x300x96 image of 1.75 x
1.75 x 2.6 mm voxels and 5e8 events presented sorted by dominant axis: one
lm_fwd + lm_back pass over all events per step (both take their paths by
transaxial line after a counting sort of the list on the GPU), then one
LM-SPDHG epoch.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# VALU issue rate: 256 CUs x 4 SIMDs x 2.4 GHz, one wavefront instruction
# per 4 cycles on a 16-lane SIMD
VALU_PEAK_INSTR = 256 * 4 * 2.4e9 / 4
N_SUB = 224
BETA = 0.03
RHO = 0.999
SEQ_SEED = 2001
DATA_SEED = 1001
N_EVENTS = 10_000_000
LARGE_SEED = 1002
LARGE_SEQ_SEED = 2002
LARGE_EVENTS = 500_000_000
SERVE_SEED = 1003
SERVE_SEQ_SEED = 2003
SERVE_POOL = 50_000_000         # events drawn once; each request is a slice
SERVE_REQUESTS = 64
SERVE_LOAD = 0.7
SERVE_BUDGET = 96 << 30         # HBM bytes the server may hold

# Algorithmic bytes per unit of each kernel class:
#   image kernels: bytes per voxel read + written once;
#   data update: bytes per event of the per-event lists (record 16, S, mu,
#   c read, c written);
#   plain projector calls: event 10 + value 4 bytes per event.
BYTES_PER_VOXEL = {"primal": 16, "dual_image": 28, "tv": 44}
BYTES_PER_EVENT = 16 + 4 + 4 + 4 + 4
BYTES_PER_EVENT_PROJ = 10 + 4
# One accelerated PDHG step of the EM-TV denoising, per voxel: the dual pass
# reads ubar and q (4 + 12) and writes q (12); the primal pass reads u, z,
# w and q (4 + 4 + 4 + 12) and writes u and ubar (8).
BYTES_PER_VOXEL_PD = 28 + 32
# A DTV prior update in 3D, one pass per voxel (the TV pass's bytes plus
# xi): reads x, w, xi, z and T (4 + 12 + 12 + 4 + 4) and writes w, z and x
# (12 + 4 + 4).
BYTES_PER_VOXEL_DTV = 56
WARM_SUBSETS = 28               # the paper's warm start: 1 EM-TV iteration, 28 subsets,
WARM_DENOISE = 20               # 20 accelerated PDHG steps per denoising

# Sources that define each kernel class; their digest (code only, comments
# and whitespace removed) is compared with the one recorded when the HBM
# traffic below was measured.
CSRC = os.path.join(HERE, "paper_2201_05497_amd", "csrc")
KERNEL_SOURCES = {
    "data_update": ["lm_tiles.hip", "lm_tiles.hpp", "lm_project.hip", "lm_device.hpp"],
    "dual_image": ["lm_image.hip"],
    "tv": ["lm_image.hip", "lm_device.hpp"],
    "primal": ["lm_image.hip"],
    "fwd": ["lm_project.hip", "lm_device.hpp", "lm_lines.hip", "lm_sort.hip", "lm_sort.hpp"],
    "back": ["lm_project.hip", "lm_device.hpp", "lm_lines.hip", "lm_sort.hip", "lm_sort.hpp"],
}

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE (separate runs), each scaled by the counter's reading for a
# plain copy of known size in the same run; `sources` is the digest of the
# kernel's sources at the time.  The summaries are under profiles/.
PMC_TRAFFIC: dict = {
    # the data update by image tile: phase 1 (k_tile_fwd) + phase 2 (k_tile_back)
    "data_update": {"fetch_bytes": 231500000, "write_bytes": 80000000, "sources": "96219cb1c080b05d",
        "profile": "profiles/epoch_3d_200x200x96_hbm_traffic.txt"},
    "tv": {"fetch_bytes": 106400000, "write_bytes": 77000000, "sources": "5157d7dc3cd01a2c",
        "profile": "profiles/epoch_3d_200x200x96_hbm_traffic.txt"},
    "dual_image": {"fetch_bytes": 61408650, "write_bytes": 46080000, "sources": "5bbf6922e857d5c6",
        "profile": "profiles/epoch_3d_200x200x96_hbm_traffic.txt"},
    # one lm_fwd / lm_back call over the 5e8-event long frame: the counting
    # sort and the line kernels
    "fwd": {"fetch_bytes": 104600000000, "write_bytes": 52000000000, "sources": "cfd073d3f5ea28e3",
        "profile": "profiles/pass_3d_300x300x96_counters.txt"},
    "back": {"fetch_bytes": 95400000000, "write_bytes": 118500000000, "sources": "cfd073d3f5ea28e3",
        "profile": "profiles/pass_3d_300x300x96_counters.txt"},
}


# VALU wavefront instructions per launch (rocprofv3 --pmc SQ_INSTS_VALU),
# with the digest of the kernel's sources at the time.
PMC_VALU: dict = {
    "data_update": {"instr_per_launch": 33050000, "sources": "96219cb1c080b05d",
        "profile": "profiles/epoch_3d_200x200x96_l2_atomics_valu.txt"},
}




def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _code_only(src: str) -> str:
    """C++ source without comments and whitespace (a comment edit does not
    change the kernel)."""
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return re.sub(r"\s+", "", src)


def source_digest(cls: str) -> str:
    h = hashlib.sha1()
    for f in KERNEL_SOURCES[cls]:
        with open(os.path.join(CSRC, f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def traffic(cls: str):
    """Measured HBM bytes per launch of a kernel class, or None when none
    were measured or the kernel's sources changed since."""
    t = PMC_TRAFFIC.get(cls)
    if t is None or t["sources"] != source_digest(cls):
        return None
    return int(t["fetch_bytes"] + t["write_bytes"])


def binding(cls: str, us_per_launch: float) -> dict:
    """The resource that bounds the data update by tile (it issues no global
    atomics; its phase 2 is bound by its arithmetic): measured VALU
    wavefront instructions per launch / live launch duration against the
    chip's issue rate."""
    out = {"kernel": cls, "resource": "VALU wavefront instructions", "unit": "instructions/s",
           "ceiling": VALU_PEAK_INSTR, "ceiling_derivation": "256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles",
           "achieved": None, "frac": None, "instr_per_launch": None, "sources": source_digest(cls)}
    t = PMC_VALU.get(cls)
    if t is not None and t["sources"] == source_digest(cls):
        achieved = t["instr_per_launch"] / (us_per_launch * 1e-6)
        out.update(achieved=float(f"{achieved:.4g}"), frac=round(achieved / VALU_PEAK_INSTR, 3),
                   instr_per_launch=t["instr_per_launch"])
    return out


def roofline(cls: str, bytes_per_launch: float, us_per_launch: float) -> dict:
    achieved = bytes_per_launch / (us_per_launch * 1e-6) / 1e9
    tr = traffic(cls)
    out = {"kernel": cls, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
           "bytes_per_launch": int(bytes_per_launch), "us_per_launch": round(us_per_launch, 2),
           "sources": source_digest(cls)}
    if tr is not None:
        # the measured HBM traffic over the same duration (context: the
        # achieved figure above counts algorithmic bytes only)
        out["traffic_GBs"] = round(tr / (us_per_launch * 1e-6) / 1e9, 1)
    return out


def cpu_baseline(p, g, n_sample_subsets: int = 12):
    """The FP64 oracle on a bounded sample of the workload: the events of a
    few data subsets (the sample problem) are initialised untimed, then as
    many data updates and prior updates are timed and scaled to one epoch."""
    import oracle
    G = oracle.Geometry.from_problem(p)
    n = N_SUB
    ev_idx = np.concatenate([np.arange(i, len(p.events), n) for i in range(n_sample_subsets)])
    ev = p.events[ev_idx]
    s = p.s[ev_idx].astype(np.float64)
    gamma = float(np.float32(3.0 / float(p.x0.max())))
    # the sample problem has n_sample_subsets subsets: its subset i is the
    # workload's subset i (interleaved split)
    su = oracle.lm_setup(G, ev, n_sample_subsets, g, gamma, RHO)
    st = oracle.lm_init(G, ev, s, su, p.x0)
    t0 = time.perf_counter()
    n_ev = 0
    for i in range(n_sample_subsets):
        oracle.lm_update(G, ev, s, su, st, i, n_sample_subsets, BETA)
        n_ev += len(su.subsets[i])
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(n_sample_subsets):
        oracle.lm_update(G, ev, s, su, st, n_sample_subsets, n_sample_subsets, BETA)
    t_prior = time.perf_counter() - t0
    # one epoch: N events in (expected) n data updates plus n prior updates
    t_epoch = t_data * (len(p.events) / n_ev) + t_prior * (n / n_sample_subsets)
    return {
        "value": len(p.events) / t_epoch,
        "unit": "events/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{n_sample_subsets} of {n} data subsets ({n_ev} events) and {n_sample_subsets} prior "
                   f"updates on the 200x200x96 image, timed ({t_data:.1f} s + {t_prior:.1f} s) and scaled "
                   f"to one epoch ({t_epoch:.0f} s/epoch)"),
    }


def cpu_baseline_pass(p, target_s: float = 12.0):
    """The FP64 oracle's forward + back projection on a bounded sample of the
    events (first a probe of 2e4 events, then a sample sized for about
    target_s seconds), in events/s."""
    import oracle
    G = oracle.Geometry.from_problem(p)
    x = p.x0.astype(np.float64)

    def run(m):
        e = p.events[:m]
        t0 = time.perf_counter()
        oracle.fwd(G, x, e)
        oracle.back(G, np.ones(m), e)
        return time.perf_counter() - t0

    m = 20_000
    t = run(m)
    if t < target_s / 2:
        m = int(min(len(p.events), 2_000_000, m * target_s / max(t, 1e-3)))
        t = run(m)
    return {"value": m / t, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"forward + back projection of the first {m} events of the 300x300x96 workload ({t:.1f} s)"}


def calibrate_copy(torch, dev, nbytes: int = 256 << 20, reps: int = 3) -> None:
    """A plain copy kernel of known size (element-wise multiply by one:
    nbytes read and nbytes written per launch), for scaling the HBM
    counters of a profiler run."""
    a = torch.ones(nbytes // 4, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    log(f"copy calibration: {reps} launches, {nbytes} bytes read and {nbytes} bytes written each")


# --------------------------------------------------------------------------- epoch


def epoch_leg(args, torch, P, lmsynth):
    dev = torch.device("cuda", 0)
    n_events = args.events or N_EVENTS
    t0 = time.perf_counter()
    p = lmsynth.simulate_3d(lmsynth.config_3d(), n_prompts=n_events, seed=DATA_SEED)
    log(f"generated {len(p.events)} events in {time.perf_counter() - t0:.1f} s")
    G = P.Geometry.from_problem(p, device=dev)
    ev = G.events(p.events)
    s = torch.as_tensor(p.s, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = P.lm_sens(G)
    torch.cuda.synchronize()
    t_sens = time.perf_counter() - t0
    log(f"lm_sens over {G.n_cry * G.n_ring * (G.n_cry * G.n_ring - 1) // 2} crystal pairs: {t_sens:.2f} s")
    gamma = float(np.float32(3.0 / float(p.x0.max())))
    t0 = time.perf_counter()
    plan = P.Plan(G, ev, s, N_SUB, gamma, RHO, BETA, g=g)
    t_plan = time.perf_counter() - t0
    x = torch.as_tensor(p.x0, device=dev).clone()
    plan.init(x)
    torch.cuda.synchronize()
    log(f"plan + init: {t_plan:.2f} s")
    perm, off = plan.layout()
    sizes = (off[1:] - off[:-1]).cpu().numpy()

    u = 0
    seqs = []
    for _ in range(args.warmup + args.steps):
        seqs.append(lmsynth.subset_sequence(SEQ_SEED, u, 2 * N_SUB, N_SUB))
        u += 2 * N_SUB
    for k in range(args.warmup):
        plan.epoch(x, seqs[k])
    torch.cuda.synchronize()
    if args.timing_every > 0:
        plan.timing(args.timing_every)
    plan.set_tracing(args.trace)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.warmup, args.warmup + args.steps):
        plan.epoch(x, seqs[k])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    plan.set_tracing(False)
    timing = plan.get_timing() if args.timing_every > 0 else None
    plan.timing(0)
    dtv = dtv_epochs(torch, P, lmsynth, plan, x, G, u)
    plan.destroy()
    full_model = full_model_epochs(torch, P, lmsynth, G, ev, s, g, p, gamma)

    timed = seqs[args.warmup:]
    n_proj = sum(int(sizes[seq[seq < N_SUB]].sum()) for seq in timed)
    value = n_proj / t_total
    ms_per_step = 1e3 * t_total / args.steps
    log(f"{args.steps} epochs in {t_total:.3f} s: {ms_per_step:.2f} ms/epoch, {value:.3e} events/s")

    roof = None
    bind = None
    kernels = None
    if timing:
        nvox = G.nvox
        n_data = sum(int((seq < N_SUB).sum()) for seq in timed)
        launches = {"primal": 2 * args.steps, "data_update": n_data, "dual_image": n_data,
                    "tv": args.steps * 2 * N_SUB - n_data}
        kernels = {}
        for k, (ms, cnt) in timing.items():
            if cnt == 0:
                continue
            us = 1e3 * ms / cnt
            kernels[k] = {"us_avg": round(us, 2), "timed_launches": cnt, "launches": launches[k],
                          "ms_per_step": round(us * launches[k] / args.steps / 1e3, 3)}
            if k in BYTES_PER_VOXEL:
                kernels[k]["GBs"] = round(BYTES_PER_VOXEL[k] * nvox / (us * 1e-6) / 1e9, 1)
        du = kernels["data_update"]
        du["events_per_s"] = round(n_proj / n_data / (du["us_avg"] * 1e-6), 1)
        # a data update is two launches: the per-event pass (forward, dual
        # prox and its back projection, or the tile records) and the pass
        # over the image that takes the z / zbar / primal step (k_dual_image,
        # or the back projection by tile fused with that step); its
        # algorithmic bytes are the per-event lists and that image step
        di = kernels.get("dual_image", {"us_avg": 0.0, "ms_per_step": 0.0})
        kernels["data_update_total"] = {
            "us_avg": round(du["us_avg"] + di["us_avg"], 2), "launches": du["launches"],
            "ms_per_step": round(du["ms_per_step"] + di["ms_per_step"], 3),
            "events_per_s": round(n_proj / n_data / ((du["us_avg"] + di["us_avg"]) * 1e-6), 1)}
        shares = {k: v["ms_per_step"] for k, v in kernels.items() if k not in ("data_update", "dual_image")}
        dom = max(shares, key=shares.get)
        if dom == "data_update_total":
            bpl = BYTES_PER_EVENT * n_proj / n_data + BYTES_PER_VOXEL["dual_image"] * nvox
            roof = roofline("data_update", bpl, kernels[dom]["us_avg"])
            bind = binding("data_update", kernels[dom]["us_avg"])
        else:
            roof = roofline(dom, BYTES_PER_VOXEL[dom] * nvox, kernels[dom]["us_avg"])

    out = {
        "metric": "TOF LM fwd+back events/s + %HBM peak; LM-SPDHG s/epoch; served p50/p99",
        "value": round(value, 1),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "s_per_epoch": round(ms_per_step / 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3d_672x96_200x200x96: 1e7 TOF events (30% contamination), 224 subsets, "
                               "TV beta 0.03, one LM-SPDHG epoch per step",
                   "events": len(p.events), "subsets": N_SUB, "image": list(G.shape)},
        "roofline": roof,
        "binding": bind,
        "kernels": kernels,
        "dtv": dtv,
        "full_model": full_model,
        "setup_s": {"lm_sens": round(t_sens, 3), "plan_create": round(t_plan, 3)},
    }
    return out, p, G, g


def full_model_epochs(torch, P, lmsynth, G, ev, s, g, p, gamma, epochs: int = 2):
    """The same workload with the full forward model of Section 1, P =
    diag(m) G B: synthetic per-LOR factors m in [0.5, 0.9] (a smooth
    function of the crystal pair, the same for both orientations) and a
    Gaussian resolution model of 4.5 mm FWHM (1.73 voxels per axis).  A new
    plan from the uniform image; one warm-up and `epochs` timed epochs.
    (Its g is the sensitivity of G, a valid input for timing.)"""
    c1 = p.events[:, 0].astype(np.float64)
    c2 = p.events[:, 2].astype(np.float64)
    m = (0.5 + 0.4 * np.cos(0.23 * (c1 + c2)) ** 2).astype(np.float32)
    fwhm = (4.5 / 2.6,) * 3
    plan = P.Plan(G, ev, s, N_SUB, gamma, RHO, BETA, g=g)
    plan.set_event_factors(torch.as_tensor(m, device=G.device))
    plan.set_resolution(fwhm)
    x = torch.as_tensor(p.x0, device=G.device).clone()
    plan.init(x)
    seqs = [lmsynth.subset_sequence(SEQ_SEED, k * 2 * N_SUB, 2 * N_SUB, N_SUB) for k in range(1 + epochs)]
    plan.epoch(x, seqs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for seq in seqs[1:]:
        plan.epoch(x, seq)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    plan.destroy()
    log(f"full forward model (factors + {fwhm[0]:.2f}-voxel blur): {1e3 * t / epochs:.2f} ms/epoch")
    return {"ms_per_epoch": round(1e3 * t / epochs, 3), "fwhm_vox": [round(f, 3) for f in fwhm]}


def dtv_epochs(torch, P, lmsynth, plan, x, G, u0, epochs: int = 2):
    """The same reconstruction continued with the DTV prior (Section 3) for
    one warm-up and `epochs` timed epochs; the structural prior image is
    the phantom with flipped contrast (eta = 1 % of its largest gradient).
    One further epoch brackets every prior update with HIP events."""
    v = lmsynth.phantom_3d_ellipsoid(lmsynth.config_3d().image).astype(np.float32)
    v = v.max() - v
    gm = np.sqrt(sum(np.diff(v.astype(np.float64), axis=a, append=v[(slice(None),) * a + (slice(-1, None),)]) ** 2
                     for a in range(3)))
    plan.set_prior_image(torch.as_tensor(v, device=G.device), 0.01 * float(gm.max()))
    seqs = [lmsynth.subset_sequence(SEQ_SEED, u0 + k * 2 * N_SUB, 2 * N_SUB, N_SUB) for k in range(2 + epochs)]
    plan.epoch(x, seqs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for seq in seqs[1:-1]:
        plan.epoch(x, seq)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    # one more epoch with every launch bracketed, for the prior update alone
    plan.timing(1)
    plan.epoch(x, seqs[-1])
    ms, cnt = plan.get_timing()["tv"]
    plan.timing(0)
    plan.set_prior_image(None)
    us = 1e3 * ms / max(cnt, 1)
    log(f"DTV: {1e3 * t / epochs:.2f} ms/epoch, {us:.1f} us per prior update")
    return {"ms_per_epoch": round(1e3 * t / epochs, 3), "prior_update_us": round(us, 2),
            "prior_updates_timed": cnt,
            "prior_update_GBs": round(BYTES_PER_VOXEL_DTV * G.nvox / (us * 1e-6) / 1e9, 1)}


# --------------------------------------------------------------------------- warm start


def warm_start_leg(torch, P, G, g, p, reps: int = 2):
    """The warm start of the epoch workload (Algorithm 3): one listmode EM-TV
    iteration with 28 subsets and 20 accelerated PDHG steps per weighted TV
    denoising, from the uniform starting image.  Timed once more without
    denoising steps; the difference, over 28 x 20 steps, gives the time and
    the bandwidth of one denoising step (dual and primal pass)."""
    dev = G.device
    ev = G.events(p.events)
    s = torch.as_tensor(p.s, device=dev)
    x0 = torch.as_tensor(p.x0, device=dev)
    stream = torch.cuda.current_stream(dev)

    def timed(denoise_iter):
        ts = []
        for k in range(1 + reps):
            x = x0.clone()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e[0].record(stream)
            P.lm_emtv(G, ev, s, g, x, WARM_SUBSETS, 1, BETA, denoise_iter)
            e[1].record(stream)
            torch.cuda.synchronize()
            if k:
                ts.append(e[0].elapsed_time(e[1]))
        return float(np.mean(ts))

    ms = timed(WARM_DENOISE)
    ms_em = timed(0)
    us_step = 1e3 * (ms - ms_em) / (WARM_SUBSETS * WARM_DENOISE)
    out = {"ms": round(ms, 2), "em_steps_ms": round(ms_em, 2), "subsets": WARM_SUBSETS,
           "denoise_iter": WARM_DENOISE, "events_per_s": round(len(p.events) / (ms * 1e-3), 1),
           "denoise_step_us": round(us_step, 2),
           "denoise_GBs": round(BYTES_PER_VOXEL_PD * G.nvox / (us_step * 1e-6) / 1e9, 1) if us_step > 0 else None}
    log(f"warm start (EM-TV, {WARM_SUBSETS} subsets): {ms:.1f} ms, EM steps alone {ms_em:.1f} ms, "
        f"{us_step:.1f} us per denoising step")
    return out


# --------------------------------------------------------------------------- 2D


def leg_2d(torch, P, lmsynth, epochs: int = 10):
    """LM-SPDHG seconds per epoch on the 2D workload (360 crystals, 128x128
    image, 1e5 events, 28 subsets, TV beta 0.03): 10 epochs after one
    warm-up epoch, on the plan's stream."""
    dev = torch.device("cuda", 0)
    p = lmsynth.simulate_2d(lmsynth.config_2d())
    G = P.Geometry.from_problem(p, device=dev)
    ev = G.events(p.events)
    s = torch.as_tensor(p.s, device=dev)
    g = P.lm_sens(G)
    gamma = float(np.float32(3.0 / float(p.x0.max())))
    n = 28
    plan = P.Plan(G, ev, s, n, gamma, RHO, BETA, g=g)
    x = torch.as_tensor(p.x0, device=dev).clone()
    plan.init(x)
    seqs = [lmsynth.subset_sequence(2000, k * 2 * n, 2 * n, n) for k in range(epochs + 1)]
    plan.epoch(x, seqs[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, epochs + 1):
        plan.epoch(x, seqs[k])
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / epochs
    plan.destroy()
    log(f"2D workload: {1e3 * t:.2f} ms per epoch ({2 * n} updates)")
    return {"workload": "2d_360_128x128: 1e5 TOF events, 28 subsets, TV beta 0.03", "epochs": epochs,
            "s_per_epoch": round(t, 6), "us_per_update": round(1e6 * t / (2 * n), 2)}


# --------------------------------------------------------------------------- convergence


CONV_SUBSETS = (28, 56, 112, 224)
CONV_EPOCHS = (1, 2, 3, 5, 7, 10, 15, 20, 30, 50, 70, 100)
CONV_REF_EPOCHS = 20000        # reference: LM-SPDHG with one subset (2 updates per epoch)
CONV_REF_SUBSETS = 1


def convergence_leg(torch, P, lmsynth):
    """The convergence study of Section 3 on the 2D workload (the stand-in
    for the 2D BrainWeb slice; TV beta 0.03): from the paper's warm start
    (one listmode EM-TV iteration with 28 subsets), LM-SPDHG with 28, 56,
    112 and 224 subsets for 100 epochs (an epoch, the paper's iteration, is
    2n updates), with the relative cost c_rel(x) = (c(x) - c(x*)) / (c(x0) -
    c(x*)) (c from lm_cost, the listmode Eq. 1) and PSNR(x) = 20 log10
    (max x* / RMSE(x, x*)) along the way.  The paper's reference is 20000
    iterations of deterministic PDHG; here x* is 20000 epochs of LM-SPDHG
    with one subset (the data and the prior dual drawn with probability
    1/2 each), checked against 2000 epochs with 28 subsets."""
    dev = torch.device("cuda", 0)
    p = lmsynth.simulate_2d(lmsynth.config_2d())
    G = P.Geometry.from_problem(p, device=dev)
    ev = G.events(p.events)
    s = torch.as_tensor(p.s, device=dev)
    g = P.lm_sens(G)
    x0 = torch.as_tensor(p.x0, device=dev).clone()
    P.lm_emtv(G, ev, s, g, x0, 28, 1, BETA, 20)  # warm start
    gamma = float(np.float32(3.0 / float(x0.max())))
    cost = lambda x: P.lm_cost(G, x, ev, s, g, BETA)[0]

    def run(n, epochs, seed, checkpoints=()):
        plan = P.Plan(G, ev, s, n, gamma, RHO, BETA, g=g)
        x = x0.clone()
        plan.init(x)
        snaps = {}
        # one call per stretch of epochs between checkpoints (at most 1000)
        stops = sorted(set(list(checkpoints) + list(range(1000, epochs, 1000)) + [epochs]))
        seqs, done = [], 0
        for e in stops:
            seqs.append((e, lmsynth.subset_sequence(seed, done * 2 * n, (e - done) * 2 * n, n)))
            done = e
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_run = 0.0
        for ep, seq in seqs:
            plan.epoch(x, seq)
            if ep in checkpoints:
                torch.cuda.synchronize()
                t_run += time.perf_counter() - t0
                snaps[ep] = (x.cpu().numpy().astype(np.float64), cost(x))
                t0 = time.perf_counter()
        torch.cuda.synchronize()
        t_run += time.perf_counter() - t0
        plan.destroy()
        return x, snaps, t_run

    t0 = time.perf_counter()
    xr, _, t_ref = run(CONV_REF_SUBSETS, CONV_REF_EPOCHS, 3000)
    xr28, _, _ = run(28, 2000, 3001)
    c_star, c_28 = cost(xr), cost(xr28)
    c0 = cost(x0)
    x_star = xr.cpu().numpy().astype(np.float64)
    mx = float(np.abs(x_star).max())

    def psnr(x):
        mse = float(np.mean((x - x_star) ** 2))
        return float("inf") if mse == 0 else 20.0 * np.log10(mx / np.sqrt(mse))

    curves = {}
    for n in CONV_SUBSETS:
        _, snaps, t_run = run(n, max(CONV_EPOCHS), 3100 + n, CONV_EPOCHS)
        curves[str(n)] = {"epochs": list(CONV_EPOCHS),
                          "c_rel": [float(f"{(snaps[e][1] - c_star) / (c0 - c_star):.4g}") for e in CONV_EPOCHS],
                          "psnr_db": [round(psnr(snaps[e][0]), 2) for e in CONV_EPOCHS],
                          "s_per_epoch": round(t_run / max(CONV_EPOCHS), 6)}
        log(f"convergence: {n} subsets: c_rel {curves[str(n)]['c_rel'][-1]:.3g}, "
            f"PSNR {curves[str(n)]['psnr_db'][-1]:.1f} dB after {max(CONV_EPOCHS)} epochs")
    out = {"workload": "2d_360_128x128: 1e5 TOF events, TV beta 0.03, warm start 1 EM-TV iteration (28 subsets)",
           "reference": {"subsets": CONV_REF_SUBSETS, "epochs": CONV_REF_EPOCHS, "cost": c_star, "s": round(t_ref, 3),
                         "cost_x0": c0,
                         "check": {"subsets": 28, "epochs": 2000,
                                   "c_rel": float(f"{(c_28 - c_star) / (c0 - c_star):.3g}"),
                                   "psnr_db": round(psnr(xr28.cpu().numpy().astype(np.float64)), 2)}},
           "curves": curves, "s": round(time.perf_counter() - t0, 2)}
    return out


# --------------------------------------------------------------------------- autograd


def autograd_leg(torch, P, lmsynth, frames: int = 16, per_frame: int = 1_000_000, reps: int = 3):
    """LMProject forward + backward of the listmode Poisson negative
    log-likelihood over 16 frames of 1e6 events on 128x128x48 images."""
    from paper_2201_05497_amd.autograd import poisson_nll
    dev = torch.device("cuda", 0)
    p = lmsynth.simulate_3d(lmsynth.config_serving_small(), n_prompts=frames * per_frame, seed=1005)
    G = P.Geometry.from_problem(p, device=dev)
    ev = G.events(p.events)
    s = torch.as_tensor(p.s, device=dev)
    g = P.lm_sens(G).expand(frames, *G.shape).contiguous()
    rng = np.random.default_rng(1005)
    x = torch.as_tensor(rng.uniform(0.5, 1.5, size=(frames,) + G.shape).astype(np.float32), device=dev)
    off = [f * per_frame for f in range(frames + 1)]
    ts = []
    for k in range(reps + 1):
        xr = x.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = poisson_nll(xr, G, ev, s, g, off)
        loss.backward()
        torch.cuda.synchronize()
        if k:
            ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    log(f"autograd: {frames} frames x {per_frame} events forward + backward in {1e3 * t:.1f} ms")
    return {"workload": "16 frames x 1e6 events, 128x128x48, Poisson NLL forward + backward", "ms": round(1e3 * t, 2),
            "events_per_s": round(frames * per_frame / t, 1)}


# --------------------------------------------------------------------------- serving


def serving_leg(torch, P, lmsynth, G3, g3, p3, n_req: int = SERVE_REQUESTS, max_active: int = 8,
                burst_test: bool = True):
    """64 Poisson-arrival requests served by Server, against the plain
    solver one request at a time on the same arrivals (its latencies follow
    from the measured service times of each request run alone)."""
    import dataclasses
    from paper_2201_05497_amd.serving import Request, Server, latency_stats, solve
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(SERVE_SEED)
    t0 = time.perf_counter()
    pool = lmsynth.simulate_3d(lmsynth.config_3d(), n_prompts=SERVE_POOL, seed=SERVE_SEED, progress=log)
    log(f"serving: generated an event pool of {len(pool.events)} in {time.perf_counter() - t0:.1f} s")
    small = dataclasses.replace(lmsynth.config_serving_small(), scanner=p3.scanner, tof=p3.tof)
    G_small = P.Geometry.from_problem(small, device=dev)
    g_small = P.lm_sens(G_small)
    geoms = [(small, G_small, g_small), (p3, G3, g3)]
    # a unit starting image per grid (level for one true), scaled per request
    units = [lmsynth.uniform_x0(pg, 1, radius=0.9 * 0.5 * pg.image.n[0] * pg.image.h[0], rng=rng)
             for pg, _, _ in geoms]
    counts = np.exp(rng.uniform(np.log(1e5), np.log(5e7), n_req)).astype(np.int64)
    grid = rng.integers(0, 2, n_req)
    reqs = []
    for i in range(n_req):
        n = int(counts[i])
        o = int(rng.integers(0, len(pool.events) - n + 1))
        _, Gi, _ = geoms[grid[i]]
        x0 = (units[grid[i]] * np.float32(round(0.7 * n))).astype(np.float32)
        reqs.append(Request(geom=Gi, events=pool.events[o:o + n], s=pool.s[o:o + n], x0=x0, n_subsets=28,
                            epochs=3, beta=BETA, rho=RHO, seq_seed=SERVE_SEQ_SEED + i, name=f"r{i}"))
    work = float(sum(r.events.shape[0] * r.epochs for r in reqs))

    # the plain solver, one request at a time (one untimed warm-up first)
    solve(reqs[0], dev, g=geoms[grid[0]][2])
    service = []
    for i, r in enumerate(reqs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solve(r, dev, g=geoms[grid[i]][2])
        service.append(time.perf_counter() - t0)
    service = np.array(service)
    log(f"serving: sequential solver {service.sum():.2f} s for {n_req} requests ({work / service.sum():.3e} events/s)")
    rate = SERVE_LOAD / service.mean()
    gaps = rng.exponential(1.0 / rate, n_req)
    arrival = np.cumsum(gaps) - gaps[0]
    fin = 0.0
    lat_seq = np.empty(n_req)
    for i in range(n_req):
        fin = max(arrival[i], fin) + service[i]
        lat_seq[i] = fin - arrival[i]

    srv = Server(hbm_budget=SERVE_BUDGET, device=dev, max_active=max_active)
    srv.warm(G_small, g_small)
    srv.warm(G3, g3)
    t0 = time.perf_counter()
    futs = []
    for i in range(n_req):
        wait = t0 + arrival[i] - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        futs.append(srv.submit(reqs[i]))
    res = [f.result() for f in futs]
    srv.close()
    st = latency_stats(res)
    # the same requests all at once: the server's throughput against the
    # solver's back-to-back total
    burst = Server(hbm_budget=SERVE_BUDGET, device=dev, max_active=max_active)
    burst.warm(G_small, g_small)
    burst.warm(G3, g3)
    t0 = time.perf_counter()
    bres = [f.result() for f in [burst.submit(r) for r in reqs]]
    t_burst = time.perf_counter() - t0
    burst.close()
    log(f"serving: all {n_req} at once in {t_burst:.2f} s ({work / t_burst:.3e} events/s) against "
        f"{service.sum():.2f} s one at a time")
    log(f"serving: p50 {st['p50_s']:.3f} s, p99 {st['p99_s']:.3f} s, {st['events_per_s']:.3e} events/s "
        f"(sequential p50 {np.percentile(lat_seq, 50):.3f} s, p99 {np.percentile(lat_seq, 99):.3f} s)")
    return {
        "requests": n_req, "events_total": int(counts.sum()), "epochs": 3, "subsets": 28,
        "offered_load": SERVE_LOAD, "arrival_rate_per_s": round(rate, 3),
        "p50_s": round(st["p50_s"], 4), "p99_s": round(st["p99_s"], 4),
        "events_per_s": round(work / st["makespan_s"], 1), "makespan_s": round(st["makespan_s"], 3),
        "peak_hbm_bytes": int(srv.peak_bytes),
        "sequential": {"p50_s": round(float(np.percentile(lat_seq, 50)), 4),
                       "p99_s": round(float(np.percentile(lat_seq, 99)), 4),
                       "events_per_s": round(work / fin, 1),
                       "busy_events_per_s": round(work / service.sum(), 1),
                       "makespan_s": round(float(fin), 3)},
        "burst": {"makespan_s": round(t_burst, 3), "events_per_s": round(work / t_burst, 1),
                  "p99_s": round(float(np.percentile([r.latency for r in bres], 99)), 4),
                  "sequential_makespan_s": round(float(service.sum()), 3)},
        "note": "events/s counts events x epochs; requests are slices of one 5e7-event pool of the 3D phantom",
    }


# --------------------------------------------------------------------------- large


def large_leg(args, torch, P, lmsynth, passes: int, warmup: int):
    """The long static frame: 5e8 events on the 300x300x96 image, presented
    sorted by dominant axis.  `warmup` untimed and `passes` timed lm_fwd +
    lm_back passes over all events (lm_back takes its by-line path for such
    a list), then one LM-SPDHG epoch (224 subsets) after a warm-up epoch."""
    dev = torch.device("cuda", 0)
    n_events = args.large_events or LARGE_EVENTS
    t0 = time.perf_counter()
    p = lmsynth.simulate_3d(lmsynth.config_3d_large(), n_prompts=n_events, seed=LARGE_SEED, progress=log)
    # the long static frame's events arrive sorted by dominant axis
    lmsynth.sort_by_dominant_axis(p)
    log(f"large: generated {len(p.events)} events (sorted by dominant axis) in {time.perf_counter() - t0:.1f} s")
    G = P.Geometry.from_problem(p, device=dev)
    ev = G.events(p.events)
    s = torch.as_tensor(p.s, device=dev)
    x = torch.as_tensor(p.x0, device=dev).clone()
    N = len(p.events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = P.lm_sens(G)
    torch.cuda.synchronize()
    t_sens = time.perf_counter() - t0
    log(f"large: lm_sens {t_sens:.2f} s")

    out = torch.empty(N, device=dev)
    v = torch.ones(N, device=dev)
    img = G.zeros()
    stream = torch.cuda.current_stream(dev)
    tf, tb = [], []
    for k in range(warmup + passes):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        img.zero_()
        e[0].record(stream)
        P.lm_fwd(G, x, ev, out)
        e[1].record(stream)
        P.lm_back(G, v, ev, img)
        e[2].record(stream)
        torch.cuda.synchronize()
        if k >= warmup:
            tf.append(e[0].elapsed_time(e[1]))
            tb.append(e[1].elapsed_time(e[2]))
        log(f"large: pass {k}: lm_fwd {e[0].elapsed_time(e[1]):.1f} ms, lm_back {e[1].elapsed_time(e[2]):.1f} ms")
    del out, v, img
    t_fwd, t_back = float(np.mean(tf)), float(np.mean(tb))
    t_pass = t_fwd + t_back

    gamma = float(np.float32(3.0 / float(p.x0.max())))
    t0 = time.perf_counter()
    plan = P.Plan(G, ev, s, N_SUB, gamma, RHO, BETA, g=g)
    plan.init(x)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    log(f"large: plan + init {t_plan:.2f} s")
    seq0 = lmsynth.subset_sequence(LARGE_SEQ_SEED, 0, 2 * N_SUB, N_SUB)
    seq1 = lmsynth.subset_sequence(LARGE_SEQ_SEED, 2 * N_SUB, 2 * N_SUB, N_SUB)
    plan.epoch(x, seq0)
    torch.cuda.synchronize()
    plan.timing(args.timing_every)
    t0 = time.perf_counter()
    plan.epoch(x, seq1)
    torch.cuda.synchronize()
    t_epoch = time.perf_counter() - t0
    timing = plan.get_timing() if args.timing_every > 0 else None
    plan.destroy()
    del plan, ev, s, x, g
    torch.cuda.empty_cache()
    log(f"large: epoch {t_epoch:.3f} s")
    kernels = None
    if timing:
        kernels = {k: {"us_avg": round(1e3 * ms / c, 2), "timed_launches": c} for k, (ms, c) in timing.items() if c}
    # algorithmic bytes: each call reads the 10-byte events and writes (lm_fwd)
    # or reads (lm_back) 4 bytes per event
    roof_fwd = roofline("fwd", BYTES_PER_EVENT_PROJ * N, t_fwd * 1e3)
    roof_back = roofline("back", BYTES_PER_EVENT_PROJ * N, t_back * 1e3)
    a_pass = 2 * BYTES_PER_EVENT_PROJ * N / (t_pass * 1e-3) / 1e9
    res = {
        "workload": "3d_672x96_300x300x96: 5e8 TOF events (30% contamination) sorted by dominant axis",
        "events": N, "subsets": N_SUB, "image": list(G.shape), "passes": passes, "warmup": warmup,
        "value": round(N / (t_pass * 1e-3), 1), "unit": "events/s (lm_fwd + lm_back pass)",
        "pass_ms": round(t_pass, 3), "s_per_epoch": round(t_epoch, 4),
        "pass": {"fwd_ms": round(t_fwd, 2), "back_ms": round(t_back, 2),
                 "fwd_events_per_s": round(N / (t_fwd * 1e-3), 1),
                 "back_events_per_s": round(N / (t_back * 1e-3), 1)},
        "roofline": {"kernel": "lm_fwd + lm_back", "bound": "hbm", "achieved": round(a_pass, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(a_pass / HBM_PEAK_GBS, 5),
                     "traffic": (None if roof_fwd["traffic"] is None or roof_back["traffic"] is None
                                 else int(roof_fwd["traffic"] + roof_back["traffic"])),
                     "bytes_per_pass": int(2 * BYTES_PER_EVENT_PROJ * N)},
        "roofline_fwd": roof_fwd,
        "roofline_back": roof_back,
        "kernels": kernels,
        "setup_s": {"lm_sens": round(t_sens, 3), "plan_create_init": round(t_plan, 3)},
    }
    return res, p


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=("epoch", "large"), default="epoch",
                    help="epoch: every leg (the 1e7-event epoch is the JSON line's value); large: the 5e8-event "
                         "long frame alone")
    ap.add_argument("--events", type=int, default=0, help="event count of the epoch workload (0: 1e7)")
    ap.add_argument("--large-events", type=int, default=0, help="event count of the long frame (0: 5e8)")
    ap.add_argument("--no-large", action="store_true", help="skip the 5e8-event long frame")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--only-epoch", action="store_true",
                    help="the 1e7-event epoch leg alone (for profiler runs): no warm start, 2D, convergence, "
                         "autograd, serving or long-frame legs")
    ap.add_argument("--timing-every", type=int, default=8,
                    help="bracket every k-th launch of each kernel class with HIP events (0: no per-kernel timing)")
    ap.add_argument("--trace", action="store_true",
                    help="roctx ranges per update in the timed epochs of the epoch leg (lm_plan_set_tracing)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with a plain copy of known size (for scaling profiler HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; sharding over several GPUs is "
                                   "designed but not built", "n_gpus": args.gpus}))
        return 2

    import torch
    import lmsynth
    import paper_2201_05497_amd as P

    if args.workload == "large":
        large, p = large_leg(args, torch, P, lmsynth, passes=args.steps, warmup=args.warmup)
        out = {"metric": "TOF LM fwd+back events/s + %HBM peak; LM-SPDHG s/epoch; served p50/p99",
               "value": large["value"], "unit": "events/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": large["pass_ms"], "s_per_epoch": large["s_per_epoch"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
               "data": "synthetic",
               "config": {"workload": large["workload"] + "; one lm_fwd + lm_back pass per step, then one "
                                                          "LM-SPDHG epoch (224 subsets)",
                          "events": large["events"], "subsets": N_SUB, "image": large["image"]},
               "roofline": large["roofline"], "large": large}
        cpu = None
        if not args.no_cpu_baseline:
            t0 = time.perf_counter()
            cpu = cpu_baseline_pass(p)
            log(f"cpu baseline: {cpu['value']:.3e} events/s ({time.perf_counter() - t0:.1f} s)")
    else:
        out, p, G, g = epoch_leg(args, torch, P, lmsynth)
        if not args.only_epoch:
            out["warm_start"] = warm_start_leg(torch, P, G, g, p)
            out["epoch_2d"] = leg_2d(torch, P, lmsynth)
            out["convergence"] = convergence_leg(torch, P, lmsynth)
            out["autograd"] = autograd_leg(torch, P, lmsynth)
        if not args.no_serve and not args.only_epoch:
            out["served"] = serving_leg(torch, P, lmsynth, G, g, p)
        cpu = None
        if not args.no_cpu_baseline:
            t0 = time.perf_counter()
            # the oracle's cost does not depend on the values of g; it gets its
            # own input (no GPU output is ever fed to the oracle)
            cpu = cpu_baseline(p, np.ones(G.shape))
            log(f"cpu baseline: {cpu['value']:.3e} events/s ({time.perf_counter() - t0:.1f} s)")
        del G, g, p
        torch.cuda.empty_cache()
        if not args.no_large and not args.only_epoch:
            # the long frame: a few passes whatever --steps says, to keep the run short
            large, pl = large_leg(args, torch, P, lmsynth, passes=min(args.steps, 5), warmup=min(args.warmup, 2))
            if not args.no_cpu_baseline:
                t0 = time.perf_counter()
                large["cpu_baseline"] = cpu_baseline_pass(pl)
                log(f"cpu baseline (long frame pass): {large['cpu_baseline']['value']:.3e} events/s "
                    f"({time.perf_counter() - t0:.1f} s)")
            del pl
            out["large"] = large
    out["cpu_baseline"] = cpu
    if args.calibrate_copy:
        calibrate_copy(torch, torch.device("cuda", 0))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
