"""GPU parity at the full size of the long static frame: 5e8 events on the
300x300x96 image of the 672 x 96-crystal scanner, through the calls and
launch configuration of the benchmark's pass and epoch on that workload
(lm_fwd and lm_back by transaxial line after a counting sort of the whole
list by crystal pair on the GPU, lm_sens, a plan of 224 subsets).  The oracle cannot
run 5e8 events; it computes sampled outputs one by one instead:

- lm_fwd (by transaxial line after the sort): the projections of sampled
  events, the events around every launch boundary of the list's own order
  and at the end of the list included, per event; every event's value
  against lm_fwd_noalloc, which projects the list per event in its own
  order, to the projection tolerance;
- lm_back: a value list that is zero except on a sample, so that the whole
  back projection equals the oracle's back projection of the sample;
- the plan: event counts, subsets and P^LM 1 of sampled events; after one
  epoch, the invariants that hold at any size (z against the back projection
  of the dual, x >= 0, y < 1).

The events are uniformly random (two distinct crystals, any rings, any TOF
bin) with planted duplicates, in place of the Monte Carlo of the phantom,
which takes minutes at this size; they reach every kind of line of
response, including those whose dominant axis is z and those that miss the
image.  Tolerances as in the other parity tests."""
import ctypes
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import lmsynth
import oracle
from paper_2201_05497_amd import _lib
from tests.helpers import img_err, proj_err, report, smooth_image

pytestmark = pytest.mark.gpu

N_EVENTS = 500_000_000
N_SUBSETS = 224
PROJ_TOL = 1e-5
BACK_TOL = 1e-4
ITER_TOL = 1e-4
RHO = 0.999
BETA = 0.03
# events per lm_fwd launch: 2^22 blocks of 256 threads, 8 lanes per event
FWD_LAUNCH = (1 << 22) * (256 // 8)


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2201_05497_amd as P
    return P


@pytest.fixture(scope="module")
def frame(P):
    p = lmsynth.config_3d_large()
    ev = lmsynth.random_events_many(p, N_EVENTS, seed=1010)
    # planted duplicates: copies of 2e5 events written over 1e6 others, half
    # of them with the crystals swapped and the TOF bin negated (same bin)
    rng = np.random.default_rng(1011)
    src = rng.integers(0, N_EVENTS, 200_000)
    dst = rng.integers(0, N_EVENTS, 1_000_000)
    cp = ev[src[rng.integers(0, len(src), len(dst))]]
    sw = rng.random(len(dst)) < 0.5
    cp[sw] = cp[sw][:, [2, 3, 0, 1, 4]]
    cp[sw, 4] = -cp[sw, 4]
    ev[dst] = cp
    del cp
    Gg = P.Geometry.from_problem(p)
    Go = oracle.Geometry.from_problem(p)
    evt = Gg.events(ev)
    report("long frame", events=N_EVENTS, planted_copies=len(dst))
    yield {"p": p, "ev": ev, "Gg": Gg, "Go": Go, "evt": evt, "planted": dst}
    del evt
    torch.cuda.empty_cache()


def _sample(k: int, seed: int, extra=()) -> np.ndarray:
    """k random event indices plus the events around every lm_fwd launch
    boundary and at the end of the list, sorted and distinct."""
    rng = np.random.default_rng(seed)
    edges = [np.arange(c - 32, c + 32) for c in range(FWD_LAUNCH, N_EVENTS, FWD_LAUNCH)]
    return np.unique(np.concatenate([rng.integers(0, N_EVENTS, k), np.arange(N_EVENTS - 32, N_EVENTS)]
                                    + edges + list(extra)))


def _sampled_counts(ev: np.ndarray, idx: np.ndarray, n_cry: int, n_det: int, chunk: int = 1 << 25) -> np.ndarray:
    """The oracle's mu_e for the events idx of the whole list.  Events of
    one bin join the same two detectors, so they share the lower detector
    id: the sub-list of events whose lower id is one of the sample's holds
    every event that can count towards a sampled one, and the oracle counts
    on that sub-list."""
    def lower(e):
        a = e[:, 0].astype(np.int32) + n_cry * e[:, 1].astype(np.int32)
        b = e[:, 2].astype(np.int32) + n_cry * e[:, 3].astype(np.int32)
        return np.minimum(a, b)

    wanted = np.zeros(n_det, dtype=bool)
    wanted[lower(ev[idx])] = True

    def select(o):
        m = wanted[lower(ev[o:o + chunk])]
        return ev[o:o + chunk][m], o + np.nonzero(m)[0]

    with ThreadPoolExecutor(8) as ex:
        parts = list(ex.map(select, range(0, len(ev), chunk)))
    pos = np.concatenate([q for _, q in parts])
    cnt = oracle.event_counts(np.concatenate([e for e, _ in parts]), n_cry)
    at = np.searchsorted(pos, idx)
    assert np.array_equal(pos[at], idx)
    return cnt[at]


def test_long_frame_pass(P, frame):
    """One lm_fwd + lm_back pass over the 5e8 events."""
    ev, Gg, Go, evt = frame["ev"], frame["Gg"], frame["Go"], frame["evt"]
    x = smooth_image(Gg.shape, 21)
    xt = torch.as_tensor(x, device="cuda")
    out = P.lm_fwd(Gg, xt, evt)
    idx = _sample(4000, 22)
    got = out[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    own = torch.full((N_EVENTS,), float("nan"), device="cuda")
    _lib.check(_lib.load().lm_fwd_noalloc(ctypes.byref(Gg._c), xt.data_ptr(), evt.data_ptr(), N_EVENTS,
                                          own.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
               "lm_fwd_noalloc")
    # |by line - per event| <= PROJ_TOL max(|per event|, 1e-3 mean |per event|) on every event
    floor = 1e-3 * float(own.abs().double().mean())
    rel = float(((out - own).abs() / own.abs().clamp_min(floor)).max())
    del out, own
    emax, emean = proj_err(got, oracle.fwd(Go, x, ev[idx]))
    report("long frame fwd", sampled=len(idx), max_err=emax, mean_err=emean, all_events_vs_per_event=rel)
    assert emax <= PROJ_TOL
    assert rel <= PROJ_TOL

    jdx = _sample(20_000, 23)
    vals = np.random.default_rng(24).uniform(-1, 1, len(jdx)).astype(np.float32)
    v = torch.zeros(N_EVENTS, device="cuda")
    v[torch.as_tensor(jdx, device="cuda")] = torch.as_tensor(vals, device="cuda")
    got = P.lm_back(Gg, v, evt).cpu().numpy()
    del v
    e = img_err(got, oracle.back(Go, vals.astype(np.float64), ev[jdx]))
    report("long frame back", nonzero=len(jdx), err=e)
    assert e <= BACK_TOL


def test_long_frame_plan_epoch(P, frame):
    """A plan of 224 subsets over the 5e8 events and one epoch."""
    p, ev, Gg, Go, evt = frame["p"], frame["ev"], frame["Gg"], frame["Go"], frame["evt"]
    sc, n = p.scanner, N_EVENTS
    g = P.lm_sens(Gg)
    # contamination per bin as in the workload: 30 % of the prompts spread
    # over every (crystal pair, TOF bin)
    s = torch.full((n,), 0.3 * n / (sc.n_det * (sc.n_det - 1) / 2 * p.tof.n_tof), device="cuda")
    x0 = lmsynth.uniform_x0(p, int(0.7 * n), radius=0.9 * 0.5 * p.image.n[0] * p.image.h[0],
                            rng=np.random.default_rng(25))
    gamma = float(np.float32(3.0 / float(x0.max())))
    plan = P.Plan(Gg, evt, s, N_SUBSETS, gamma, RHO, BETA, g=g)
    y, mu, sub, p1 = plan.lists()
    idx = _sample(2000, 26, extra=(frame["planted"][:1000],))
    it = torch.as_tensor(idx, device="cuda")
    mu_s, sub_s, p1_s = mu[it].cpu().numpy(), sub[it].cpu().numpy(), p1[it].cpu().numpy()
    del y, sub, p1
    want_mu = _sampled_counts(ev, idx, sc.n_cry, sc.n_det)
    assert np.array_equal(mu_s, want_mu)
    assert np.array_equal(sub_s, oracle.subset_ids(n, N_SUBSETS)[idx])
    emax, _ = proj_err(p1_s, oracle.fwd(Go, np.ones(Go.shape), ev[idx]))
    report("long frame plan", sampled=len(idx), mu_max=int(want_mu.max()), dup=int((want_mu > 1).sum()),
           p1_max=emax)
    assert emax <= PROJ_TOL
    assert (want_mu > 1).sum() >= 500  # the planted duplicates are among the sampled events

    x = torch.as_tensor(x0, device="cuda").clone()
    plan.init(x)
    plan.epoch(x, lmsynth.subset_sequence(2010, 0, 2 * N_SUBSETS, N_SUBSETS))
    st = plan.get_state()
    plan.destroy()
    z_ref = g.clone()
    P.lm_back(Gg, -st["c"] / mu.float(), evt, z_ref)
    z_ref -= P.tv_div(st["w"])
    einv = img_err(st["z"].cpu().numpy(), z_ref.cpu().numpy().astype(np.float64))
    report("long frame epoch", z_invariant=einv, x_min=float(x.min()), c_min=float(st["c"].min()))
    assert einv <= ITER_TOL
    assert float(x.min()) >= 0.0 and float(st["c"].min()) > 0.0
