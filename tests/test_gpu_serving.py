"""The continuous-batching server: every served reconstruction equals the
same reconstruction run alone by the plain solver (float32 atomics aside),
admission never exceeds the HBM budget, oversized requests fail cleanly and
waiting and running requests can be cancelled."""
import time
from concurrent.futures import CancelledError

import numpy as np
import pytest
import torch

import lmsynth
from tests.helpers import img_err, report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2201_05497_amd as P
    return P


def _requests(P, count=8, seed=31):
    """Frames of a small 3D scanner on two image grids, uneven sizes."""
    sc = lmsynth.Scanner(96, 16, 120.0, 4.0)
    tof = lmsynth.TOF(9, 24.0, 60.0, 3.0, True)
    grids = [lmsynth.ImageGeom((48, 48, 16), (3.5, 3.5, 4.0)), lmsynth.ImageGeom((32, 32, 16), (5.0, 5.0, 4.0))]
    geoms = []
    rng = np.random.default_rng(seed)
    reqs = []
    for grid in grids:
        geoms.append(P.Geometry.from_problem(lmsynth.Problem("srv", sc, grid, tof, 8, 1, 0.03)))
    for r in range(count):
        gi = r % 2
        n = int(10 ** rng.uniform(4, 5.3))
        p = lmsynth.simulate_3d(lmsynth.Problem("srv", sc, grids[gi], tof, 8, 1, 0.03), n_prompts=n,
                                seed=seed * 100 + r, workers=1)
        reqs.append(P_serving().Request(geoms[gi], p.events, p.s, p.x0, n_subsets=8, epochs=1 + r % 2,
                                        beta=0.03, seq_seed=1000 + r, name=f"r{r}"))
    return reqs, geoms


def P_serving():
    from paper_2201_05497_amd import serving
    return serving


def test_served_equals_alone(P):
    S = P_serving()
    reqs, geoms = _requests(P)
    alone = [S.solve(r) for r in reqs]
    with S.Server(hbm_budget=8 << 30, max_active=4) as srv:
        for g in geoms:
            srv.warm(g)
        futs = [srv.submit(r) for r in reqs]
        res = [f.result(timeout=120) for f in futs]
    worst = 0.0
    for r, a, b in zip(reqs, res, alone):
        e = img_err(a.x, b.astype(np.float64))
        worst = max(worst, e)
        assert a.name == r.name
    st = S.latency_stats(res)
    report("served vs alone", requests=len(reqs), worst=worst, p50=st["p50_s"], p99=st["p99_s"])
    assert worst <= 1e-4


def test_admission_budget_and_errors(P):
    S = P_serving()
    reqs, geoms = _requests(P, count=6, seed=32)
    need = max(S.footprint(r) for r in reqs)
    budget = 2 * need + sum(4 * g.nvox for g in geoms)
    srv = S.Server(hbm_budget=budget, max_active=8)
    for g in geoms:
        srv.warm(g)
    futs = [srv.submit(r) for r in reqs]
    # a request larger than the whole budget fails without blocking the rest
    big = reqs[0]
    big_req = S.Request(big.geom, np.tile(big.events, (40, 1)), np.tile(big.s, 40), big.x0, n_subsets=8,
                        epochs=1, name="big")
    fbig = srv.submit(big_req)
    # a waiting request can be cancelled
    extra = srv.submit(reqs[1])
    cancelled = extra.cancel()
    srv.close()
    for f in futs:
        assert f.result().x.shape == reqs[0].x0.shape or f.result().x.ndim == 3
    with pytest.raises(MemoryError):
        fbig.result()
    report("admission", budget=budget, peak=srv.peak_bytes, cancelled=int(cancelled))
    assert srv.peak_bytes <= budget
    assert len(srv.results) == len(reqs) + (0 if cancelled else 1)


def test_failed_preparation_fails_alone(P):
    """A request whose plan cannot be built (an event index out of range)
    fails with the library's error; the others complete and the budget is
    released."""
    S = P_serving()
    reqs, geoms = _requests(P, count=3, seed=33)
    bad_ev = reqs[0].events.copy()
    bad_ev[5, 0] = 30000
    bad = S.Request(reqs[0].geom, bad_ev, reqs[0].s, reqs[0].x0, n_subsets=8, epochs=1, name="bad")
    with S.Server(hbm_budget=8 << 30, max_active=2) as srv:
        for g in geoms:
            srv.warm(g)
        fb = srv.submit(bad)
        futs = [srv.submit(r) for r in reqs]
        res = [f.result(timeout=120) for f in futs]
        with pytest.raises(P.LMError):
            fb.result(timeout=120)
    assert [r.name for r in res] == [r.name for r in reqs]
    assert srv._used == 0


def test_running_request_can_be_cancelled(P):
    """A request cancelled while its epochs run stops, raises CancelledError
    and frees its slot and memory; a request admitted beside it, and one
    that needs the freed slot, complete and equal their plain-solver runs."""
    S = P_serving()
    reqs, geoms = _requests(P, count=3, seed=34)
    r0 = reqs[0]
    long_req = S.Request(r0.geom, r0.events, r0.s, r0.x0, n_subsets=8, epochs=2000, seq_seed=7, name="long")
    with S.Server(hbm_budget=8 << 30, max_active=2) as srv:
        for g in geoms:
            srv.warm(g)
        f_long = srv.submit(long_req)
        f1 = srv.submit(reqs[1])
        f2 = srv.submit(reqs[2])  # waits for a slot
        t0 = time.perf_counter()
        while not f_long.running() and time.perf_counter() - t0 < 60:
            time.sleep(0.01)
        time.sleep(0.2)  # let it prepare and queue epochs
        assert f_long.running() and not f_long.done()
        assert srv.cancel(f_long)
        with pytest.raises(CancelledError):
            f_long.result(timeout=120)
        res = [f1.result(timeout=120), f2.result(timeout=120)]
        assert not srv.cancel(f1)  # finished: nothing to cancel
    assert srv._used == 0
    assert sorted(r.name for r in srv.results) == sorted(r.name for r in reqs[1:])
    worst = max(img_err(a.x, S.solve(r).astype(np.float64)) for a, r in zip(res, reqs[1:]))
    report("cancel running", worst=worst, elapsed=time.perf_counter() - t0)
    assert worst <= 1e-4
