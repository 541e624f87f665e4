"""lm_cost (the listmode objective of Eq. (1), for relative-cost monitoring)
against the oracle's cost, through the C ABI: on the 2D workload at the
starting image and at the oracle's own iterate after two LM-SPDHG epochs,
and on a ragged 3D grid at a smooth random image.  Each of the three terms
is compared: <g, x> and ||K x||_{2,1} to 1e-6 relative (sums of float32
inputs accumulated in double), and the sum of log((P^LM x)_e + s_e) to the
bound the per-event projection tolerance gives, 1e-5 per event."""
import numpy as np
import pytest
import torch

import lmsynth
import oracle
from tests.helpers import problem_2d, report, smooth_image

pytestmark = pytest.mark.gpu

PROJ_TOL = 1e-5


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2201_05497_amd as P
    return P


def _terms_orc(Go, x, ev, s, g):
    q = oracle.fwd(Go, x, ev) + s
    return (float((g * x).sum()), float(np.log(q).sum()), oracle.tv(x))


def _check(P, name, p, x, ev, s, g, beta):
    Go = oracle.Geometry.from_problem(p)
    G = P.Geometry.from_problem(p)
    x32, g32, s32 = (np.asarray(a, np.float32) for a in (x, g, s))
    cuda = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    c, t = P.lm_cost(G, cuda(x32), G.events(ev), cuda(s32), cuda(g32), beta)
    to = _terms_orc(Go, x32.astype(np.float64), ev, s32.astype(np.float64), g32.astype(np.float64))
    co = oracle.cost(Go, x32.astype(np.float64), ev, s32.astype(np.float64), g32.astype(np.float64), beta)
    e_gx = abs(t[0] - to[0]) / abs(to[0])
    e_log = abs(t[1] - to[1])
    e_tv = abs(t[2] - to[2]) / max(abs(to[2]), 1e-30)
    e_c = abs(c - co)
    report(f"lm_cost {name}", gx_rel=e_gx, log_abs=e_log, log_abs_per_event=e_log / max(len(ev), 1), tv_rel=e_tv,
           cost_abs=e_c, cost=c)
    assert e_gx <= 1e-6 and e_tv <= 1e-6
    assert e_log <= PROJ_TOL * len(ev)
    assert e_c <= PROJ_TOL * len(ev) + 1e-6 * (abs(to[0]) + beta * abs(to[2]))
    assert np.isclose(c, t[0] - t[1] + beta * t[2], rtol=0, atol=1e-9 * abs(c))


def test_cost_2d(P):
    p = problem_2d()
    Go = oracle.Geometry.from_problem(p)
    g = oracle.sens(Go)
    beta, n = 0.03, 28
    _check(P, "2d x0", p, p.x0, p.events, p.s, g, beta)
    gamma = float(np.float32(3.0 / float(p.x0.max())))
    seq = lmsynth.subset_sequence(2000, 0, 4 * n, n)
    x_o, _, _ = oracle.lm_spdhg(Go, p.events, p.s.astype(np.float64), g.astype(np.float32).astype(np.float64),
                                p.x0, n, seq, gamma, 0.999, beta)
    _check(P, "2d after 2 epochs", p, x_o, p.events, p.s, g, beta)
    _check(P, "2d beta 0", p, x_o, p.events, p.s, g, 0.0)


def test_cost_3d_ragged(P):
    sc = lmsynth.Scanner(96, 16, 120.0, 4.0)
    tof = lmsynth.TOF(9, 24.0, 60.0, 3.0, True)
    img = lmsynth.ImageGeom((37, 29, 11), (3.0, 2.5, 3.5))
    p = lmsynth.simulate_3d(lmsynth.Problem("ragged", sc, img, tof, 4, 1, 0.03), n_prompts=20000, seed=81,
                            workers=1)
    rng = np.random.default_rng(82)
    g = 5.0 + rng.uniform(0.0, 1.0, img.shape_zyx)
    _check(P, "3d ragged", p, smooth_image(img.shape_zyx, 83), p.events, p.s, g, 0.05)
    # no events: only the image terms
    _check(P, "3d no events", p, smooth_image(img.shape_zyx, 84), p.events[:0], p.s[:0], g, 0.05)
