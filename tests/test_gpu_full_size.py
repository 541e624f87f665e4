"""Full-size GPU parity against expected values the FP64 oracle computed
once (``tests/golden/full_size.py``; the oracle needs minutes to half an
hour of one core per case, too long for a test):

* the 3D reconstruction exactly as the benchmark runs it (1e7 prompts,
  224 subsets, 5 epochs of Algorithm 2 with the benchmark's subset
  sequence): x after every epoch, z and zbar at the end in sup norm, the
  dual complement c on every 32nd event, the TV dual w on three slices;
* three data and three prior updates at the shape of the long static frame
  (300x300x96 image, 2.2e6 events per data update) from a seeded state;
* the sensitivity image P^T 1 over every crystal pair of the full
  672-crystal ring (3 rings, TOF on), the path lm_sens takes on that
  scanner (by transaxial line plus the per-LOR kernel for z-dominant
  pairs).

Tolerances: iterates and back projections ||gpu - orc||_inf <= 1e-4
||orc||_inf; the TV dual w in relative L2 <= 1e-4 and in sup norm <= ten
times the oracle's own sensitivity of w to float32 rounding on the
benchmarked case (``c2_sensitivity.json``: the oracle with its state
rounded to float32 after every update moves w by 2.7e-3 beta in sup norm,
x by 3.9e-6; the TV dual is ill-conditioned where K x is nearly zero, and
the GPU's float32 projections perturb the state more than rounding
alone)."""
import json
import os

import numpy as np
import pytest
import torch

from tests.golden import full_size as FS
from tests.helpers import img_err, report

pytestmark = pytest.mark.gpu

ITER_TOL = 1e-4
with open(os.path.join(os.path.dirname(FS.__file__), "c2_sensitivity.json")) as _f:
    W_SUP_TOL = 10.0 * json.load(_f)["w_inf_over_beta"]


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2201_05497_amd as P
    return P


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def _w_errs(wg, wo, beta):
    wg = np.asarray(wg, dtype=np.float64)
    wo = np.asarray(wo, dtype=np.float64)
    return (float(np.linalg.norm(wg - wo) / max(np.linalg.norm(wo), 1e-30)),
            float(np.abs(wg - wo).max() / beta))


def test_c2_benchmarked_reconstruction(P):
    """1e7 events, 224 subsets, TV beta 0.03, 5 epochs: x after every epoch."""
    gold = FS.load("c2")
    p, g = FS.c2_inputs()
    C = FS.C2
    G = P.Geometry.from_problem(p)
    print(f"[full size] c2: {len(p.events)} events, {C['n_sub']} subsets, {C['epochs']} epochs", flush=True)
    plan = P.Plan(G, G.events(p.events), _cuda(p.s), C["n_sub"], FS.gamma_of(p.x0), C["rho"], C["beta"],
                  g=_cuda(g))
    x = _cuda(p.x0).clone()
    plan.init(x)
    errs = []
    for ep in range(C["epochs"]):
        plan.epoch(x, FS.c2_sequence(ep))
        e = img_err(x.cpu().numpy(), gold[f"x{ep + 1}"])
        errs.append(e)
        report(f"c2 full size epoch {ep + 1}", x_err=e)
    st = plan.get_state()
    ez = img_err(st["z"].cpu().numpy(), gold["z"])
    ezb = img_err(st["zbar"].cpu().numpy(), gold["zbar"])
    ec = img_err(st["c"].cpu().numpy()[::C["c_stride"]], gold["c"])
    ew2, ewinf = _w_errs(st["w"].cpu().numpy()[:, list(C["w_slices"])], gold["w"], C["beta"])
    report("c2 full size final", z_err=ez, zbar_err=ezb, c_err=ec, w_l2=ew2, w_inf_over_beta=ewinf, u=st["u"])
    plan.destroy()
    assert st["u"] == int(gold["u"])
    assert max(errs) <= ITER_TOL
    assert max(ez, ezb, ec) <= ITER_TOL
    assert ew2 <= ITER_TOL and ewinf <= W_SUP_TOL


def test_c3_shaped_updates(P):
    """300x300x96, 8.9e6 events in 4 subsets (2.2e6 per data update), three
    data and three prior updates in one call from a seeded state."""
    gold = FS.load("c3")
    p, g, s0 = FS.c3_inputs()
    C = FS.C3
    G = P.Geometry.from_problem(p)
    print(f"[full size] c3: {len(p.events)} events, {C['n_sub']} subsets, updates {C['seq']}", flush=True)
    plan = P.Plan(G, G.events(p.events), _cuda(p.s), C["n_sub"], FS.gamma_of(p.x0), C["rho"], C["beta"],
                  g=_cuda(g))
    plan.set_state({"z": _cuda(s0["z"]), "zbar": _cuda(s0["zbar"]), "w": _cuda(s0["w"]), "c": _cuda(s0["c"]),
                    "u": 0})
    x = _cuda(s0["x"])
    plan.epoch(x, np.asarray(C["seq"], dtype=np.int32))
    st = plan.get_state()
    sl = list(C["slices"])
    ex = img_err(x.cpu().numpy()[sl], gold["x"])
    ez = img_err(st["z"].cpu().numpy()[sl], gold["z"])
    ezb = img_err(st["zbar"].cpu().numpy()[sl], gold["zbar"])
    ec = img_err(st["c"].cpu().numpy()[::C["c_stride"]], gold["c"])
    ew2, ewinf = _w_errs(st["w"].cpu().numpy()[:, sl], gold["w"], C["beta"])
    report("c3 shaped updates", x_err=ex, z_err=ez, zbar_err=ezb, c_err=ec, w_l2=ew2, w_inf_over_beta=ewinf)
    plan.destroy()
    assert st["u"] == int(gold["u"])
    assert max(ex, ez, ezb, ec) <= ITER_TOL
    assert ew2 <= ITER_TOL and ewinf <= W_SUP_TOL


def test_sens_full_ring(P):
    """lm_sens over every crystal pair and TOF bin of the 672-crystal ring with
    3 rings (2.03e6 pairs), 200x200x5 grid."""
    gold = FS.load("sens")
    p = FS.sens_problem()
    G = P.Geometry.from_problem(p)
    print(f"[full size] lm_sens: {p.scanner.n_cry} x {p.scanner.n_ring} crystals, image {G.shape}", flush=True)
    g = P.lm_sens(G)
    e = img_err(g.cpu().numpy(), gold["g"])
    report("lm_sens 672x3 ring", err=e)
    assert e <= ITER_TOL
