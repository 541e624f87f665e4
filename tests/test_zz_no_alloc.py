"""lm_fwd_noalloc (the forward projector for callers that cannot allocate)
against lm_fwd, both through the C ABI: two calls in a row on the same
device, the second with a smaller image and fewer events, each compared
with lm_fwd on the same inputs (the kernels are the same, so the values
agree to the projection tolerance; in practice bit for bit).  Also the
size limit of the scratch array."""
import ctypes

import numpy as np
import pytest
import torch

import lmsynth
from tests.helpers import proj_err, report, smooth_image

pytestmark = pytest.mark.gpu

PROJ_TOL = 1e-5


def _call(fn, G, x, ev, out):
    from paper_2201_05497_amd import _lib
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fn(ctypes.byref(G._c), x.data_ptr(), ev.data_ptr(), ev.shape[0], out.data_ptr(), stream)
    _lib.check(rc, fn.__name__)


def test_noalloc_matches_lm_fwd_on_two_calls():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2201_05497_amd as P
    from paper_2201_05497_amd import _lib
    L = _lib.load()
    cases = [(lmsynth.config_3d_large(), 300_000, 31), (lmsynth.config_3d(), 40_000, 32)]
    for k, (cfg, n, seed) in enumerate(cases):
        G = P.Geometry.from_problem(cfg)
        ev = G.events(lmsynth.random_events(cfg, n, seed=seed))
        x = torch.as_tensor(smooth_image(G.shape, seed), device="cuda")
        want = torch.empty(n, device="cuda")
        got = torch.full((n,), float("nan"), device="cuda")
        _call(L.lm_fwd, G, x, ev, want)
        _call(L.lm_fwd_noalloc, G, x, ev, got)
        torch.cuda.synchronize()
        w, g = want.cpu().numpy(), got.cpu().numpy()
        emax, _ = proj_err(g, w)
        report(f"lm_fwd_noalloc call {k + 1} ({G.shape}, {n} events)", err=emax,
               identical=int(np.array_equal(w, g)))
        assert np.isfinite(g).all()
        assert emax <= PROJ_TOL


def test_noalloc_rejects_images_beyond_the_scratch():
    import paper_2201_05497_amd as P
    from paper_2201_05497_amd import _lib
    L = _lib.load()
    cfg = lmsynth.config_3d()
    G = P.Geometry(cfg.det, cfg.scanner.n_cry, cfg.scanner.n_ring, (512, 512, 72), (1.0, 1.0, 3.4),
                   cfg.tof.n_tof, cfg.tof.bin, cfg.tof.fwhm)
    ev = G.events(lmsynth.random_events(cfg, 10, seed=1))
    x = torch.zeros(G.shape, device="cuda")
    out = torch.zeros(10, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.lm_fwd_noalloc(ctypes.byref(G._c), x.data_ptr(), ev.data_ptr(), 10, out.data_ptr(), stream)
    assert rc == _lib.LM_EINVAL
    assert b"scratch" in L.lm_last_error()
