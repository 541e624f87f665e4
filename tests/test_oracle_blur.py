"""Pins of the oracle's image-space resolution model B (Section 1: the
forward model includes limited spatial resolution; P = G B): B is
symmetric, keeps mass, centre and linear ramps away from the edges, has the
variance of its Gaussian, and LM-SPDHG with P' = diag(m) G B equals sinogram
SPDHG (Algorithm 1) on the dense matrix diag(m) G B."""
import numpy as np
import pytest

import lmsynth
from tests.test_oracle_algorithm import _sino_setup, tiny_problem


@pytest.mark.parametrize("shape,fwhm", [((5, 7, 9), (1.5, 2.0, 1.2)), ((1, 8, 8), (2.5, 0.0, 0.0)),
                                        ((6, 3, 4), (0.0, 1.0, 3.0))])
def test_blur_symmetric(orc, shape, fwhm):
    rng = np.random.default_rng(sum(shape))
    for _ in range(4):
        x, y = rng.normal(size=shape), rng.normal(size=shape)
        lhs, rhs = float((orc.blur(x, fwhm) * y).sum()), float((x * orc.blur(y, fwhm)).sum())
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_blur_moments_and_ramps(orc):
    """A point in the middle of a long line keeps mass 1 and its centre, and
    spreads with the variance of the Gaussian (to the truncation at 3
    sigma); a linear ramp is unchanged away from the edges."""
    for fw in (2.355, 4.0, 6.0):  # sigma >= 1 voxel: the sampled Gaussian resolves its variance
        sig = fw / (2 * np.sqrt(2 * np.log(2)))
        x = np.zeros((1, 1, 81))
        x[0, 0, 40] = 1.0
        b = orc.blur(x, (fw, 0, 0))[0, 0]
        t = np.arange(81) - 40
        assert abs(b.sum() - 1) < 1e-14 and abs((t * b).sum()) < 1e-14
        var = float((t * t * b).sum())
        assert abs(var - sig * sig) <= 0.04 * sig * sig, (fw, var, sig * sig)
        # full width at half maximum of the sampled response, for the wider ones
        if fw >= 4.0:
            half = b.max() / 2
            above = np.nonzero(b >= half)[0]
            assert abs((above[-1] - above[0]) - fw) <= 1.0
    ramp = np.broadcast_to(np.arange(30.0), (3, 4, 30)).copy()
    b = orc.blur(ramp, (2.0, 0, 0))
    np.testing.assert_allclose(b[:, :, 6:-6], ramp[:, :, 6:-6], atol=1e-12)


def test_lm_with_blur_equals_sinogram(orc):
    p, ev, s, x0 = tiny_problem(dup=False, n_events=300)
    G = orc.Geometry.from_problem(p)
    bins, boe, d = _sino_setup(orc, p, ev)
    fwhm = (1.8, 1.3, 0.0)
    nv = int(np.prod(G.shape))
    Bmat = np.stack([orc.blur(np.eye(nv)[j].reshape(G.shape), fwhm).reshape(-1) for j in range(nv)], axis=1)
    m_bin = np.random.default_rng(3).uniform(0.4, 1.1, len(bins))
    Pm = m_bin[:, None] * (orc.dense_matrix(G, bins) @ Bmat)
    g = Pm.sum(axis=0).reshape(G.shape)
    n = 5
    sub = orc.subset_ids(len(ev), n)
    empty = np.nonzero(d == 0)[0]
    bos = [np.concatenate([boe[sub == i], empty if i == 0 else np.zeros(0, int)]) for i in range(n)]
    gamma, rho, beta = 3 / x0.max(), 0.999, 0.05
    seq = lmsynth.subset_sequence(5, 0, 80, n)
    x_lm, st, su = orc.lm_spdhg(G, ev, s, g, x0, n, seq, gamma, rho, beta, m=m_bin[boe], fwhm=fwhm)
    x_sino = orc.spdhg_sino(Pm, d, np.full(len(bins), 0.05), x0, bos, seq, gamma, rho, beta, G.shape, T=su.T,
                            p1_min=orc.p1_floor(G))
    np.testing.assert_allclose(x_lm, x_sino, rtol=0, atol=1e-12 * np.abs(x_sino).max())
    # the blur matters
    x_sharp, _, _ = orc.lm_spdhg(G, ev, s, g, x0, n, seq, gamma, rho, beta, m=m_bin[boe])
    assert np.abs(x_sharp - x_lm).max() > 1e-3 * np.abs(x_lm).max()
