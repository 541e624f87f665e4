"""Pins of the oracle's per-event multiplicative factors (attenuation times
normalisation of each event's LOR; the forward model is P' = diag(m) P):
LM-SPDHG with the factors of its events equals sinogram SPDHG (Algorithm 1)
on the dense matrix whose rows are scaled by the factor of their bin, with
duplicates in one subset and with unit counts in several subsets."""
import numpy as np

import lmsynth
from tests.test_oracle_algorithm import _sino_setup, tiny_problem


def _scaled(orc, p, ev, seed):
    G = orc.Geometry.from_problem(p)
    bins, boe, d = _sino_setup(orc, p, ev)
    P = orc.dense_matrix(G, bins)
    m_bin = np.random.default_rng(seed).uniform(0.3, 1.2, len(bins))
    Pm = m_bin[:, None] * P
    g = Pm.sum(axis=0).reshape(G.shape)  # the sensitivity of P'
    return G, bins, boe, d, Pm, m_bin, g


def test_factors_one_subset_with_duplicates(orc):
    p, ev, s, x0 = tiny_problem(dup=True)
    G, bins, boe, d, Pm, m_bin, g = _scaled(orc, p, ev, 1)
    assert d.max() >= 3
    gamma, rho, beta = 3 / x0.max(), 0.999, 0.05
    seq = lmsynth.subset_sequence(3, 0, 40, 1)
    x_lm, _, _ = orc.lm_spdhg(G, ev, s, g, x0, 1, seq, gamma, rho, beta, m=m_bin[boe])
    x_sino = orc.spdhg_sino(Pm, d, np.full(len(bins), 0.05), x0, [np.arange(len(bins))], seq, gamma, rho, beta,
                            G.shape, p1_min=orc.p1_floor(G))
    np.testing.assert_allclose(x_lm, x_sino, rtol=0, atol=1e-12 * np.abs(x_sino).max())
    # the factors matter: without them the iterates differ
    x_plain, _, _ = orc.lm_spdhg(G, ev, s, g, x0, 1, seq, gamma, rho, beta)
    assert np.abs(x_plain - x_lm).max() > 1e-3 * np.abs(x_lm).max()


def test_factors_subsets_unit_counts(orc):
    p, ev, s, x0 = tiny_problem(dup=False, n_events=300)
    G, bins, boe, d, Pm, m_bin, g = _scaled(orc, p, ev, 2)
    assert d.max() == 1
    n = 5
    sub = orc.subset_ids(len(ev), n)
    empty = np.nonzero(d == 0)[0]
    bos = [np.concatenate([boe[sub == i], empty if i == 0 else np.zeros(0, int)]) for i in range(n)]
    gamma, rho, beta = 3 / x0.max(), 0.999, 0.05
    seq = lmsynth.subset_sequence(4, 0, 80, n)
    x_lm, st, su = orc.lm_spdhg(G, ev, s, g, x0, n, seq, gamma, rho, beta, m=m_bin[boe])
    x_sino = orc.spdhg_sino(Pm, d, np.full(len(bins), 0.05), x0, bos, seq, gamma, rho, beta, G.shape, T=su.T,
                            p1_min=orc.p1_floor(G))
    np.testing.assert_allclose(x_lm, x_sino, rtol=0, atol=1e-12 * np.abs(x_sino).max())
