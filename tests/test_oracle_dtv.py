"""Pins of the oracle's directional TV prior (Section 3, DTV): K = D grad
with D_j = I - xi_j xi_j^T and xi the normalised gradient of a structural
prior image.  Adjointness and the norm bound that keeps the TV step sizes
valid, the removed direction, the reductions to TV, and LM-SPDHG with DTV
equal to sinogram SPDHG (Algorithm 1) with DTV on tiny binned data."""
import numpy as np
import pytest

import lmsynth
from tests.test_oracle_algorithm import _sino_setup, tiny_problem


@pytest.mark.parametrize("shape", [(4, 5, 6), (1, 7, 9), (3, 1, 8)])
def test_dtv_adjoint_and_norm_bound(orc, shape):
    rng = np.random.default_rng(sum(shape))
    xi = orc.dtv_field(rng.uniform(0, 1, shape), 0.05)
    assert np.sqrt((xi ** 2).sum(axis=0)).max() < 1.0
    for _ in range(5):
        x = rng.normal(size=shape)
        w = rng.normal(size=(3,) + shape)
        lhs = float((orc.k_op(x, xi) * w).sum())
        rhs = float((x * orc.k_adj(w, xi)).sum())
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    # power iteration: ||D grad||^2 <= ||grad||^2, the bound the step sizes use
    x = rng.normal(size=shape)
    for _ in range(300):
        x = orc.k_adj(orc.k_op(x, xi), xi)
        lam = np.linalg.norm(x)
        x /= lam
    assert lam <= orc.grad_norm(shape) ** 2 * (1 + 1e-9)


def test_dtv_removes_the_prior_direction(orc):
    """xi . (K x)_j = (1 - |xi_j|^2) xi . (grad x)_j; a constant prior image
    gives TV; an image is nearly flat under DTV with its own flipped
    contrast as prior (the paper's perfect structural information)."""
    rng = np.random.default_rng(3)
    shape = (5, 8, 9)
    x = rng.uniform(0, 1, shape)
    xi = orc.dtv_field(rng.uniform(0, 1, shape), 0.1)
    kx, gx = orc.k_op(x, xi), orc.grad(x)
    n2 = (xi ** 2).sum(axis=0)
    np.testing.assert_allclose((xi * kx).sum(axis=0), (1 - n2) * (xi * gx).sum(axis=0), atol=1e-13)
    assert np.array_equal(orc.k_op(x, orc.dtv_field(np.full(shape, 2.0), 0.1)), gx)
    # piecewise-constant image: steps of at least 1, eta 1e-3
    pc = np.floor(3 * rng.uniform(0, 1, shape))
    tv = orc.tv(pc)
    dtv = float(np.sqrt((orc.k_op(pc, orc.dtv_field(4.0 - pc, 1e-3)) ** 2).sum(axis=0)).sum())
    assert tv > 10 and dtv <= 1e-6 * tv


def test_lm_equals_sinogram_dtv(orc):
    """Algorithm 2 with the DTV prior equals Algorithm 1 with the same prior
    (unit counts, 5 subsets): the prior's operator enters both the same way."""
    p, ev, s, x0 = tiny_problem(dup=False, n_events=300)
    G = orc.Geometry.from_problem(p)
    bins, boe, d = _sino_setup(orc, p, ev)
    n = 5
    sub = orc.subset_ids(len(ev), n)
    empty = np.nonzero(d == 0)[0]
    bos = [np.concatenate([boe[sub == i], empty if i == 0 else np.zeros(0, int)]) for i in range(n)]
    P = orc.dense_matrix(G, bins)
    g = orc.sens(G)
    xi = orc.dtv_field(np.random.default_rng(5).uniform(0, 2, G.shape), 0.2)
    gamma, rho, beta = 3 / x0.max(), 0.999, 0.05
    seq = lmsynth.subset_sequence(6, 0, 80, n)
    x_lm, st, su = orc.lm_spdhg(G, ev, s, g, x0, n, seq, gamma, rho, beta, xi=xi)
    sb = np.full(len(bins), 0.05)
    x_sino = orc.spdhg_sino(P, d, sb, x0, bos, seq, gamma, rho, beta, G.shape, T=su.T, xi=xi, p1_min=orc.p1_floor(G))
    np.testing.assert_allclose(x_lm, x_sino, rtol=0, atol=1e-12 * np.abs(x_sino).max())
    # and DTV changes the iterates (the prior is not silently TV)
    x_tv, _, _ = orc.lm_spdhg(G, ev, s, g, x0, n, seq, gamma, rho, beta)
    assert np.abs(x_tv - x_lm).max() > 1e-6 * np.abs(x_lm).max()


def test_dtv_z_invariant(orc):
    """z = g + P^LM^T((y-1)/mu) + K^T w holds after every update with the
    DTV operator (the prior branch adds K^T of the change of w)."""
    p, ev, s, x0 = tiny_problem(dup=True)
    G = orc.Geometry.from_problem(p)
    g = orc.sens(G)
    xi = orc.dtv_field(np.random.default_rng(8).uniform(0, 2, G.shape), 0.2)
    mu = orc.event_counts(ev, p.scanner.n_cry)

    def check(st, su):
        z = su.g + orc.back(G, (st.y - 1.0) / mu, ev) + orc.k_adj(st.w, xi)
        assert np.abs(st.z - z).max() <= 1e-10 * np.abs(z).max()
        assert np.sqrt((st.w ** 2).sum(axis=0)).max() <= 0.05 * (1 + 1e-12)

    orc.lm_spdhg(G, ev, s, g, x0, 3, lmsynth.subset_sequence(9, 0, 30, 3), 3 / x0.max(), 0.999, 0.05,
                 callback=check, xi=xi)
