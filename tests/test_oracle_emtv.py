"""Pins of the oracle's listmode EM-TV warm start (Algorithm 3) against the
mathematics: the EM step's count identity, the monotone likelihood and the
optimality conditions of MLEM, and the weighted TV denoising against convex
duality (a vanishing primal-dual gap), a closed-form two-voxel solution and
its fixed points."""
import numpy as np

import lmsynth


def _tiny(orc, n_events=400, seed=0, tof=True):
    p = lmsynth.tiny_2d(n_det=16, nxy=8, tof_on=tof)
    G = orc.Geometry.from_problem(p)
    ev = lmsynth.random_events(p, n_events, seed=seed, min_sep=3)
    g = orc.sens(G)
    return p, G, ev, g


def test_em_step_count_identity(orc):
    """sum_j g_j z_j = n sum_{e in subset} (Px)_e / ((Px)_e + s_e): the EM
    step redistributes the subset's (scaled) events over the image."""
    p, G, ev, g = _tiny(orc)
    rng = np.random.default_rng(1)
    x = rng.uniform(0.2, 2.0, G.shape)
    for n, s in ((1, np.zeros(len(ev))), (4, rng.uniform(0.01, 0.5, len(ev))), (7, rng.uniform(0, 2, len(ev)))):
        sub = orc.subset_ids(len(ev), n)
        for i in range(n):
            m = sub == i
            z = orc.em_step(G, x, ev[m], s[m], g, n)
            q = orc.fwd(G, x, ev[m])
            hit = q + s[m] > 0
            want = n * float((q[hit] / (q[hit] + s[m][hit])).sum())
            assert abs(float((g * z).sum()) - want) <= 1e-10 * max(want, 1.0)
            assert np.all(z >= 0) and np.all(z[x == 0] == 0)


def _loglik(orc, G, ev, s, g, x):
    """Listmode Poisson log-likelihood: sum_e log((Px)_e + s_e) - <g, x>."""
    return float(np.log(orc.fwd(G, x, ev) + s).sum() - (g * x).sum())


def test_mlem_monotone_and_kkt(orc):
    """beta = 0 and one subset make Algorithm 3 MLEM: the log-likelihood
    never decreases, and the iterates approach its optimality conditions
    (P^T 1/(Px+s) = g where x > 0)."""
    p, G, ev, g = _tiny(orc, n_events=600, seed=2)
    s = np.random.default_rng(3).uniform(0.05, 0.2, len(ev))
    x = np.ones(G.shape)
    ll = [_loglik(orc, G, ev, s, g, x)]
    for _ in range(60):
        x = orc.emtv(G, ev, s, g, x, n_subsets=1, n_iter=1, beta=0.0)
        ll.append(_loglik(orc, G, ev, s, g, x))
    assert np.all(np.diff(ll) >= -1e-9 * np.abs(ll[1:]))
    assert ll[-1] > ll[0]

    def kkt(x):
        r = orc.back(G, 1.0 / (orc.fwd(G, x, ev) + s), ev) / np.where(g > 0, g, 1.0) - 1.0
        return float(np.abs(r[(x > 1e-3 * x.max()) & (g > 0)]).max())

    k60 = kkt(x)
    for _ in range(400):
        x = orc.emtv(G, ev, s, g, x, n_subsets=1, n_iter=1, beta=0.0)
    assert kkt(x) < 0.5 * k60 and kkt(x) < 0.05


def _gap(orc, z, w, u, q):
    """Primal-dual gap of min_{u>=0} sum w/2 (u-z)^2 + ||Ku||_{2,1} at (u, q),
    |q_j| <= 1: primal value plus G*(-K^T q), where G*(v) = sum_j sup_{u>=0}
    (v u - w/2 (u - z)^2) = v z + v^2/(2w) if z + v/w >= 0, else -w z^2/2;
    for w = inf (u held at z) it is v z."""
    fixed = np.isinf(w)
    wf = np.where(fixed, 1.0, w)
    primal = float((np.where(fixed, 0.0, w) / 2 * (u - z) ** 2).sum() + orc.tv(u))
    assert np.all(u >= 0) and np.allclose(u[fixed], z[fixed])
    v = -orc.grad_adjoint(q)
    conj = np.where(z + v / wf >= 0, v * z + v * v / (2 * wf), -wf * z * z / 2)
    conj = np.where(fixed, v * z, conj)
    assert np.sqrt((q ** 2).sum(axis=0)).max() <= 1 + 1e-12
    return primal + float(conj.sum()), primal


def test_denoise_duality_gap(orc):
    """Many accelerated PDHG steps close the primal-dual gap of the weighted
    TV denoising problem (3D, ragged sizes, a few voxels held by infinite
    weights, weights spanning three decades)."""
    rng = np.random.default_rng(4)
    for shape in ((5, 6, 7), (1, 9, 8), (3, 1, 11)):
        z = rng.uniform(0, 3, shape) * (rng.random(shape) < 0.8)
        w = 10 ** rng.uniform(-1, 2, shape)
        w[rng.random(shape) < 0.1] = np.inf
        u, q = orc.weighted_tv_denoise(z, w, 4000, return_dual=True)
        gap, primal = _gap(orc, z, w, u, q)
        assert -1e-9 <= gap <= 1e-6 * max(primal, 1.0), (shape, gap, primal)
        # 20 steps, as the warm start takes them, already close most of it
        u0 = z.copy()
        g20, _ = _gap(orc, z, w, *orc.weighted_tv_denoise(z, w, 20, return_dual=True))
        g0, _ = _gap(orc, z, w, u0, np.zeros((3,) + shape))
        assert g20 < 0.2 * g0


def test_denoise_two_voxels_closed_form(orc):
    """Two voxels along x: min w0/2 (u0-z0)^2 + w1/2 (u1-z1)^2 + |u1 - u0|
    fuses them at the weighted mean when |z1 - z0| <= 1/w0 + 1/w1, else
    moves each by 1/w towards the other.  The iterate approaches the
    minimiser at rate O(1/N) (O(1/N^2) in squared distance)."""
    for z0, z1, w0, w1 in ((1.0, 1.2, 2.0, 3.0), (1.0, 3.0, 2.0, 4.0), (5.0, 1.0, 1.0, 0.5), (2.0, 2.0, 1.0, 1.0)):
        z = np.array([[[z0, z1]]])
        w = np.array([[[w0, w1]]])
        u = orc.weighted_tv_denoise(z, w, 20000)
        d = z1 - z0
        if abs(d) <= 1 / w0 + 1 / w1:
            want = np.full(2, (w0 * z0 + w1 * z1) / (w0 + w1))
        else:
            want = np.array([z0 + np.sign(d) / w0, z1 - np.sign(d) / w1])
        assert np.allclose(u.reshape(-1), want, atol=5e-4), (z0, z1, w0, w1, u)


def test_denoise_fixed_points(orc):
    """A constant image is its own denoised image (K z = 0; to rounding of the
    prox quotient); infinite weights
    hold their voxels; a zero image stays zero."""
    rng = np.random.default_rng(5)
    w = 10 ** rng.uniform(-1, 1, (4, 5, 6))
    z = np.full((4, 5, 6), 1.7)
    assert np.allclose(orc.weighted_tv_denoise(z, w, 20), z, rtol=1e-14, atol=0)
    w2 = w.copy()
    w2[1, 2, 3] = np.inf
    z2 = rng.uniform(0, 2, (4, 5, 6))
    assert orc.weighted_tv_denoise(z2, w2, 20)[1, 2, 3] == z2[1, 2, 3]
    assert np.array_equal(orc.weighted_tv_denoise(np.zeros((4, 5, 6)), w, 20), np.zeros((4, 5, 6)))


def test_emtv_small_beta_is_osem(orc):
    """w = g / (beta x) grows without bound as beta -> 0: EM-TV becomes OSEM
    (beta = 0); a large beta flattens the image (its TV drops)."""
    p, G, ev, g = _tiny(orc, n_events=500, seed=6)
    s = np.full(len(ev), 0.1)
    x0 = np.ones(G.shape)
    osem = orc.emtv(G, ev, s, g, x0, n_subsets=4, n_iter=2, beta=0.0)
    small = orc.emtv(G, ev, s, g, x0, n_subsets=4, n_iter=2, beta=1e-9)
    assert np.abs(small - osem).max() <= 1e-6 * osem.max()
    big = orc.emtv(G, ev, s, g, x0, n_subsets=4, n_iter=2, beta=10.0)
    assert orc.tv(big) < 0.5 * orc.tv(osem)


def test_emtv_fixed_point_minimises_eq1(orc):
    """With one subset and a denoising solved to high accuracy, Algorithm 3
    converges to the minimiser of the penalised listmode objective (Eq. 1),
    the problem LM-SPDHG solves: both end at the same image and cost.  The
    weights w = g / (beta x) taken at the image before the EM step are what
    makes that fixed point the minimiser (weights taken at the EM image
    leave the image 3 % away)."""
    p = lmsynth.tiny_2d(n_det=16, nxy=8)
    G = orc.Geometry.from_problem(p)
    ev = lmsynth.random_events(p, 600, seed=7, min_sep=3)
    g = orc.sens(G)
    s = np.full(len(ev), 0.05)
    beta, x0 = 0.5, np.ones(G.shape)
    x = x0
    for _ in range(300):
        x = orc.emtv(G, ev, s, g, x, n_subsets=1, n_iter=1, beta=beta, denoise_iter=200)
    xs, _, _ = orc.lm_spdhg(G, ev, s, g, x0, 1, lmsynth.subset_sequence(3, 0, 12000, 1), 3.0, 0.999, beta)
    c_em, c_pd = orc.cost(G, x, ev, s, g, beta), orc.cost(G, xs, ev, s, g, beta)
    assert abs(c_em - c_pd) <= 2e-6 * abs(c_pd)
    assert np.abs(x - xs).max() <= 0.01 * xs.max()
