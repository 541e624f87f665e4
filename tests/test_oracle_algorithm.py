"""Pins of the FP64 oracle's algorithm (LM-SPDHG, Algorithm 2) against the
mathematics: the prox's optimality condition and fixed point, the adjoint
and norm of K, the projection onto the beta-ball, the z invariant, equality
with sinogram SPDHG (Algorithm 1) on tiny binned data, event counts by brute
force and the subset sequence's published first value."""
import itertools

import numpy as np
import pytest
from scipy import optimize

import lmsynth


# ------------------------------------------------------------------ P7: prox


def test_prox_first_order_and_brute_force(orc):
    rng = np.random.default_rng(10)
    for _ in range(200):
        a = rng.uniform(-3, 3)
        S = 10 ** rng.uniform(-3, 2)
        mu = int(rng.integers(1, 5))
        v = float(orc.prox_poisson_dual(np.array(a), np.array(S), np.array(mu)))
        assert v < 1.0
        # optimality: (v - a)/S + d/dv D*(v) = 0, with D*(v) = -mu + mu log(mu/(1-v))
        assert abs((v - a) / S + mu / (1.0 - v)) < 1e-8 * (1 + abs(a) / S + mu / (1 - v))
        # brute-force minimisation of 1/(2S)(v-a)^2 + D*(v) over v < 1
        f = lambda u: 0.5 / S * (u - a) ** 2 + float(orc.poisson_dual_conj(np.array(u), np.array(mu)))
        r = optimize.minimize_scalar(f, bounds=(min(a, v) - 50.0, 1.0 - 1e-15), method="bounded",
                                     options={"xatol": 1e-12})
        assert abs(r.x - v) < 1e-5 * max(1.0, abs(v))


def test_prox_zero_count_bins():
    """With d = 0 the prox is min(a, 1) (Section 2, memory-efficient SPDHG)."""
    import oracle
    a = np.linspace(-2, 3, 41)
    np.testing.assert_allclose(oracle.prox_poisson_dual(a, 0.7, 0.0), np.minimum(a, 1.0), atol=1e-15)


def test_dual_fixed_point(orc):
    """y = 1 - mu/q (Eq. yinit) is a fixed point of the data update when x is
    unchanged: (a-1)^2 + 4 S mu = (S q + mu/q)^2 for a = y + S q."""
    rng = np.random.default_rng(11)
    q = 10 ** rng.uniform(-2, 2, size=1000)
    S = 10 ** rng.uniform(-3, 2, size=1000)
    mu = rng.integers(1, 6, size=1000).astype(float)
    y = 1.0 - mu / q
    yp = orc.prox_poisson_dual(y + S * q, S, mu)
    np.testing.assert_allclose(yp, y, rtol=1e-9, atol=1e-11)


# ------------------------------------------------------------------ P8: TV


@pytest.mark.parametrize("shape", [(1, 7, 9), (4, 5, 6), (3, 1, 8)])
def test_grad_adjoint_and_norm(orc, shape):
    rng = np.random.default_rng(12)
    x = rng.normal(size=shape)
    q = rng.normal(size=(3,) + shape)
    lhs = float((orc.grad(x) * q).sum())
    rhs = float((x * orc.grad_adjoint(q)).sum())
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))
    # ||K|| by power iteration on K^T K vs. the closed form
    v = rng.normal(size=shape)
    for _ in range(3000):
        v = orc.grad_adjoint(orc.grad(v))
        v /= np.linalg.norm(v)
    lam = float(np.sqrt(np.linalg.norm(orc.grad_adjoint(orc.grad(v)))))
    assert abs(lam - orc.grad_norm(shape)) < 1e-6 * lam
    # and via the dense matrix for the smallest shape
    if np.prod(shape) <= 64:
        n = int(np.prod(shape))
        K = np.stack([orc.grad(np.eye(n)[i].reshape(shape)).reshape(-1) for i in range(n)], axis=1)
        assert abs(np.linalg.norm(K, 2) - orc.grad_norm(shape)) < 1e-10


def test_grad_values():
    """Forward differences: a ramp along each axis has unit gradient except in
    the last layer, where the difference is zero."""
    import oracle
    z, y, x = np.meshgrid(np.arange(3.0), np.arange(4.0), np.arange(5.0), indexing="ij")
    g = oracle.grad(2 * x + 3 * y - z)
    assert np.all(g[0][:, :, :-1] == 2) and np.all(g[0][:, :, -1] == 0)
    assert np.all(g[1][:, :-1, :] == 3) and np.all(g[1][:, -1, :] == 0)
    assert np.all(g[2][:-1] == -1) and np.all(g[2][-1] == 0)


def test_tv_dual_projection(orc):
    rng = np.random.default_rng(13)
    beta = 0.3
    v = rng.normal(scale=0.4, size=(3, 50))
    p = orc.prox_tv_dual(v, beta)
    nrm = np.sqrt((p ** 2).sum(0))
    assert np.all(nrm <= beta * (1 + 1e-12))
    inside = np.sqrt((v ** 2).sum(0)) <= beta
    np.testing.assert_array_equal(p[:, inside], v[:, inside])
    # nearest point of the ball: no random point of the ball is closer
    for j in range(v.shape[1]):
        cand = rng.normal(size=(3, 500))
        cand *= beta * rng.uniform(0, 1, size=500) ** (1 / 3) / np.sqrt((cand ** 2).sum(0))
        dbest = np.linalg.norm(p[:, j] - v[:, j])
        assert np.all(np.linalg.norm(cand - v[:, j:j + 1], axis=0) >= dbest - 1e-12)


# ------------------------------------------------- tiny listmode problem


def tiny_problem(seed=20, n_events=400, dup=True, nxy=8, n_det=16):
    """A 2D ring with few detectors: events drawn from the bins of a smooth
    image so that duplicates (mu > 1) occur."""
    p = lmsynth.tiny_2d(n_det=n_det, nxy=nxy)
    rng = np.random.default_rng(seed)
    sc = p.scanner
    i1, i2 = np.triu_indices(sc.n_det, 1)
    pairs = np.stack([i1, i2], 1)
    ks = np.arange(-p.tof.kmax, p.tof.kmax + 1)
    nb = len(pairs) * len(ks)
    if dup:
        pick = rng.integers(0, nb // 3, size=n_events)  # few bins -> duplicates
    else:
        pick = rng.choice(nb, size=n_events, replace=False)
    pr = pairs[pick % len(pairs)]
    k = ks[pick // len(pairs)]
    swap = rng.uniform(size=n_events) < 0.5
    a = np.where(swap, pr[:, 1], pr[:, 0])
    b = np.where(swap, pr[:, 0], pr[:, 1])
    k = np.where(swap, -k, k)
    ev = np.stack([a % sc.n_cry, a // sc.n_cry, b % sc.n_cry, b // sc.n_cry, k], 1).astype(np.int16)
    s = np.full(n_events, 0.05)
    x0 = np.full(p.image.shape_zyx, 0.8)
    return p, ev, s, x0


# ------------------------------------------------------------ P9: invariant


def test_z_invariant_every_update(orc):
    p, ev, s, x0 = tiny_problem()
    G = orc.Geometry.from_problem(p)
    g = orc.sens(G)
    n = 4
    seq = lmsynth.subset_sequence(7, 0, 60, n)
    checks = []

    def cb(st, su):
        z_ref = su.g + orc.back(G, (st.y - 1.0) / su.mu, ev) + orc.grad_adjoint(st.w)
        checks.append(np.abs(st.z - z_ref).max() / np.abs(z_ref).max())
        zb = st.zbar
        assert np.all(np.isfinite(zb))

    orc.lm_spdhg(G, ev, s, g, x0, n, seq, gamma=3 / x0.max(), rho=0.999, beta=0.05, callback=cb)
    assert len(checks) == 60 and max(checks) < 1e-12
    assert (seq == n).any() and (seq < n).any()


def test_z_init_equals_sinogram_dual_backprojection(orc):
    """z after initialisation is P^T y_sino with y_sino = 1 - d/(Px+s) over all
    bins (text after Algorithm 2); P is built densely over every bin."""
    p, ev, s, x0 = tiny_problem()
    G = orc.Geometry.from_problem(p)
    from tests.test_oracle_projector import all_bins
    bins = all_bins(p)
    keys_bins = orc.bin_keys(bins, p.scanner.n_cry)
    keys_ev = orc.bin_keys(ev, p.scanner.n_cry)
    index = {tuple(k): i for i, k in enumerate(keys_bins)}
    d = np.zeros(len(bins))
    for k in keys_ev:
        d[index[tuple(k)]] += 1
    P = orc.dense_matrix(G, bins)
    sb = np.full(len(bins), 0.05)
    y_sino = 1 - d / (P @ x0.reshape(-1) + sb)
    g = orc.sens(G)
    su = orc.lm_setup(G, ev, 1, g, 1.0, 0.999)
    st = orc.lm_init(G, ev, s, su, x0)
    np.testing.assert_allclose(st.z.reshape(-1), P.T @ y_sino, rtol=0, atol=1e-11 * np.abs(P.T @ y_sino).max())


# ------------------------------------------------- P10: LM = sinogram SPDHG


def _sino_setup(orc, p, ev):
    from tests.test_oracle_projector import all_bins
    bins = all_bins(p)
    keys_bins = orc.bin_keys(bins, p.scanner.n_cry)
    index = {tuple(k): i for i, k in enumerate(keys_bins)}
    bin_of_event = np.array([index[tuple(k)] for k in orc.bin_keys(ev, p.scanner.n_cry)])
    d = np.bincount(bin_of_event, minlength=len(bins)).astype(float)
    return bins, bin_of_event, d


def test_lm_equals_sinogram_one_subset_with_duplicates(orc):
    p, ev, s, x0 = tiny_problem(dup=True)
    G = orc.Geometry.from_problem(p)
    bins, boe, d = _sino_setup(orc, p, ev)
    assert d.max() >= 3
    P = orc.dense_matrix(G, bins)
    g = orc.sens(G)
    gamma, rho, beta = 3 / x0.max(), 0.999, 0.05
    seq = lmsynth.subset_sequence(3, 0, 40, 1)
    x_lm, st, su = orc.lm_spdhg(G, ev, s, g, x0, 1, seq, gamma, rho, beta)
    sb = np.full(len(bins), 0.05)
    # with one subset the sinogram step-size rule and the listmode rule coincide,
    # so the sinogram run derives T itself
    x_sino = orc.spdhg_sino(P, d, sb, x0, [np.arange(len(bins))], seq, gamma, rho, beta, G.shape,
                            p1_min=orc.p1_floor(G))
    np.testing.assert_allclose(x_lm, x_sino, rtol=0, atol=1e-12 * np.abs(x_sino).max())


def test_lm_equals_sinogram_subsets_unit_counts(orc):
    p, ev, s, x0 = tiny_problem(dup=False, n_events=300)
    G = orc.Geometry.from_problem(p)
    bins, boe, d = _sino_setup(orc, p, ev)
    assert d.max() == 1
    n = 5
    sub = orc.subset_ids(len(ev), n)
    # sinogram subset i = the bins of listmode subset i; empty bins in subset 0
    empty = np.nonzero(d == 0)[0]
    bos = [np.concatenate([boe[sub == i], empty if i == 0 else np.zeros(0, int)]) for i in range(n)]
    P = orc.dense_matrix(G, bins)
    g = orc.sens(G)
    gamma, rho, beta = 3 / x0.max(), 0.999, 0.05
    seq = lmsynth.subset_sequence(4, 0, 80, n)
    x_lm, st, su = orc.lm_spdhg(G, ev, s, g, x0, n, seq, gamma, rho, beta)
    sb = np.full(len(bins), 0.05)
    x_sino = orc.spdhg_sino(P, d, sb, x0, bos, seq, gamma, rho, beta, G.shape, T=su.T, p1_min=orc.p1_floor(G))
    np.testing.assert_allclose(x_lm, x_sino, rtol=0, atol=1e-12 * np.abs(x_sino).max())


def test_primal_step_rule_with_n_subsets(orc):
    """Pins the 1/n of Eq. lm_stepsizes, T_k = rho p_k / (gamma (P^T 1)/n),
    for n > 1 against the sinogram rule of Algorithm 1, which sums each
    subset's own rows, T_k = rho p_k / (gamma P_k^T 1).  A sinogram made of
    n copies of every bin, subset k = copy k, has P_k^T 1 = P^T 1 / n
    exactly (P^T 1 summed over the whole sinogram), so sinogram SPDHG with
    its own rule must coincide with LM-SPDHG given that sinogram's P^T 1 as
    g.  Event e lies in copy e mod n, as the interleaved listmode subsets
    put it; all counts are 1.  (With the 1/n dropped, T would be n times
    smaller and the two runs would part after the first update.)"""
    p, ev, s, x0 = tiny_problem(dup=False, n_events=300)
    G = orc.Geometry.from_problem(p)
    bins, boe, d1 = _sino_setup(orc, p, ev)
    assert d1.max() == 1
    n = 3
    M = len(bins)
    P1 = orc.dense_matrix(G, bins)
    P = np.tile(P1, (n, 1))                      # row c M + b: copy c of bin b
    row = (np.arange(len(ev)) % n) * M + boe     # event e -> copy e mod n
    d = np.zeros(n * M)
    d[row] = 1.0
    sb = np.full(n * M, 0.05)
    bos = [np.arange(c * M, (c + 1) * M) for c in range(n)]
    g = P.sum(axis=0).reshape(G.shape)           # P^T 1 of the sinogram = n orc.sens(G)
    np.testing.assert_allclose(g, n * orc.sens(G), rtol=1e-12, atol=0)
    gamma, rho, beta = 3 / x0.max(), 0.999, 0.05
    seq = lmsynth.subset_sequence(6, 0, 60, n)
    assert (seq < n).sum() > 10
    x_lm, st, su = orc.lm_spdhg(G, ev, s, g, x0, n, seq, gamma, rho, beta)
    # the sinogram run derives T from its subsets (T=None)
    x_sino = orc.spdhg_sino(P, d, sb, x0, bos, seq, gamma, rho, beta, G.shape, p1_min=orc.p1_floor(G))
    np.testing.assert_allclose(x_lm, x_sino, rtol=0, atol=1e-12 * np.abs(x_sino).max())


# ------------------------------------------------------------ P11: counts


def test_event_counts_brute_force(orc):
    p, ev, s, x0 = tiny_problem(n_events=1500)
    mu = orc.event_counts(ev, p.scanner.n_cry)
    nc = p.scanner.n_cry

    def same_bin(a, b):
        ia, ja = a[0] + nc * a[1], a[2] + nc * a[3]
        ib, jb = b[0] + nc * b[1], b[2] + nc * b[3]
        return (ia == ib and ja == jb and a[4] == b[4]) or (ia == jb and ja == ib and a[4] == -b[4])

    evl = [tuple(int(v) for v in e) for e in ev]
    for e in range(0, len(evl), 7):
        want = sum(1 for f in evl if same_bin(evl[e], f))
        assert mu[e] == want
    assert mu.max() > 1


# ------------------------------------------------------------ P12: subsets


def test_subsets_and_sequence():
    import oracle
    ids = oracle.subset_ids(1000, 28)
    assert np.array_equal(ids[:60], np.arange(60) % 28)
    # published first output of SplitMix64 seeded with 0
    assert lmsynth.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    seq = lmsynth.subset_sequence(2000, 0, 20000, 28)
    frac_prior = float((seq == 28).mean())
    assert abs(frac_prior - 0.5) < 0.02
    cnt = np.bincount(seq[seq < 28], minlength=28)
    assert cnt.min() > 0.6 * cnt.mean()
    # consecutive blocks equal one long draw (global update counter)
    a = lmsynth.subset_sequence(5, 0, 100, 28)
    b = np.concatenate([lmsynth.subset_sequence(5, 0, 56, 28), lmsynth.subset_sequence(5, 56, 44, 28)])
    assert np.array_equal(a, b)


# ------------------------------------------------------ P13: convergence


def test_cost_decreases(orc):
    """Qualitative only (the paper reports relative cost curves, no values):
    LM-SPDHG lowers the cost of Eq. (1) from the initial image."""
    p, ev, s, x0 = tiny_problem(n_events=600, seed=21)
    G = orc.Geometry.from_problem(p)
    g = orc.sens(G)
    gamma, rho, beta, n = 3 / x0.max(), 0.999, 0.05, 4
    c0 = orc.cost(G, x0, ev, s, g, beta)
    st = su = None
    costs = []
    for ep in range(12):
        seq = lmsynth.subset_sequence(9, ep * 2 * n, 2 * n, n)
        x, st, su = orc.lm_spdhg(G, ev, s, g, x0, n, seq, gamma, rho, beta, state=st, setup=su)
        costs.append(orc.cost(G, x, ev, s, g, beta))
    assert costs[-1] < c0
    assert costs[-1] <= min(costs[:3]) + 1e-9 * abs(c0)


def test_cost_equals_sinogram_objective(orc):
    """The listmode objective equals Eq. (1) written over every sinogram bin
    (dense P, binned counts d, the contamination of every bin) less the
    constant sum of s, with the TV term summed voxel by voxel: the data
    term's sign, the <g, x> term, the isotropic norm and the place of beta
    each change the value."""
    p, ev, s, _ = tiny_problem(n_events=500, seed=23)
    G = orc.Geometry.from_problem(p)
    bins, _, d = _sino_setup(orc, p, ev)
    P = orc.dense_matrix(G, bins)
    rng = np.random.default_rng(24)
    shape = p.image.shape_zyx
    x = rng.uniform(0.2, 2.0, size=shape)
    g = P.sum(axis=0).reshape(shape)
    sb = np.full(len(bins), 0.05)
    q = P @ x.reshape(-1) + sb
    data = float((q - d * np.log(q)).sum() - sb.sum())
    tv = 0.0
    nz, ny, nx = shape
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                dx = x[k, j, i + 1] - x[k, j, i] if i + 1 < nx else 0.0
                dy = x[k, j + 1, i] - x[k, j, i] if j + 1 < ny else 0.0
                dz = x[k + 1, j, i] - x[k, j, i] if k + 1 < nz else 0.0
                tv += np.sqrt(dx * dx + dy * dy + dz * dz)
    beta = 0.07
    want = data + beta * tv
    got = orc.cost(G, x, ev, s, g, beta)
    assert abs(got - want) <= 1e-11 * abs(want)
    assert abs(orc.cost(G, x, ev, s, g, 0.0) - data) <= 1e-11 * abs(data)


# ------------------------------------- conditioning of the TV dual w


def test_tv_dual_sup_norm_follows_rounding_of_the_state(orc):
    """How far float32 rounding alone moves the iterates of Algorithm 2 on
    the 2D workload (28 subsets, TV beta 0.03): two oracle runs with the
    same inputs and sequence, one of which rounds its state (x, z, zbar,
    w, 1 - y) to float32 after every update.  After 5 epochs x moves by
    ~1e-6 of its maximum and w by ~1e-5 in relative L2, but w moves by
    ~1e-3 beta in sup norm: on the beta-sphere w follows the direction of
    K x, a difference of nearly equal values of x in flat regions, whose
    relative error is far above that of x.  This fixes the sup-norm
    tolerance of w in the GPU parity tests (1e-2 beta, about ten times what
    the rounding of the stored state alone produces here) and keeps the other
    iterates at the 1e-4 bound."""
    import copy
    from tests.helpers import problem_2d
    p = problem_2d()
    G = orc.Geometry.from_problem(p)
    g = orc.sens(G).astype(np.float32).astype(np.float64)
    n, beta, rho = 28, 0.03, 0.999
    gamma = float(np.float32(3.0 / float(p.x0.max())))
    s = p.s.astype(np.float64)
    su = orc.lm_setup(G, p.events, n, g, gamma, rho)
    a = orc.lm_init(G, p.events, s, su, p.x0)
    b = copy.deepcopy(a)
    f32 = lambda v: v.astype(np.float32).astype(np.float64)
    w_sup = []
    for ep in range(5):
        for i in lmsynth.subset_sequence(2000, ep * 2 * n, 2 * n, n):
            orc.lm_update(G, p.events, s, su, a, int(i), n, beta)
            orc.lm_update(G, p.events, s, su, b, int(i), n, beta)
            b.x, b.z, b.zbar, b.w, b.y = f32(b.x), f32(b.z), f32(b.zbar), f32(b.w), 1.0 - f32(1.0 - b.y)
        w_sup.append(float(np.abs(a.w - b.w).max() / beta))
    dx = float(np.abs(a.x - b.x).max() / np.abs(a.x).max())
    dz = float(np.abs(a.z - b.z).max() / np.abs(a.z).max())
    dw2 = float(np.linalg.norm(a.w - b.w) / np.linalg.norm(a.w))
    print(f"rounded state after 5 epochs: x {dx:.2e}, z {dz:.2e}, w rel. L2 {dw2:.2e}, "
          f"w sup / beta per epoch {['%.1e' % v for v in w_sup]}")
    assert dx < 1e-5 and dz < 1e-5 and dw2 < 1e-4
    # the sup norm of w is two to three orders of magnitude more sensitive
    assert max(w_sup) > 100 * dx
    # the GPU tolerance of 1e-2 beta stays well above this figure
    assert 1e-4 < max(w_sup) < 2e-3
