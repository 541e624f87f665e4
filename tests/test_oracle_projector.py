"""Pins of the FP64 oracle's projector pair against facts outside the oracle:
matrix adjointness, exact line integrals of linear images, chord lengths of
a uniform disc, quadrature of the truncated Gaussian TOF kernel, the
telescoping sum over TOF bins and the detector-swap symmetry."""
import math

import numpy as np
import pytest
from scipy import integrate

import lmsynth


def geom_of(p, orc, tof_on=None):
    return orc.Geometry.from_problem(p, tof_on=tof_on)


def all_bins(p):
    """Every (unordered crystal pair, TOF bin) of a small scanner as events."""
    sc = p.scanner
    nd = sc.n_det
    i1, i2 = np.triu_indices(nd, 1)
    c1, r1 = i1 % sc.n_cry, i1 // sc.n_cry
    c2, r2 = i2 % sc.n_cry, i2 // sc.n_cry
    ks = np.arange(-p.tof.kmax, p.tof.kmax + 1)
    rows = []
    for k in ks:
        rows.append(np.stack([c1, r1, c2, r2, np.full_like(c1, k)], axis=1))
    return np.concatenate(rows).astype(np.int16)


# ---------------------------------------------------------------- P1: adjoint


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_dense_adjoint(orc, which):
    p = lmsynth.tiny_2d() if which == "2d" else lmsynth.tiny_3d(n_cry=12, n_ring=3, nxy=6, nz=3)
    G = geom_of(p, orc)
    ev = all_bins(p)
    P = orc.dense_matrix(G, ev)
    assert P.shape[1] == p.image.nvox and np.count_nonzero(P) > 0
    rng = np.random.default_rng(1)
    v = rng.normal(size=len(ev))
    x = rng.normal(size=G.shape)
    # the back projector is the transpose of the matrix built from the forward one
    np.testing.assert_allclose(orc.back(G, v, ev).reshape(-1), P.T @ v, rtol=0, atol=1e-12 * np.abs(P).sum())
    lhs = float(orc.fwd(G, x, ev) @ v)
    rhs = float((x * orc.back(G, v, ev)).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


# ------------------------------------------------------- P2: exact integrals


def test_axis_aligned_row_sum(orc):
    """LOR along x through the centre row of an image with odd ny: Joseph is
    h times the sum of that row."""
    p = lmsynth.tiny_2d(n_det=16, nxy=9, h=1.5, radius=20.0, tof_on=False)
    G = geom_of(p, orc, tof_on=False)
    rng = np.random.default_rng(2)
    x = rng.uniform(0.5, 2.0, size=G.shape)
    ev = np.array([[0, 0, 8, 0, 0], [8, 0, 0, 0, 0], [4, 0, 12, 0, 0]], dtype=np.int16)
    val = orc.fwd(G, x, ev)
    j0 = (9 - 1) // 2
    assert abs(val[0] - 1.5 * x[0, j0, :].sum()) < 1e-12 * val[0]
    assert abs(val[1] - 1.5 * x[0, j0, :].sum()) < 1e-12 * val[1]
    # crystal 4 / 12 sit at +-90 degrees: the LOR runs along y through column j0
    assert abs(val[2] - 1.5 * x[0, :, j0].sum()) < 1e-12 * val[2]


def _linear_image(G, coef):
    z = (np.arange(G.n[2]) - (G.n[2] - 1) / 2) * G.h[2]
    y = (np.arange(G.n[1]) - (G.n[1] - 1) / 2) * G.h[1]
    x = (np.arange(G.n[0]) - (G.n[0] - 1) / 2) * G.h[0]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return coef[0] + coef[1] * X + coef[2] * Y + coef[3] * Z


def _line_integral_linear(G, det, ev, coef):
    """Exact integral of a linear function along the LOR between the two image
    faces perpendicular to the dominant axis: length times the value at the
    midpoint (the midpoint rule is exact for linear functions)."""
    p1 = det[ev[0] + G.n_cry * ev[1]].astype(np.float64)
    p2 = det[ev[2] + G.n_cry * ev[3]].astype(np.float64)
    d = p2 - p1
    a = int(np.argmax(np.abs(det[ev[2] + G.n_cry * ev[3]] - det[ev[0] + G.n_cry * ev[1]])))
    half = 0.5 * G.n[a] * G.h[a]
    lam_c = (0.0 - p1[a]) / d[a]
    mid = p1 + lam_c * d
    length = 2 * half * np.linalg.norm(d) / abs(d[a])
    val = coef[0] + coef[1] * mid[0] + coef[2] * mid[1] + coef[3] * mid[2]
    return length * val, p1, d, a


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_image_exact(orc, dim):
    """Bilinear interpolation reproduces a linear image, so the Joseph value of
    a LOR that stays well inside the image equals the exact line integral."""
    if dim == 2:
        p = lmsynth.tiny_2d(n_det=180, nxy=41, h=1.0, radius=40.0, tof_on=False)
        coef = (3.0, 0.2, -0.5, 0.0)
        evs = [(0, 0, 91, 0, 0), (1, 0, 90, 0, 0), (45, 0, 136, 0, 0), (92, 0, 2, 0, 0), (44, 0, 133, 0, 0)]
    else:
        p = lmsynth.tiny_3d(n_cry=180, n_ring=9, nxy=41, nz=9, h=1.0, radius=40.0, pitch=1.0, tof_on=False)
        coef = (3.0, 0.2, -0.5, 0.7)
        evs = [(0, 2, 91, 6, 0), (1, 7, 90, 1, 0), (45, 4, 136, 5, 0), (92, 0, 2, 8, 0)]
    G = geom_of(p, orc, tof_on=False)
    x = _linear_image(G, coef)
    det = p.det
    for e in evs:
        ev = np.array([e], dtype=np.int16)
        want, p1, d, a = _line_integral_linear(G, det, e, coef)
        # the LOR must stay at least one voxel inside the other axes
        for b in range(3):
            if b == a or G.n[b] == 1:
                continue
            for lam in ((-(0.5 * G.n[a] * G.h[a]) - p1[a]) / d[a], ((0.5 * G.n[a] * G.h[a]) - p1[a]) / d[a]):
                assert abs(p1[b] + lam * d[b]) < 0.5 * (G.n[b] - 3) * G.h[b]
        got = orc.fwd(G, x, ev)[0]
        assert abs(got - want) < 1e-10 * abs(want), (e, got, want)


# ------------------------------------------------------- P3: disc chords


def _disc_image(G, cx, cy, r, ss=8):
    xs = (np.arange(G.n[0]) - (G.n[0] - 1) / 2) * G.h[0]
    ys = (np.arange(G.n[1]) - (G.n[1] - 1) / 2) * G.h[1]
    off = (np.arange(ss) + 0.5) / ss - 0.5
    acc = np.zeros((G.n[1], G.n[0]))
    for dy in off:
        for dx in off:
            X = xs[None, :] + dx * G.h[0]
            Y = ys[:, None] + dy * G.h[1]
            acc += ((X - cx) ** 2 + (Y - cy) ** 2 <= r * r)
    return (acc / ss ** 2)[None]


def _lor_geometry(det, e, n_cry):
    p1 = det[e[0] + n_cry * e[1]].astype(np.float64)
    p2 = det[e[2] + n_cry * e[3]].astype(np.float64)
    return p1, p2, p2 - p1


def test_disc_chords_nontof(orc):
    p = lmsynth.tiny_2d(n_det=256, nxy=200, h=0.25, radius=40.0, tof_on=False)
    G = geom_of(p, orc, tof_on=False)
    r = 20.0
    x = _disc_image(G, 0.0, 0.0, r)
    ev = lmsynth.random_events(p, 300, seed=3, min_sep=20)
    vals = orc.fwd(G, x, ev)
    det = p.det
    checked = 0
    for e, v in zip(ev, vals):
        p1, p2, d = _lor_geometry(det, e, G.n_cry)
        b = abs(p1[0] * d[1] - p1[1] * d[0]) / np.hypot(d[0], d[1])
        if b < 0.9 * r:
            chord = 2 * math.sqrt(r * r - b * b)
            assert abs(v - chord) < 0.01 * chord, (e, v, chord)
            checked += 1
        elif b > r + 1.0:
            assert v == 0.0
    assert checked > 50


# --------------------------------------------- P4, P5: the TOF kernel


def _w_quad(G, k, t):
    """Bin-k integral of the truncated, renormalised Gaussian centred at t,
    by quadrature of exp (independent of the erf closed form)."""
    sig = G.sigma
    ns = G.tof_nsig
    Z = integrate.quad(lambda u: math.exp(-0.5 * (u / sig) ** 2), -ns * sig, ns * sig, epsabs=1e-14)[0]
    lo = max(k * G.tof_bin - 0.5 * G.tof_bin - t, -ns * sig)
    hi = min(k * G.tof_bin + 0.5 * G.tof_bin - t, ns * sig)
    if hi <= lo:
        return 0.0
    return integrate.quad(lambda u: math.exp(-0.5 * (u / sig) ** 2), lo, hi, epsabs=1e-14)[0] / Z


def test_tof_weight_quadrature(orc):
    p = lmsynth.tiny_2d(n_tof=9, tof_bin=6.0, fwhm=9.0)
    G = geom_of(p, orc)
    for k in (-4, -1, 0, 2, 4):
        for t in (-31.0, -10.3, -2.0, 0.0, 1.7, 5.5, 14.0, 30.0):
            assert abs(orc.tof_weight(G, k, t) - _w_quad(G, k, t)) < 1e-12


def test_tof_weights_sum_to_one(orc):
    p = lmsynth.config_2d()
    G = geom_of(p, orc)
    cover = p.tof.n_tof * p.tof.bin / 2 - p.tof.nsigma * p.tof.sigma
    for t in np.linspace(-cover, cover, 57):
        tot = sum(orc.tof_weight(G, k, t) for k in range(-p.tof.kmax, p.tof.kmax + 1))
        assert abs(tot - 1.0) < 1e-14
    # outside the covered range the sum drops below one
    tot = sum(orc.tof_weight(G, k, cover + 20.0) for k in range(-p.tof.kmax, p.tof.kmax + 1))
    assert tot < 1.0 - 1e-3


def test_tof_sum_equals_nontof_projection(orc):
    """Summing the TOF projections over all bins gives the non-TOF projection
    for LORs whose image part lies inside the covered TOF range."""
    p = lmsynth.config_2d()
    G = geom_of(p, orc)
    Gn = geom_of(p, orc, tof_on=False)
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, size=G.shape)
    base = lmsynth.random_events(p, 40, seed=5, min_sep=60)
    tot = np.zeros(len(base))
    for k in range(-p.tof.kmax, p.tof.kmax + 1):
        ev = base.copy()
        ev[:, 4] = k
        tot += orc.fwd(G, x, ev)
    nontof = orc.fwd(Gn, x, base)
    np.testing.assert_allclose(tot, nontof, rtol=1e-12, atol=1e-12)


def test_tof_disc_offcentre(orc):
    """TOF-weighted chord of an off-centre uniform disc: the integral of the
    bin weight over the chord, with t measured from the LOR centre towards
    crystal 2.  Pins the sign of t and the bin centres."""
    p = lmsynth.tiny_2d(n_det=256, nxy=200, h=0.25, radius=40.0, n_tof=9, tof_bin=5.0, fwhm=8.0)
    G = geom_of(p, orc)
    cx, cy, r = 6.0, -4.0, 12.0
    x = _disc_image(G, cx, cy, r)
    det = p.det
    rng = np.random.default_rng(6)
    n_ok = 0
    cand = lmsynth.random_events(p, 400, seed=9, min_sep=40)
    for e in cand:
        p1, p2, d = _lor_geometry(det, e, G.n_cry)
        dn = np.linalg.norm(d)
        u = d / dn
        mid = p1 + 0.5 * d
        c = np.array([cx, cy, 0.0])
        tc = float((c - mid) @ u)
        b = float(np.linalg.norm((c - mid) - tc * u))
        if b > 0.8 * r:
            continue
        half = math.sqrt(r * r - b * b)
        # a TOF bin that overlaps the disc, on either side of its centre
        e = e.copy()
        e[4] = int(np.clip(round(tc / G.tof_bin) + rng.integers(-1, 2), -p.tof.kmax, p.tof.kmax))
        want = integrate.quad(lambda t: _w_quad(G, int(e[4]), t), tc - half, tc + half,
                              epsabs=1e-10, limit=200)[0]
        got = orc.fwd(G, x, e[None])[0]
        assert abs(got - want) < 0.01 * want + 1e-3 * 2 * half, (e, got, want)
        n_ok += 1
        if n_ok == 30:
            break
    assert n_ok >= 15


# ------------------------------------------------------- P6: symmetry


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_swap_symmetry(orc, which):
    p = lmsynth.config_2d() if which == "2d" else lmsynth.tiny_3d(n_cry=64, n_ring=8, nxy=24, nz=8,
                                                                   radius=40.0, pitch=2.0)
    G = geom_of(p, orc)
    rng = np.random.default_rng(7)
    x = rng.uniform(0, 1, size=G.shape)
    ev = lmsynth.random_events(p, 200, seed=8)
    sw = ev[:, [2, 3, 0, 1, 4]].copy()
    sw[:, 4] = -sw[:, 4]
    a, b = orc.fwd(G, x, ev), orc.fwd(G, x, sw)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)


# --------------------------------------------------- sensitivity image


def test_sens_is_backprojection_of_all_bins(orc):
    p = lmsynth.tiny_3d(n_cry=12, n_ring=3, nxy=6, nz=3)
    G = geom_of(p, orc)
    ev = all_bins(p)
    g = orc.sens(G)
    np.testing.assert_allclose(g, orc.back(G, np.ones(len(ev)), ev), rtol=1e-12, atol=1e-12)


def test_sens_tof_equals_nontof_inside_coverage(orc):
    """With the TOF range covering every LOR inside the image, the TOF-summed
    sensitivity equals the non-TOF one."""
    p = lmsynth.tiny_2d(n_det=32, nxy=8, h=2.0, radius=20.0, n_tof=21, tof_bin=6.0, fwhm=9.0)
    G = geom_of(p, orc)
    np.testing.assert_allclose(orc.sens(G), orc.sens(G.with_tof(False)), rtol=1e-12, atol=1e-12)
