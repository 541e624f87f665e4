"""FP64 CPU oracle for listmode SPDHG (LM-SPDHG).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline of the benchmark are the only code allowed to import this package.
It shares no code with the HIP library (``paper_2201_05497_amd``) and never
imports it; the library never imports this.  Everything is plain, slow,
float64 and single-threaded, written to be checked against the paper by eye.

The projector pair lives in ``lm_oracle.c`` (compiled with gcc on first
use); this module holds the algorithm: event counts, subsets, step sizes,
the dual proxes, the finite-difference operator K, LM-SPDHG (Algorithm 2),
sinogram SPDHG on a dense system matrix (Algorithm 1), the cost (Eq. 1) and
the listmode EM-TV warm start (Algorithm 3).

Readings of the paper taken here, where it is silent or ambiguous:

* event count mu_e: the number of events in the list whose bin (unordered
  crystal pair, TOF bin with the sign flipped when the pair is swapped) is
  the bin of e (footnote to Algorithm 2);
* subsets: event e (0-based chronological index) belongs to subset e mod n
  (text after Algorithm 2);
* the subset sequence is an input (random choices are drawn outside);
* the dual prox of the data branch uses 4 S_e mu_e under the square root
  (Eq. proxD with d_{i_e} = mu_e; Appendix A gives the same term);
* z initialisation uses "+": z = P^T 1 + P^LM^T((y-1)/mu) + K^T w, the only
  sign for which z equals P^T of the sinogram dual built from Eq. (yinit)
  (the printed "-" contradicts the sentence that follows the algorithm);
* K = forward differences with zero (Neumann) boundary, no voxel-size
  scaling; ||K|| is its exact largest singular value; for DTV, K = D grad
  with the full projection D and the same ||grad|| as the norm bound;
* T = min over the subset step sizes and the prior step size:
  T_j = rho / (2 gamma max(g_j, ||K||)) with p_k = 1/(2n), p_prior = 1/2;
  S_e = gamma rho / (P^LM 1)_e, and 0 where the LOR misses the image,
  read as (P^LM 1)_e <= 1e-6 of the smallest voxel size (in mm, the unit
  of P^LM 1): a LOR that meets the image only within rounding (a corner
  weight of 1e-12 where a boundary plane is crossed at an edge) carries no
  dual step, where 1 / (P^LM 1)_e would make it arbitrarily large;
* attenuation and normalisation (inside P, Section 1) are one factor per
  event's LOR, P' = diag(m) P; limited resolution is an image-space
  separable Gaussian B with a zero boundary, P = G B; the sensitivity g of
  the whole operator is an input.

The readings of the EM-TV warm start and of the DTV prior are listed with
their code below.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Callable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lm_oracle.c")
_LIB = os.path.join(_HERE, "liblm_oracle.so")


def build(force: bool = False) -> str:
    """Compile lm_oracle.c into liblm_oracle.so with gcc (plain -O2, IEEE)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c11",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [("det", ctypes.POINTER(ctypes.c_float)),
                ("n_cry", ctypes.c_int32), ("n_ring", ctypes.c_int32),
                ("n", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3),
                ("n_tof", ctypes.c_int32), ("tof_bin", ctypes.c_double),
                ("tof_fwhm", ctypes.c_double), ("tof_nsig", ctypes.c_double),
                ("tof_on", ctypes.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        sp = ctypes.POINTER(ctypes.c_int16)
        gp = ctypes.POINTER(_Geom)
        lib.orc_fwd.argtypes = [gp, dp, sp, ctypes.c_int64, dp]
        lib.orc_back.argtypes = [gp, dp, sp, ctypes.c_int64, dp]
        lib.orc_sens.argtypes = [gp, dp]
        lib.orc_tof_weight.argtypes = [gp, ctypes.c_int, ctypes.c_double]
        lib.orc_tof_weight.restype = ctypes.c_double
        _lib = lib
    return _lib


class Geometry:
    """Scanner table + image grid + TOF parameters, as the C oracle sees them.

    ``det`` is the float32 crystal table; ``n`` = (nx, ny, nz); ``h`` the voxel
    size in mm; TOF: ``n_tof`` bins of width ``tof_bin``, Gaussian FWHM
    ``tof_fwhm``, truncated at ``tof_nsig`` sigma; ``tof_on`` False gives the
    non-TOF projector.
    """

    def __init__(self, det, n_cry, n_ring, n, h, n_tof, tof_bin, tof_fwhm,
                 tof_nsig=3.0, tof_on=True):
        self.det = np.ascontiguousarray(det, dtype=np.float32)
        assert self.det.shape == (n_cry * n_ring, 3)
        self.n_cry, self.n_ring = int(n_cry), int(n_ring)
        self.n = tuple(int(v) for v in n)
        self.h = tuple(float(v) for v in h)
        self.n_tof, self.tof_bin, self.tof_fwhm = int(n_tof), float(tof_bin), float(tof_fwhm)
        self.tof_nsig, self.tof_on = float(tof_nsig), bool(tof_on)
        self._c = _Geom(self.det.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                        self.n_cry, self.n_ring, (ctypes.c_int32 * 3)(*self.n),
                        (ctypes.c_double * 3)(*self.h), self.n_tof, self.tof_bin,
                        self.tof_fwhm, self.tof_nsig, int(self.tof_on))

    @classmethod
    def from_problem(cls, p, tof_on: Optional[bool] = None) -> "Geometry":
        sc, img, tof = p.scanner, p.image, p.tof
        return cls(p.det, sc.n_cry, sc.n_ring, img.n, img.h, tof.n_tof, tof.bin, tof.fwhm,
                   tof.nsigma, tof.on if tof_on is None else tof_on)

    def with_tof(self, on: bool) -> "Geometry":
        return Geometry(self.det, self.n_cry, self.n_ring, self.n, self.h, self.n_tof,
                        self.tof_bin, self.tof_fwhm, self.tof_nsig, on)

    @property
    def shape(self):
        """Image array shape, C-order [z][y][x]."""
        return (self.n[2], self.n[1], self.n[0])

    @property
    def sigma(self) -> float:
        return self.tof_fwhm / (2.0 * np.sqrt(2.0 * np.log(2.0)))


def _ev(events) -> np.ndarray:
    ev = np.ascontiguousarray(events, dtype=np.int16)
    assert ev.ndim == 2 and ev.shape[1] == 5
    return ev


# --------------------------------------------------------------------------
# operators (C): P^LM, its adjoint, sensitivity


def fwd(geom: Geometry, x: np.ndarray, events) -> np.ndarray:
    """(P^LM x)_e for every event (Eq. lmop), float64."""
    lib = _load()
    ev = _ev(events)
    xd = np.ascontiguousarray(x, dtype=np.float64).reshape(geom.shape)
    out = np.zeros(len(ev), dtype=np.float64)
    lib.orc_fwd(ctypes.byref(geom._c), xd.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                ev.ctypes.data_as(ctypes.POINTER(ctypes.c_int16)), len(ev),
                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def back(geom: Geometry, v: np.ndarray, events, img: Optional[np.ndarray] = None) -> np.ndarray:
    """img + (P^LM)^T v (the adjoint of ``fwd``), float64."""
    lib = _load()
    ev = _ev(events)
    vd = np.ascontiguousarray(v, dtype=np.float64)
    assert vd.shape == (len(ev),)
    out = np.zeros(geom.shape, dtype=np.float64) if img is None else np.array(img, dtype=np.float64)
    lib.orc_back(ctypes.byref(geom._c), vd.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                 ev.ctypes.data_as(ctypes.POINTER(ctypes.c_int16)), len(ev),
                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def sens(geom: Geometry) -> np.ndarray:
    """g = P^T 1 over all unordered crystal pairs and all TOF bins."""
    lib = _load()
    out = np.zeros(geom.shape, dtype=np.float64)
    lib.orc_sens(ctypes.byref(geom._c), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def tof_weight(geom: Geometry, k: int, t: float) -> float:
    return float(_load().orc_tof_weight(ctypes.byref(geom._c), int(k), float(t)))


def dense_matrix(geom: Geometry, events) -> np.ndarray:
    """Rows of P for the given events, built by projecting every basis image."""
    ev = _ev(events)
    nvox = int(np.prod(geom.n))
    P = np.zeros((len(ev), nvox))
    for v in range(nvox):
        b = np.zeros(nvox)
        b[v] = 1.0
        P[:, v] = fwd(geom, b, ev)
    return P


# --------------------------------------------------------------------------
# event bookkeeping (Algorithm 2: event counts and the split into sublists)


def bin_keys(events, n_cry: int) -> np.ndarray:
    """Canonical bin of each event: (id1, id2, k) with id1 <= id2, where the
    two crystals are swapped and k negated when id1 > id2."""
    ev = np.asarray(events, dtype=np.int64)
    id1 = ev[:, 0] + n_cry * ev[:, 1]
    id2 = ev[:, 2] + n_cry * ev[:, 3]
    k = ev[:, 4]
    sw = id1 > id2
    a = np.where(sw, id2, id1)
    b = np.where(sw, id1, id2)
    kk = np.where(sw, -k, k)
    return np.stack([a, b, kk], axis=1)


def event_counts(events, n_cry: int) -> np.ndarray:
    """mu_e = number of events in the list with the same bin as e."""
    keys = bin_keys(events, n_cry)
    # one integer per bin: (id1, id2, k) packed into 20 + 20 + 20 bits
    assert keys[:, :2].max(initial=0) < (1 << 20) and np.abs(keys[:, 2]).max(initial=0) < (1 << 19)
    flat = (keys[:, 0] << 40) | (keys[:, 1] << 20) | (keys[:, 2] + (1 << 19))
    _u, inv, cnt = np.unique(flat, return_inverse=True, return_counts=True)
    return cnt[np.asarray(inv).reshape(-1)].astype(np.int64)


def subset_ids(n_events: int, n_subsets: int) -> np.ndarray:
    """Subset of each event: every n-th event goes to the same sublist."""
    return np.arange(n_events, dtype=np.int64) % n_subsets


# --------------------------------------------------------------------------
# prior: K = forward differences, R = mixed L2-L1 norm (Section 3, TV prior)


def grad(x: np.ndarray) -> np.ndarray:
    """K x: forward differences along x, y, z (array axes 2, 1, 0), zero in
    the last layer of each axis.  Returns [3][nz][ny][nx]."""
    out = np.zeros((3,) + x.shape)
    for comp, ax in enumerate((2, 1, 0)):
        sl_hi = [slice(None)] * 3
        sl_lo = [slice(None)] * 3
        sl_hi[ax] = slice(1, None)
        sl_lo[ax] = slice(None, -1)
        out[comp][tuple(sl_lo)] = x[tuple(sl_hi)] - x[tuple(sl_lo)]
    return out


def grad_adjoint(q: np.ndarray) -> np.ndarray:
    """K^T q, the exact adjoint of ``grad``."""
    out = np.zeros(q.shape[1:])
    for comp, ax in enumerate((2, 1, 0)):
        sl_hi = [slice(None)] * 3
        sl_lo = [slice(None)] * 3
        sl_hi[ax] = slice(1, None)
        sl_lo[ax] = slice(None, -1)
        qc = q[comp]
        out[tuple(sl_hi)] += qc[tuple(sl_lo)]
        out[tuple(sl_lo)] -= qc[tuple(sl_lo)]
    return out


def grad_norm(shape_zyx: Sequence[int]) -> float:
    """Largest singular value of K: the forward-difference matrix of length N
    with a zero last row has singular values 2 sin(pi j / (2N)), j < N, so
    ||K||^2 = sum over axes of 4 sin^2(pi (N-1) / (2N))."""
    return float(np.sqrt(sum(4.0 * np.sin(np.pi * (N - 1) / (2.0 * N)) ** 2 for N in shape_zyx)))


def prox_tv_dual(v: np.ndarray, beta: float) -> np.ndarray:
    """beta * prox_{R*}(v / beta) for R = ||.||_{2,1}: the projection of v onto
    the pointwise Euclidean ball of radius beta (v has components first)."""
    nrm = np.sqrt((v ** 2).sum(axis=0))
    return v / np.maximum(1.0, nrm / beta)[None]


def tv(x: np.ndarray) -> float:
    return float(np.sqrt((grad(x) ** 2).sum(axis=0)).sum())


# Directional TV (Section 3; Ehrhardt & Betcke, SIAM J. Imaging Sci. 9,
# 2016): K = D grad with D_j = I - xi_j xi_j^T, which removes from the
# finite-difference vector of voxel j its component along the normalised
# gradient of a structural prior image v:
#   xi = grad v / sqrt(|grad v|^2 + eta^2).
# Readings: the full projection (no weight below one on xi xi^T); eta is an
# input; ||D grad|| <= ||grad|| (|D_j| <= 1), so the step sizes keep ||grad||.


def dtv_field(v: np.ndarray, eta: float) -> np.ndarray:
    """xi of the DTV prior for the prior image v, [3][nz][ny][nx]."""
    gv = grad(np.asarray(v, dtype=np.float64))
    return gv / np.sqrt((gv ** 2).sum(axis=0) + eta * eta)[None]


def dtv_project(xi: np.ndarray, q: np.ndarray) -> np.ndarray:
    """D q = q - xi (xi . q) per voxel (D is symmetric)."""
    return q - xi * (xi * q).sum(axis=0)[None]


# Image-space resolution model (Section 1: P includes limited spatial
# resolution): P = G B with B a separable Gaussian convolution.  Readings:
# FWHM given in voxels per axis, taps truncated at ceil(3 sigma) and
# normalised to sum 1, zero outside the image (so B is symmetric: B^T = B).


def blur(x: np.ndarray, fwhm_vox: Sequence[float]) -> np.ndarray:
    """B x for an image [nz][ny][nx]; fwhm_vox = (fx, fy, fz) in voxels, 0
    leaves that axis alone."""
    out = np.array(x, dtype=np.float64)
    for comp, ax in enumerate((2, 1, 0)):
        fw = float(fwhm_vox[comp])
        if fw <= 0:
            continue
        sig = fw / (2.0 * np.sqrt(2.0 * np.log(2.0)))
        r = int(np.ceil(3.0 * sig))
        t = np.arange(-r, r + 1)
        w = np.exp(-t * t / (2.0 * sig * sig))
        w /= w.sum()
        n = out.shape[ax]
        res = np.zeros_like(out)
        for tk, wk in zip(t, w):
            # res[j] += wk * out[j + tk] where 0 <= j + tk < n
            lo, hi = max(0, -tk), min(n, n - tk)
            if lo >= hi:
                continue
            dst = [slice(None)] * 3
            src = [slice(None)] * 3
            dst[ax] = slice(lo, hi)
            src[ax] = slice(lo + tk, hi + tk)
            res[tuple(dst)] += wk * out[tuple(src)]
        out = res
    return out


def k_op(x: np.ndarray, xi: Optional[np.ndarray] = None) -> np.ndarray:
    """K x: grad x for TV, D grad x for DTV."""
    return grad(x) if xi is None else dtv_project(xi, grad(x))


def k_adj(w: np.ndarray, xi: Optional[np.ndarray] = None) -> np.ndarray:
    """K^T w: grad^T w for TV, grad^T D w for DTV."""
    return grad_adjoint(w if xi is None else dtv_project(xi, w))


# --------------------------------------------------------------------------
# data term


def prox_poisson_dual(a: np.ndarray, S: np.ndarray, d: np.ndarray) -> np.ndarray:
    """prox of S D*(.; d) at a, pointwise (Eq. proxD)."""
    return 0.5 * (a + 1.0 - np.sqrt((a - 1.0) ** 2 + 4.0 * S * d))


def poisson_dual_conj(y: np.ndarray, d: np.ndarray) -> np.ndarray:
    """D*(y; d) (the conjugate of the Poisson negative log-likelihood)."""
    y = np.asarray(y, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    out = np.full(np.broadcast(y, d).shape, np.inf)
    pos = (d > 0) & (y < 1)
    out = np.where(pos, -d + d * np.log(np.where(pos, d, 1.0) / np.where(pos, 1.0 - y, 1.0)), out)
    out = np.where((d == 0) & (y <= 1), 0.0, out)
    return out


def cost(geom: Geometry, x: np.ndarray, events, s: np.ndarray, g: np.ndarray, beta: float,
         xi: Optional[np.ndarray] = None) -> float:
    """Listmode form of Eq. (1) without the constant sum of s over all bins:
    <g, x> - sum_e log((P^LM x)_e + s_e) + beta ||K x||_{2,1} (K of DTV
    when xi is given)."""
    q = fwd(geom, x, events) + s
    prior = float(np.sqrt((k_op(x, xi) ** 2).sum(axis=0)).sum())
    return float((g * x).sum() - np.log(q).sum() + beta * prior)


# --------------------------------------------------------------------------
# LM-SPDHG (Algorithm 2)


@dataclasses.dataclass
class LMState:
    x: np.ndarray
    z: np.ndarray
    zbar: np.ndarray
    w: np.ndarray
    y: np.ndarray
    u: int = 0


@dataclasses.dataclass
class LMSetup:
    mu: np.ndarray
    subsets: list
    S: np.ndarray
    S_prior: float
    T: np.ndarray
    g: np.ndarray
    knorm: float
    xi: Optional[np.ndarray] = None  # DTV field; None: TV
    m: Optional[np.ndarray] = None   # per-event multiplicative factors; None: 1
    fwhm: Optional[Sequence[float]] = None  # resolution model B (voxels); None: none


def _fwd_model(geom: Geometry, setup: "LMSetup", x: np.ndarray, ev: np.ndarray, m) -> np.ndarray:
    """(P' x)_e = m_e (G B x)_e for the events ev (m a scalar or per event)."""
    xb = x if setup.fwhm is None else blur(x, setup.fwhm)
    return m * fwd(geom, xb, ev)


def _back_model(geom: Geometry, setup: "LMSetup", v: np.ndarray, ev: np.ndarray, m) -> np.ndarray:
    """P'^T v = B G^T (m v)."""
    b = back(geom, m * v, ev)
    return b if setup.fwhm is None else blur(b, setup.fwhm)


P1_FLOOR = 1e-6  # of the smallest voxel size: below it a LOR misses the image


def p1_floor(geom: "Geometry") -> float:
    """The (P^LM 1)_e at or below which S_e = 0 (see the readings above)."""
    return P1_FLOOR * float(min(geom.h))


def step_S(P1: np.ndarray, gamma: float, rho: float, p1_min: float) -> np.ndarray:
    """S_e = gamma rho / (P^LM 1)_e where (P^LM 1)_e > p1_min, else 0
    (Eq. lm_stepsizes)."""
    P1 = np.asarray(P1, dtype=np.float64)
    on = P1 > p1_min
    return np.where(on, gamma * rho / np.where(on, P1, 1.0), 0.0)


def lm_setup(geom: Geometry, events, n_subsets: int, g: np.ndarray, gamma: float,
             rho: float, knorm: Optional[float] = None, xi: Optional[np.ndarray] = None,
             m: Optional[np.ndarray] = None, fwhm: Optional[Sequence[float]] = None) -> LMSetup:
    """Event counts, subsets and step sizes (Algorithm 2, preprocessing;
    Eq. lm_stepsizes).  m: per-event multiplicative factors of the forward
    model (attenuation times normalisation of the event's LOR), so that the
    operator is P' = diag(m) P^LM; fwhm: the resolution model B, P^LM = G B
    with G the projector; g must be the sensitivity of the whole operator."""
    ev = _ev(events)
    mu = event_counts(ev, geom.n_cry)
    sub = subset_ids(len(ev), n_subsets)
    subsets = [np.nonzero(sub == i)[0] for i in range(n_subsets)]
    P1 = fwd(geom, np.ones(geom.shape) if fwhm is None else blur(np.ones(geom.shape), fwhm), ev)
    if m is not None:
        P1 = np.asarray(m, dtype=np.float64) * P1
    S = step_S(P1, gamma, rho, p1_floor(geom))
    kn = grad_norm(geom.shape) if (knorm is None or knorm <= 0) else float(knorm)
    T = rho / (2.0 * gamma * np.maximum(g, kn))
    return LMSetup(mu=mu, subsets=subsets, S=S, S_prior=gamma * rho / kn, T=T, g=g, knorm=kn, xi=xi,
                   m=None if m is None else np.asarray(m, dtype=np.float64),
                   fwhm=None if fwhm is None else tuple(float(f) for f in fwhm))


def lm_init(geom: Geometry, events, s: np.ndarray, setup: LMSetup, x0: np.ndarray) -> LMState:
    """Initialisation of Algorithm 2: y = 1 - mu / (P^LM x + s); w = 0;
    z = zbar = g + P^LM^T((y-1)/mu) + K^T w (with the sign reading described
    in the module doc)."""
    ev = _ev(events)
    x = np.array(x0, dtype=np.float64).reshape(geom.shape)
    m = np.ones(len(ev)) if setup.m is None else setup.m
    y = 1.0 - setup.mu / (_fwd_model(geom, setup, x, ev, m) + s)
    w = np.zeros((3,) + geom.shape)
    z = setup.g + _back_model(geom, setup, (y - 1.0) / setup.mu, ev, m) + k_adj(w, setup.xi)
    return LMState(x=x, z=z, zbar=z.copy(), w=w, y=y, u=0)


def lm_update(geom: Geometry, events, s: np.ndarray, setup: LMSetup, st: LMState,
              i: int, n_subsets: int, beta: float) -> LMState:
    """One update of Algorithm 2 (primal step, one dual branch, z and zbar)
    with the subset choice i given."""
    ev = _ev(events)
    st.x = np.maximum(0.0, st.x - setup.T * st.zbar)
    if i < n_subsets:
        e = setup.subsets[i]
        me = 1.0 if setup.m is None else setup.m[e]
        q = _fwd_model(geom, setup, st.x, ev[e], me) + s[e]
        a = st.y[e] + setup.S[e] * q
        yp = prox_poisson_dual(a, setup.S[e], setup.mu[e])
        dz = _back_model(geom, setup, (yp - st.y[e]) / setup.mu[e], ev[e], me)
        st.y[e] = yp
        p = 1.0 / (2.0 * n_subsets)
    else:
        v = st.w + setup.S_prior * k_op(st.x, setup.xi)
        wp = prox_tv_dual(v, beta)
        dz = k_adj(wp - st.w, setup.xi)
        st.w = wp
        p = 0.5
    st.z = st.z + dz
    st.zbar = st.z + dz / p
    st.u += 1
    return st


def lm_spdhg(geom: Geometry, events, s: np.ndarray, g: np.ndarray, x0: np.ndarray,
             n_subsets: int, seq: Sequence[int], gamma: float, rho: float, beta: float,
             knorm: Optional[float] = None, state: Optional[LMState] = None,
             setup: Optional[LMSetup] = None,
             callback: Optional[Callable[[LMState, LMSetup], None]] = None,
             xi: Optional[np.ndarray] = None, m: Optional[np.ndarray] = None,
             fwhm: Optional[Sequence[float]] = None):
    """Run the updates listed in ``seq`` (each entry a subset index, or
    n_subsets for the prior) and return (x, state, setup).  x is the image of
    the last x-update (the value Algorithm 2 returns)."""
    s = np.asarray(s, dtype=np.float64)
    if setup is None:
        setup = lm_setup(geom, events, n_subsets, np.asarray(g, dtype=np.float64), gamma, rho, knorm, xi, m, fwhm)
    if state is None:
        state = lm_init(geom, events, s, setup, x0)
    for i in seq:
        lm_update(geom, events, s, setup, state, int(i), n_subsets, beta)
        if callback is not None:
            callback(state, setup)
    return state.x, state, setup


# --------------------------------------------------------------------------
# sinogram SPDHG (Algorithm 1) on a dense system matrix, with the y
# initialisation of Eq. (yinit); used only to check LM-SPDHG on tiny problems


def spdhg_sino(P: np.ndarray, d: np.ndarray, s: np.ndarray, x0: np.ndarray, bins_of_subset,
               seq, gamma: float, rho: float, beta: float, shape_zyx,
               T: Optional[np.ndarray] = None, knorm: Optional[float] = None,
               xi: Optional[np.ndarray] = None, p1_min: float = 0.0):
    """P: [m, nvox] rows of the TOF sinogram operator; d: counts per bin;
    bins_of_subset: list of bin-index arrays; T: primal step, by default the
    preconditioned rule of Algorithm 1, T = min_k T_k with
    T_k = rho p_k / (gamma P_k^T 1) and T_prior = rho p_prior / (gamma ||K||),
    p_k = 1/(2n), p_prior = 1/2; p1_min: S is 0 for bins with P 1 at or
    below it (p1_floor of the geometry, as in lm_setup); returns x after
    the updates."""
    n = len(bins_of_subset)
    kn = grad_norm(shape_zyx) if (knorm is None or knorm <= 0) else float(knorm)
    P1 = P.sum(axis=1)
    S = step_S(P1, gamma, rho, p1_min)
    S_prior = gamma * rho / kn
    if T is None:
        Tk = [rho * (1.0 / (2 * n)) / (gamma * P[b].sum(axis=0)) for b in bins_of_subset]
        T = np.minimum(np.min(np.stack(Tk), axis=0), rho * 0.5 / (gamma * kn))
    x = np.array(x0, dtype=np.float64).reshape(-1)
    y = 1.0 - d / (P @ x + s)
    w = np.zeros((3,) + tuple(shape_zyx))
    z = P.T @ y + k_adj(w, xi).reshape(-1)
    zbar = z.copy()
    Tf = np.asarray(T, dtype=np.float64).reshape(-1)
    for i in seq:
        x = np.maximum(0.0, x - Tf * zbar)
        if i < n:
            b = bins_of_subset[i]
            a = y[b] + S[b] * (P[b] @ x + s[b])
            yp = prox_poisson_dual(a, S[b], d[b])
            dz = P[b].T @ (yp - y[b])
            y[b] = yp
            p = 1.0 / (2.0 * n)
        else:
            v = w + S_prior * k_op(x.reshape(shape_zyx), xi)
            wp = prox_tv_dual(v, beta)
            dz = k_adj(wp - w, xi).reshape(-1)
            w = wp
            p = 0.5
        z = z + dz
        zbar = z + dz / p
    return x.reshape(shape_zyx)


# --------------------------------------------------------------------------
# warm start: listmode EM-TV (Algorithm 3), each subset update an EM step
# followed by a weighted TV denoising problem solved by the accelerated
# primal-dual algorithm of Chambolle & Pock (J. Math. Imaging Vis. 40, 2011,
# their Algorithm 2).
#
# Readings taken where the paper is silent:
# * the EM step's quotient is 1 / (P^LM x + s); an event with P^LM x + s = 0
#   adds nothing, and z = 0 where g = 0;
# * w = g / (beta x) is infinite where x = 0: such voxels keep u = z (= 0,
#   since z is proportional to x); beta = 0 skips the denoising (x = z, OSEM);
# * subsets are the interleaved ones of LM-SPDHG, visited in the order
#   0, 1, ..., n-1 in every iteration;
# * the denoising starts from u = z with a zero dual, tau_0 = sigma_0 =
#   1/||K||, and takes the uniform convexity constant as the smallest finite
#   weight.


def em_step(geom: Geometry, x: np.ndarray, events, s: np.ndarray, g: np.ndarray, n_subsets: int) -> np.ndarray:
    """Subset EM step of Algorithm 3 for the events (and s) of one subset:
    z = x n / g * P^LM^T (1 / (P^LM x + s))."""
    x = np.asarray(x, dtype=np.float64)
    q = fwd(geom, x, events) + np.asarray(s, dtype=np.float64)
    v = np.where(q > 0, 1.0 / np.where(q > 0, q, 1.0), 0.0)
    bp = back(geom, v, events)
    return np.where(g > 0, x * n_subsets * bp / np.where(g > 0, g, 1.0), 0.0)


def emtv_weights(g: np.ndarray, x: np.ndarray, beta: float) -> np.ndarray:
    """w = g / (beta x) of Algorithm 3 (inf where x = 0)."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(x > 0, g / (beta * np.where(x > 0, x, 1.0)), np.inf)


def weighted_tv_denoise(z: np.ndarray, w: np.ndarray, n_iter: int, return_dual: bool = False):
    """argmin_{u >= 0} sum_j w_j / 2 (u_j - z_j)^2 + ||K u||_{2,1} by n_iter
    steps of accelerated PDHG: with G(u) the weighted quadratic plus the
    constraint and F = ||.||_{2,1},
        q     <- projection of q + sigma K ubar onto the unit balls,
        u+    <- prox_{tau G}(u - tau K^T q),
        theta  = 1 / sqrt(1 + 2 gam tau), tau <- theta tau, sigma <- sigma / theta,
        ubar  <- u+ + theta (u+ - u).
    prox_{tau G}(v) = max(0, (v + tau w z) / (1 + tau w)), and u = z where w
    is infinite.  Returns u (and the dual q)."""
    z = np.asarray(z, dtype=np.float64)
    fixed = np.isinf(w)
    wf = np.where(fixed, 0.0, w)
    gam = float(w[~fixed].min()) if np.any(~fixed) else 0.0
    tau = sigma = 1.0 / grad_norm(z.shape)
    u = z.copy()
    ubar = z.copy()
    q = np.zeros((3,) + z.shape)
    for _ in range(n_iter):
        q = prox_tv_dual(q + sigma * grad(ubar), 1.0)
        v = u - tau * grad_adjoint(q)
        up = np.where(fixed, z, np.maximum(0.0, (v + tau * wf * z) / (1.0 + tau * wf)))
        theta = 1.0 / np.sqrt(1.0 + 2.0 * gam * tau)
        tau, sigma = theta * tau, sigma / theta
        ubar = up + theta * (up - u)
        u = up
    return (u, q) if return_dual else u


def emtv(geom: Geometry, events, s: np.ndarray, g: np.ndarray, x0: np.ndarray, n_subsets: int, n_iter: int,
         beta: float, denoise_iter: int = 20) -> np.ndarray:
    """Listmode EM-TV (Algorithm 3): n_iter passes over the n_subsets
    interleaved subsets; each subset update is the EM step, the weights
    w = g / (beta x) and the weighted TV denoising from the EM image."""
    ev = _ev(events)
    s = np.asarray(s, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    x = np.array(x0, dtype=np.float64)
    sub = subset_ids(len(ev), n_subsets)
    for _ in range(n_iter):
        for i in range(n_subsets):
            m = sub == i
            z = em_step(geom, x, ev[m], s[m], g, n_subsets)
            x = z if beta <= 0 else weighted_tv_denoise(z, emtv_weights(g, x, beta), denoise_iter)
    return x
