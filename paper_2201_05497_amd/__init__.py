"""MI355X (gfx950) listmode SPDHG: Python binding of liblmspdhg.so.

Every function here only marshals arguments into the C ABI declared in
``include/lmspdhg.h``; all arithmetic runs in the library's HIP kernels.
PyTorch supplies device memory (tensors) and streams (the current stream
of the tensors' device).  There is no CPU fallback: importing the package
without the built library raises.

Paper: listmode SPDHG (LM-SPDHG, Algorithm 2) for the Poisson problem of
Eq. (1) with a time-of-flight Joseph projector and a TV prior.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import LMError

__all__ = ["Geometry", "lm_fwd", "lm_back", "lm_sens", "lm_validate_events", "tv_grad", "tv_div",
           "lm_cost", "lm_plan_bytes", "Plan", "lm_emtv", "LMError", "PART_DTV", "PART_FACTORS", "PART_RESOLUTION"]

_L = _lib.load()


def _stream(dev: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _need(t: torch.Tensor, dtype, name: str, device: torch.device, numel: Optional[int] = None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


class Geometry:
    """Scanner, image grid and TOF model (``lm_geom``).

    det: float32 [n_cry * n_ring, 3] crystal centres in mm (id = c + n_cry r);
    n = (nx, ny, nz); h = voxel size in mm; TOF bins of width ``tof_bin``
    (``n_tof`` odd), Gaussian FWHM ``tof_fwhm`` truncated at ``tof_nsigma``.
    Every crystal must lie outside the image box (the projector's plane
    range assumes the LOR end points are outside the image).
    """

    def __init__(self, det, n_cry: int, n_ring: int, n, h, n_tof: int, tof_bin: float,
                 tof_fwhm: float, tof_nsigma: float = 3.0, tof_on: bool = True,
                 device: str | torch.device = "cuda"):
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        det_np = np.asarray(det.cpu() if isinstance(det, torch.Tensor) else det, dtype=np.float32)
        if det_np.shape != (n_cry * n_ring, 3):
            raise ValueError(f"det must be [{n_cry * n_ring}, 3]")
        half = 0.5 * np.asarray(n, dtype=np.float64) * np.asarray(h, dtype=np.float64)
        inside = np.all(np.abs(det_np.astype(np.float64)) < half[None, :], axis=1)
        if inside.any():
            raise ValueError("a crystal lies inside the image box")
        self.det_host = det_np
        self.det = torch.as_tensor(det_np, device=self.device).contiguous()
        self.n_cry, self.n_ring = int(n_cry), int(n_ring)
        self.n = tuple(int(v) for v in n)
        self.h = tuple(float(v) for v in h)
        self.n_tof, self.tof_bin, self.tof_fwhm = int(n_tof), float(tof_bin), float(tof_fwhm)
        self.tof_nsigma, self.tof_on = float(tof_nsigma), bool(tof_on)
        self._c = _lib.LMGeom(self.det.data_ptr(), self.n_cry, self.n_ring,
                              (ctypes.c_int32 * 3)(*self.n), (ctypes.c_double * 3)(*self.h),
                              self.n_tof, self.tof_bin, self.tof_fwhm, self.tof_nsigma,
                              int(self.tof_on))

    @classmethod
    def from_problem(cls, p, tof_on: Optional[bool] = None, device="cuda") -> "Geometry":
        sc, img, tof = p.scanner, p.image, p.tof
        return cls(p.det, sc.n_cry, sc.n_ring, img.n, img.h, tof.n_tof, tof.bin, tof.fwhm,
                   tof.nsigma, tof.on if tof_on is None else tof_on, device=device)

    def with_tof(self, on: bool) -> "Geometry":
        return Geometry(self.det_host, self.n_cry, self.n_ring, self.n, self.h, self.n_tof,
                        self.tof_bin, self.tof_fwhm, self.tof_nsigma, on, self.device)

    @property
    def shape(self):
        """Image tensor shape [nz, ny, nx]."""
        return (self.n[2], self.n[1], self.n[0])

    @property
    def nvox(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def zeros(self) -> torch.Tensor:
        return torch.zeros(self.shape, dtype=torch.float32, device=self.device)

    def events(self, ev) -> torch.Tensor:
        """Events as a contiguous int16 [N, 5] tensor on this device."""
        t = torch.as_tensor(np.asarray(ev, dtype=np.int16) if not isinstance(ev, torch.Tensor) else ev)
        return t.to(device=self.device, dtype=torch.int16).contiguous()


def _ev_check(geom: Geometry, ev: torch.Tensor) -> int:
    _need(ev, torch.int16, "events", geom.device)
    if ev.dim() != 2 or ev.shape[1] != 5:
        raise ValueError("events must be [N, 5] int16")
    return ev.shape[0]


def lm_fwd(geom: Geometry, x: torch.Tensor, ev: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """(P^LM x)_e for every event (Eq. lmop)."""
    n = _ev_check(geom, ev)
    _need(x, torch.float32, "x", geom.device, geom.nvox)
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=geom.device)
    _need(out, torch.float32, "out", geom.device, n)
    _lib.check(_L.lm_fwd(ctypes.byref(geom._c), x.data_ptr(), ev.data_ptr(), n, out.data_ptr(),
                         _stream(geom.device)), "lm_fwd")
    return out


def lm_back(geom: Geometry, v: torch.Tensor, ev: torch.Tensor, img: Optional[torch.Tensor] = None) -> torch.Tensor:
    """img += (P^LM)^T v (img is zeroed first when not given)."""
    n = _ev_check(geom, ev)
    _need(v, torch.float32, "v", geom.device, n)
    if img is None:
        img = geom.zeros()
    _need(img, torch.float32, "img", geom.device, geom.nvox)
    _lib.check(_L.lm_back(ctypes.byref(geom._c), v.data_ptr(), ev.data_ptr(), n, img.data_ptr(),
                          _stream(geom.device)), "lm_back")
    return img


def lm_sens(geom: Geometry, g: Optional[torch.Tensor] = None) -> torch.Tensor:
    """g += P^T 1 over every crystal pair and TOF bin (zeroed when not given)."""
    if g is None:
        g = geom.zeros()
    _need(g, torch.float32, "g", geom.device, geom.nvox)
    _lib.check(_L.lm_sens(ctypes.byref(geom._c), g.data_ptr(), _stream(geom.device)), "lm_sens")
    return g


def lm_validate_events(geom: Geometry, ev: torch.Tensor) -> int:
    """Number of events with an out-of-range crystal, ring or TOF index."""
    n = _ev_check(geom, ev)
    bad = ctypes.c_int64(0)
    _lib.check(_L.lm_validate_events(ctypes.byref(geom._c), ev.data_ptr(), n, ctypes.byref(bad),
                                     _stream(geom.device)), "lm_validate_events")
    return int(bad.value)


def _dims(x: torch.Tensor):
    if x.dim() != 3:
        raise ValueError("image must be [nz, ny, nx]")
    nz, ny, nx = x.shape
    return (ctypes.c_int32 * 3)(nx, ny, nz)


def tv_grad(x: torch.Tensor, gx: Optional[torch.Tensor] = None) -> torch.Tensor:
    """K x, forward differences, as [3, nz, ny, nx] (component 0 = x)."""
    _need(x, torch.float32, "x", x.device)
    if gx is None:
        gx = torch.empty((3,) + tuple(x.shape), dtype=torch.float32, device=x.device)
    _need(gx, torch.float32, "gx", x.device, 3 * x.numel())
    _lib.check(_L.tv_grad(_dims(x), x.data_ptr(), gx.data_ptr(), _stream(x.device)), "tv_grad")
    return gx


def tv_div(w: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """div w = -K^T w for w of shape [3, nz, ny, nx]."""
    _need(w, torch.float32, "w", w.device)
    if w.dim() != 4 or w.shape[0] != 3:
        raise ValueError("w must be [3, nz, ny, nx]")
    if out is None:
        out = torch.empty(tuple(w.shape[1:]), dtype=torch.float32, device=w.device)
    _need(out, torch.float32, "out", w.device, w[0].numel())
    _lib.check(_L.tv_div(_dims(out), w.data_ptr(), out.data_ptr(), _stream(w.device)), "tv_div")
    return out


def lm_emtv(geom: Geometry, ev: torch.Tensor, s: torch.Tensor, g: torch.Tensor, x: torch.Tensor, n_subsets: int,
            n_iter: int = 1, beta: float = 0.0, denoise_iter: int = 20) -> torch.Tensor:
    """Listmode EM-TV (Algorithm 3), the warm start of LM-SPDHG: n_iter
    passes over the n_subsets interleaved subsets, each an EM step and, for
    beta > 0, a weighted TV denoising by denoise_iter accelerated PDHG
    steps.  x (x0 >= 0) is updated in place and returned."""
    n = _ev_check(geom, ev)
    _need(s, torch.float32, "s", geom.device, n)
    _need(g, torch.float32, "g", geom.device, geom.nvox)
    _need(x, torch.float32, "x", geom.device, geom.nvox)
    _lib.check(_L.lm_emtv(ctypes.byref(geom._c), ev.data_ptr(), s.data_ptr(), n, int(n_subsets), int(n_iter),
                          g.data_ptr(), float(beta), int(denoise_iter), x.data_ptr(), _stream(geom.device)),
               "lm_emtv")
    return x


def lm_cost(geom: Geometry, x: torch.Tensor, ev: torch.Tensor, s: torch.Tensor, g: torch.Tensor,
            beta: float) -> tuple:
    """(c(x), (<g, x>, sum_e log((P^LM x)_e + s_e), ||K x||_{2,1})): the
    listmode form of the objective of Eq. (1) without the constant sum of s
    over all bins (synchronous)."""
    n = _ev_check(geom, ev)
    _need(x, torch.float32, "x", geom.device, geom.nvox)
    _need(g, torch.float32, "g", geom.device, geom.nvox)
    _need(s, torch.float32, "s", geom.device, n)
    c = ctypes.c_double(0.0)
    t = (ctypes.c_double * 3)()
    _lib.check(_L.lm_cost(ctypes.byref(geom._c), x.data_ptr(), ev.data_ptr(), s.data_ptr(), n, g.data_ptr(),
                          float(beta), ctypes.byref(c), t, _stream(geom.device)), "lm_cost")
    return float(c.value), (float(t[0]), float(t[1]), float(t[2]))


# optional parts of a plan, for lm_plan_bytes(parts=...)
PART_DTV, PART_FACTORS, PART_RESOLUTION = 1, 2, 4


def lm_plan_bytes(geom: Geometry, n_events: int, n_subsets: int, parts: int = 0) -> int:
    """Device bytes a plan allocates (used for admission against a budget),
    with the optional parts in `parts` (an OR of PART_*)."""
    b = ctypes.c_size_t(0)
    _lib.check(_L.lm_plan_bytes_ex(ctypes.byref(geom._c), int(n_events), int(n_subsets), int(parts),
                                   ctypes.byref(b)), "lm_plan_bytes_ex")
    return int(b.value)


class Plan:
    """An LM-SPDHG reconstruction resident on the GPU (``lm_plan``).

    ``Plan(geom, events, s, n_subsets, gamma, rho, beta, g=None, knorm=0)``
    runs the preprocessing (event counts, subsets, step sizes; g = P^T 1 is
    computed with lm_sens when not given).  ``init(x0)`` initialises y, z,
    zbar, w; ``epoch(x, seq)`` runs the updates listed in ``seq`` (each a
    subset index, or n_subsets for the prior), updating x in place.
    """

    def __init__(self, geom: Geometry, ev: torch.Tensor, s: torch.Tensor, n_subsets: int, gamma: float,
                 rho: float = 0.999, beta: float = 0.0, g: Optional[torch.Tensor] = None, knorm: float = 0.0):
        self.geom = geom
        n = _ev_check(geom, ev)
        _need(s, torch.float32, "s", geom.device, n)
        if g is not None:
            _need(g, torch.float32, "g", geom.device, geom.nvox)
        self.n_events, self.n_subsets = n, int(n_subsets)
        self.gamma, self.rho, self.beta = float(gamma), float(rho), float(beta)
        h = ctypes.c_void_p(None)
        _lib.check(_L.lm_plan_create(ctypes.byref(geom._c), ev.data_ptr(), s.data_ptr(), n, self.n_subsets,
                                     _ptr(g), self.gamma, self.rho, self.beta, float(knorm),
                                     _stream(geom.device), ctypes.byref(h)), "lm_plan_create")
        self._h = h

    def _handle(self):
        if self._h is None or self._h.value is None:
            raise RuntimeError("plan destroyed")
        return self._h

    def init(self, x0: torch.Tensor) -> None:
        _need(x0, torch.float32, "x0", self.geom.device, self.geom.nvox)
        _lib.check(_L.lm_spdhg_init(self._handle(), x0.data_ptr(), _stream(self.geom.device)), "lm_spdhg_init")

    def epoch(self, x: torch.Tensor, seq) -> torch.Tensor:
        _need(x, torch.float32, "x", self.geom.device, self.geom.nvox)
        sq = np.ascontiguousarray(np.asarray(seq, dtype=np.int32))
        _lib.check(_L.lm_spdhg_epoch(self._handle(), x.data_ptr(),
                                     sq.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(sq),
                                     _stream(self.geom.device)), "lm_spdhg_epoch")
        return x

    def set_event_factors(self, m: torch.Tensor) -> None:
        """Per-event multiplicative factors (attenuation x normalisation of
        each event's LOR): the operator becomes diag(m) P.  Once, before
        init; g must be the sensitivity of that operator."""
        _need(m, torch.float32, "m", self.geom.device, self.n_events)
        _lib.check(_L.lm_plan_set_event_factors(self._handle(), m.data_ptr(), _stream(self.geom.device)),
                   "lm_plan_set_event_factors")

    def set_resolution(self, fwhm_vox) -> None:
        """Image-space resolution model: the operator becomes G B with B a
        separable Gaussian of FWHM fwhm_vox = (fx, fy, fz) voxels.  Before
        init; g must be the sensitivity of G B."""
        f = (ctypes.c_double * 3)(*[float(v) for v in fwhm_vox])
        _lib.check(_L.lm_plan_set_resolution(self._handle(), f, _stream(self.geom.device)), "lm_plan_set_resolution")

    def set_prior_image(self, v: Optional[torch.Tensor], eta: float = 0.0) -> None:
        """Directional TV: later prior updates use K = D grad with the
        normalised gradient of the prior image v (eta > 0); None: TV."""
        if v is not None:
            _need(v, torch.float32, "v", self.geom.device, self.geom.nvox)
        _lib.check(_L.lm_plan_set_prior_image(self._handle(), _ptr(v), float(eta), _stream(self.geom.device)),
                   "lm_plan_set_prior_image")

    def lists(self):
        """(y, mu, subset, P^LM 1) per event in the caller's order."""
        n, dev = self.n_events, self.geom.device
        y = torch.empty(n, dtype=torch.float32, device=dev)
        mu = torch.empty(n, dtype=torch.int32, device=dev)
        sub = torch.empty(n, dtype=torch.int32, device=dev)
        p1 = torch.empty(n, dtype=torch.float32, device=dev)
        _lib.check(_L.lm_plan_get_lists(self._handle(), y.data_ptr(), mu.data_ptr(), sub.data_ptr(),
                                        p1.data_ptr(), _stream(dev)), "lm_plan_get_lists")
        return y, mu, sub, p1

    def layout(self):
        n, dev = self.n_events, self.geom.device
        perm = torch.empty(n, dtype=torch.int32, device=dev)
        off = torch.empty(self.n_subsets + 1, dtype=torch.int32, device=dev)
        _lib.check(_L.lm_plan_get_layout(self._handle(), perm.data_ptr(), off.data_ptr(), _stream(dev)),
                   "lm_plan_get_layout")
        return perm, off

    def images(self):
        """(g, T): sensitivity image and primal step size."""
        g, T = self.geom.zeros(), self.geom.zeros()
        _lib.check(_L.lm_plan_get_images(self._handle(), g.data_ptr(), T.data_ptr(), _stream(self.geom.device)),
                   "lm_plan_get_images")
        return g, T

    def get_state(self):
        """Checkpoint: z, zbar, w, c = 1 - y (caller event order) and the
        update counter u."""
        dev = self.geom.device
        z, zbar = self.geom.zeros(), self.geom.zeros()
        w = torch.zeros((3,) + self.geom.shape, dtype=torch.float32, device=dev)
        c = torch.empty(self.n_events, dtype=torch.float32, device=dev)
        u = ctypes.c_int64(0)
        _lib.check(_L.lm_plan_get_state(self._handle(), z.data_ptr(), zbar.data_ptr(), w.data_ptr(), c.data_ptr(),
                                        ctypes.byref(u), _stream(dev)), "lm_plan_get_state")
        return {"z": z, "zbar": zbar, "w": w, "c": c, "u": int(u.value)}

    def set_state(self, st) -> None:
        dev = self.geom.device
        for k in ("z", "zbar"):
            _need(st[k], torch.float32, k, dev, self.geom.nvox)
        _need(st["w"], torch.float32, "w", dev, 3 * self.geom.nvox)
        _need(st["c"], torch.float32, "c", dev, self.n_events)
        _lib.check(_L.lm_plan_set_state(self._handle(), st["z"].data_ptr(), st["zbar"].data_ptr(),
                                        st["w"].data_ptr(), st["c"].data_ptr(), int(st["u"]), _stream(dev)),
                   "lm_plan_set_state")

    KERNELS = ("primal", "data_update", "dual_image", "tv")

    def timing(self, every: int = 1) -> None:
        """Reset per-kernel timing of epoch() and time every ``every``-th
        launch of each kernel class (0 or False: off, True: every launch)."""
        _lib.check(_L.lm_plan_timing(self._handle(), int(every)), "lm_plan_timing")

    def set_tracing(self, on: bool = True) -> None:
        """roctx ranges per epoch() call and per update (lm_plan_set_tracing)."""
        _lib.check(_L.lm_plan_set_tracing(self._handle(), int(bool(on))), "lm_plan_set_tracing")

    def get_timing(self):
        """{kernel: (total ms, timed launches)} since the last reset (synchronises)."""
        ms = (ctypes.c_double * len(self.KERNELS))()
        n = (ctypes.c_int64 * len(self.KERNELS))()
        _lib.check(_L.lm_plan_get_timing(self._handle(), ms, n), "lm_plan_get_timing")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(self.KERNELS)}

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value is not None:
            _lib.check(_L.lm_plan_destroy(self._h), "lm_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()
