"""torch.autograd.Function over the listmode projector.

``LMProject.apply(x, geom, events, offsets)`` projects a batch of F frames:
x is [F, nz, ny, nx] (or one image [nz, ny, nx]), the events of all frames
are concatenated in ``events`` (int16 [N, 5]) with frame f owning rows
offsets[f]:offsets[f+1] (host integers), and the result is the
concatenation of (P^LM x_f)_e over frames (the paper's listmode operator,
Eq. lmop).  The backward pass is the adjoint, computed by lm_back from the
incoming gradient: d loss / d x_f = (P^LM)^T (d loss / d out_f).

Used with ``loss = <g, x> - sum log(LMProject(x) + s)``, the listmode Poisson
negative log-likelihood of Eq. (1) up to a constant, the gradient is
g - (P^LM)^T (1 / (P^LM x + s)).
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import Geometry, lm_back, lm_fwd

__all__ = ["LMProject", "poisson_nll"]


def _offsets(events: torch.Tensor, offsets: Optional[Sequence[int]], frames: int):
    if offsets is None:
        if frames != 1:
            raise ValueError("offsets are required for more than one frame")
        return [0, int(events.shape[0])]
    off = [int(v) for v in offsets]
    if len(off) != frames + 1 or off[0] != 0 or off[-1] != int(events.shape[0]) or any(
            b < a for a, b in zip(off, off[1:])):
        raise ValueError("offsets must be non-decreasing, start at 0, end at N, one more than frames")
    return off


class LMProject(torch.autograd.Function):
    """Listmode forward projection with the adjoint as its backward pass."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, geom: Geometry, events: torch.Tensor, offsets=None):
        single = x.dim() == 3
        xb = x.unsqueeze(0) if single else x
        if xb.dim() != 4 or tuple(xb.shape[1:]) != geom.shape:
            raise ValueError(f"x must be [F, {geom.shape}] or {geom.shape}")
        off = _offsets(events, offsets, xb.shape[0])
        xb = xb.detach().to(torch.float32).contiguous()
        out = torch.empty(int(events.shape[0]), dtype=torch.float32, device=x.device)
        for f in range(xb.shape[0]):
            a, b = off[f], off[f + 1]
            if b > a:
                lm_fwd(geom, xb[f], events[a:b], out[a:b])
        ctx.geom, ctx.off, ctx.single = geom, off, single
        ctx.save_for_backward(events)
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (events,) = ctx.saved_tensors
        geom, off = ctx.geom, ctx.off
        frames = len(off) - 1
        gx = torch.zeros((frames,) + geom.shape, dtype=torch.float32, device=grad_out.device)
        go = grad_out.detach().to(torch.float32).contiguous()
        for f in range(frames):
            a, b = off[f], off[f + 1]
            if b > a:
                lm_back(geom, go[a:b], events[a:b], gx[f])
        return (gx[0] if ctx.single else gx), None, None, None


def poisson_nll(x: torch.Tensor, geom: Geometry, events: torch.Tensor, s: torch.Tensor, g: torch.Tensor,
                offsets=None) -> torch.Tensor:
    """Listmode Poisson negative log-likelihood of Eq. (1) without its
    constant (the sum of s over all bins): sum_f <g, x_f> - sum_e log((P^LM x)_e + s_e),
    accumulated in float64."""
    q = LMProject.apply(x, geom, events, offsets) + s
    return (g.double() * x.double()).sum() - torch.log(q.double()).sum()
