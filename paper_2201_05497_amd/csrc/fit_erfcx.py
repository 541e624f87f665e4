"""Coefficients of the polynomial the projector uses for erfc (lm_device.hpp,
erfc_fit): erfcx(x) = exp(x^2) erfc(x) on 0 <= x <= 6 as a polynomial of
degree 9 in t = 1 / (1 + x/2), fitted here by iteratively reweighted least
squares on the relative error (toward the minimax fit), against scipy's
erfcx.  Prints the coefficients (lowest degree first), the relative error of
the fit in double precision and of a float32 evaluation that mirrors the
device code (compensated exponent), against erfc of the float32 argument.

Run: python paper_2201_05497_amd/csrc/fit_erfcx.py
"""
import numpy as np
from scipy.special import erfc, erfcx

X_MAX, DEGREE = 6.0, 9
f32 = np.float32


def fit(x_max: float = X_MAX, degree: int = DEGREE, npts: int = 40001):
    x = np.linspace(0.0, x_max, npts)
    t = 1.0 / (1.0 + 0.5 * x)
    g = erfcx(x)
    V = np.vander(t, degree + 1, increasing=True)
    w = 1.0 / g
    best = (np.inf, None)
    for _ in range(60):
        c, *_ = np.linalg.lstsq(V * w[:, None], g * w, rcond=None)
        r = (V @ c - g) / g
        if np.abs(r).max() < best[0]:
            best = (np.abs(r).max(), c)
        w = w * (1.0 + 20.0 * np.abs(r) / np.abs(r).max())
        w /= w.mean()
    return best[1], best[0]


def eval_f32(c, x):
    """float32 evaluation in the order of the device code."""
    x = x.astype(f32)
    t = (f32(1) / (f32(0.5) * np.minimum(x, f32(X_MAX)) + f32(1))).astype(f32)
    c = c.astype(f32)
    p = np.full_like(t, c[-1])
    for k in range(len(c) - 2, -1, -1):
        p = (p * t + c[k]).astype(f32)
    hi = (x * x).astype(f32)
    lo = (x.astype(np.float64) ** 2 - hi).astype(f32)
    l2e = 1.4426950408889634
    lh = f32(l2e)
    ll = f32(l2e - float(lh))
    a = (hi * lh).astype(f32)
    da = (hi.astype(np.float64) * float(lh) - a).astype(f32)
    da = (da + (hi * ll + lo * lh).astype(f32)).astype(f32)
    e = np.exp2(-a.astype(np.float64)).astype(f32)
    e = (e * (f32(1) - (da * f32(np.log(2.0))).astype(f32))).astype(f32)
    return (p * e).astype(f32)


if __name__ == "__main__":
    c, err = fit()
    x = np.linspace(0.0, X_MAX, 200001)
    xr = x.astype(f32).astype(np.float64)
    r32 = np.abs(eval_f32(c, x).astype(np.float64) - erfc(xr)) / erfc(xr)
    print("coefficients:", ", ".join(f"{v:.9e}f" for v in c))
    print(f"relative error: fit {err:.2e}, float32 evaluation {r32.max():.2e}")
