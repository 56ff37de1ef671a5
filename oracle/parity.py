"""Moment parity against the oracle -- TEST INFRASTRUCTURE ONLY (used by the
tests and the benchmark's oracle leg).

Bar: |b_j - b_j_ref| <= tol * max(b0_ref, floor) per pixel and j, and exactly 0
where b0_ref = 0.  A pixel that misses it passes a backward-error bar instead
when the tested value lies within the oracle's own spread over cameras moved by
a few FP32 ulps: the library's vertex positions and the in-plane coordinates of
its side products are FP32, and a grazing ray's moments are sensitive to that
rounding (a 1e-7 change of the ray moves b0 by ~1e-7 there).
"""
from __future__ import annotations

import numpy as np

from . import render

PERTURB = 2.0 ** -21  # 4 FP32 ulps, relative


def perturbed_views(view: dict) -> list:
    """Camera frames moved by PERTURB (relative) along each axis of the eye and of the direction."""
    out = []
    for key in ("dir", "eye"):
        base = np.asarray(view[key], dtype=np.float64)
        scale = max(np.abs(base).max(), 1e-3) * PERTURB
        for k in range(3):
            for sgn in (-1.0, 1.0):
                v = dict(view)
                vec = base.copy()
                vec[k] += sgn * scale
                v[key] = tuple(vec)
                out.append(v)
    return out


def moment_parity(sc, pix, got, ref, tol=1e-5, floor=1e-3, per_sub=False, threads=None) -> dict:
    """Compare moments `got` ([m+1, P], or [S, m+1, P] with per_sub) with the oracle's `ref` (a render()
    result for the pixel indices `pix`).  Returns the forward error, the pixels that needed the backward
    bar, and how many of those lie outside the band (0 when parity holds)."""
    key = "moments_sub" if per_sub else "moments"
    b0 = ref["moments"][0]
    bg = b0 == 0
    background_exact = bool(np.all(got[..., bg] == 0.0))
    den = np.maximum(b0, floor)
    diff = np.abs(got - ref[key]) / den
    diff[..., bg] = 0.0
    per_pix = diff.reshape(-1, diff.shape[-1]).max(axis=0)
    bad = np.where(per_pix > tol)[0]
    outside = 0
    if len(bad):
        lo = ref[key][..., bad].copy()
        hi = lo.copy()
        for v in perturbed_views(sc.view):
            sc2 = type(sc)(**{**sc.__dict__, "view": v})
            rr = render(sc2, pixels=np.asarray(pix)[bad], pass2=False, per_sub=per_sub, threads=threads)
            lo = np.minimum(lo, rr[key])
            hi = np.maximum(hi, rr[key])
        g = got[..., bad]
        slack = tol * den[bad]
        ok = (g >= lo - slack) & (g <= hi + slack)
        outside = int(np.count_nonzero(~ok.reshape(-1, len(bad)).all(axis=0)))
    cov_err = per_pix[~bg] if per_pix.shape[-1] == bg.shape[-1] else per_pix
    q = np.quantile(cov_err, [0.5, 0.99, 0.999]) if cov_err.size else np.zeros(3)
    return {"covered": int(np.count_nonzero(~bg)), "background_exact": background_exact,
            "forward_max": float(per_pix.max()) if per_pix.size else 0.0,
            "forward_p50": float(q[0]), "forward_p99": float(q[1]), "forward_p999": float(q[2]),
            "backward_bar_pixels": int(len(bad)), "outside_backward_band": outside}
