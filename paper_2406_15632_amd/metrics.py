"""Image comparison norms and time-to-error interpolation (host side).

* integral norm dI = (I - I_ref) / I_ref of the total intensity (Sec. 4.1);
* image norm Delta I / I = sum|A - B| / sum(|A + B| / 2) over pixels (Sec. 4.2),
  the same for Q and U;
* relative image RMS error ||A - B||_2 / ||B||_2 over the pixels of I, the
  error the time-to-error comparisons use;
* time to reach a target error, read off a (time, error) curve by log-log
  interpolation between the two bracketing measurements (Sec. 5, the
  time-to-error tables);
* least-squares power laws a t^-b of an error against time (Sec. 5).
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np


def integral_norm(I: np.ndarray, I_ref: np.ndarray) -> float:
    return float((I.sum() - I_ref.sum()) / I_ref.sum())


def image_norm(A: np.ndarray, B: np.ndarray, mask: Optional[np.ndarray] = None) -> float:
    if mask is not None:
        A, B = A[mask], B[mask]
    den = np.sum(np.abs(A + B)) / 2.0
    return float(np.sum(np.abs(A - B)) / den) if den > 0 else 0.0


def rms_error(A: np.ndarray, B: np.ndarray, mask: Optional[np.ndarray] = None) -> float:
    if mask is not None:
        A, B = A[mask], B[mask]
    nb = np.linalg.norm(B)
    return float(np.linalg.norm(A - B) / nb) if nb > 0 else 0.0


def time_to_error(times: Sequence[float], errors: Sequence[float], target: float) -> Optional[float]:
    """Time at which the error first falls to `target`, by log-log interpolation
    between consecutive points of increasing time; None if never reached, or the
    first time if the first point is already below the target."""
    pts = sorted(zip(times, errors))
    for i, (t, e) in enumerate(pts):
        if e <= target:
            if i == 0:
                return float(t)
            t0, e0 = pts[i - 1]
            if e0 <= 0 or e <= 0 or t0 <= 0 or t <= 0:
                return float(t)
            f = (math.log(target) - math.log(e0)) / (math.log(e) - math.log(e0))
            return float(math.exp(math.log(t0) + f * (math.log(t) - math.log(t0))))
    return None


def power_fit(times: Sequence[float], errors: Sequence[float], b: Optional[float] = None):
    """Least-squares fit of error = a t^-b on log-log axes (the paper's error
    approximations of Sec. 5: a t^-0.5 with b fixed, or a t^-b with both
    fitted).  Points with a non-positive time or error are left out.
    Returns (a, b), or None with fewer than two points (one when b is given)."""
    pts = [(math.log(t), math.log(e)) for t, e in zip(times, errors) if t > 0 and e > 0]
    if len(pts) < (1 if b is not None else 2):
        return None
    x = np.array([p[0] for p in pts])
    y = np.array([p[1] for p in pts])
    if b is None:
        slope, icpt = np.polyfit(x, y, 1)
        return float(math.exp(icpt)), float(-slope)
    return float(math.exp(np.mean(y + b * x))), float(b)


def central_mask(npix: int, half_width: float, radius: float) -> np.ndarray:
    """True for pixels whose centre lies outside a central circle of `radius`
    (the masked star of a sphere source)."""
    c = (np.arange(npix) + 0.5) / npix * 2 * half_width - half_width
    X, Y = np.meshgrid(c, c)
    return X * X + Y * Y > radius * radius
