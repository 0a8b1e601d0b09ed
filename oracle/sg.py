"""Oracle: environment-light prefiltering of the NDF query (Sec. 5.4), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A spherical Gaussian light lobe G(w) = A exp(lambda (cos(w) - 1)) (w the
angle to the lobe axis) is above a threshold eps exactly within its
compact-eps support angle theta = arccos((ln eps - ln A) / lambda + 1)
(Sec. 5.4, Eq. for theta).  The NDF is then averaged over a square angular
range whose side, on an NDF image of N bins spanning the projected
half-vector square [-1, 1]^2 (pi radians across), is Q = N theta / pi bins
(the paper's 256 theta / pi for its 256-bin images).

Readings:
  * the argument of arccos is clamped to [-1, 1]: a lobe that never
    exceeds eps (A < eps) has theta = 0, and one above eps everywhere has
    theta = pi; the side is capped at the whole image (2 in projected units);
  * the square is centred on the query's projected half vector h; its
    continuous extent [h - w/2, h + w/2] (w = 2 theta / pi) becomes bins
    lo = clamp(floor((h - w/2 + 1) N / 2), 0, N - 1),
    hi = clamp(floor((h + w/2 + 1) N / 2), 0, N - 1) + 1,
    so a zero-width box is the point query of the bin holding h;
  * the result is the average bin mass over the box: the range query's box
    sum divided by its number of bins.
"""
from __future__ import annotations

import math

import numpy as np

from .query import range_query

EPS_DEFAULT = 0.3


def support_angle(lam, amp, eps: float = EPS_DEFAULT):
    """Compact-eps support angle of SG lobes (radians), elementwise."""
    lam = np.asarray(lam, dtype=np.float64)
    amp = np.asarray(amp, dtype=np.float64)
    arg = (math.log(eps) - np.log(amp)) / lam + 1.0
    return np.arccos(np.clip(arg, -1.0, 1.0))


def sg_value(lam, amp, angle):
    """The lobe's value at an angle to its axis."""
    return np.asarray(amp, dtype=np.float64) * np.exp(np.asarray(lam, dtype=np.float64) * (np.cos(angle) - 1.0))


def box_bins(h, theta, nbins: int):
    """Half-open bin range [lo, hi) of the square of side N theta / pi bins
    centred on h (projected coordinates in [-1, 1]), elementwise."""
    h = np.asarray(h, dtype=np.float64)
    w = np.minimum(2.0 * np.asarray(theta, dtype=np.float64) / math.pi, 2.0)
    lo = np.floor((h - 0.5 * w + 1.0) * (nbins / 2.0)).astype(np.int64)
    hi = np.floor((h + 0.5 * w + 1.0) * (nbins / 2.0)).astype(np.int64)
    return np.clip(lo, 0, nbins - 1), np.clip(hi, 0, nbins - 1) + 1


def sg_records(uvl, h, lam, amp, nbins: int, eps: float = EPS_DEFAULT):
    """Query records (u, v, l, s_lo, s_hi, t_lo, t_hi) of SG-prefiltered
    lookups: h [n][2] projected half vectors, lam/amp [n] the chosen lobe."""
    uvl = np.asarray(uvl, dtype=np.int64)
    h = np.asarray(h, dtype=np.float64)
    theta = support_angle(lam, amp, eps)
    slo, shi = box_bins(h[:, 0], theta, nbins)
    tlo, thi = box_bins(h[:, 1], theta, nbins)
    return np.stack([uvl[:, 0], uvl[:, 1], uvl[:, 2], slo, shi, tlo, thi], axis=1)


def query_sg(U, V, L, CS, CT, uvl, h, lam, amp, eps: float = EPS_DEFAULT):
    """Average bin mass of the NDF over each lookup's SG box, and the records."""
    nbins = CS.shape[0] - 1
    q = sg_records(uvl, h, lam, amp, nbins, eps)
    total = range_query(U, V, L, CS, CT, q)
    area = (q[:, 4] - q[:, 3]) * (q[:, 6] - q[:, 5])
    return total / area, q
