"""Oracle: NDF bin masses, brute-force NDF tensor and range integral (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed (Sec. 3.1, Eq. geom; Sec. 4.1):
  The P-NDF of a footprint is the footprint-weighted sum, over texels, of a
  2D Gaussian of standard deviation sigma centred on each texel's projected
  normal.  Integrating it over an NDF bin factorises per axis, so a texel
  with projected normal (n_x, n_y) puts mass m_x[s] * m_y[t] into bin (s, t):

      m_x[i] = P(e_i < n_x + sigma * Z < e_{i+1}) / Zn(n_x),
      e_i    = -1 + i * (2 / N),   Zn(n) = P(-1 < n + sigma * Z < 1),

  with Z a standard normal.

Readings where the paper is silent:
  * Footprint: a box of side k = 2^l texels anchored at u - floor(k/2),
    wrapping toroidally, uniform weight 1/k^2 (the paper uses a Gaussian
    footprint on a sparse grid; here every texel is a centre).
  * Mass outside [-1, 1]^2 is renormalised away (division by Zn), so every
    texel contributes unit mass.
  * Bin index of a value on an edge goes to the upper bin:
    i0 = clamp(floor((n + 1) * N / 2), 0, N - 1) evaluated in FP64.
  * Every bin is evaluated (no truncation window).
  * A texel whose normal has a non-finite component is absent: it puts no
    mass anywhere (the footprint weight stays 1/k^2).  Wang tiles use this
    for the margin around a tile (Sec. 5.5).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

_SQRT1_2 = 1.0 / math.sqrt(2.0)


def gauss_interval(a, b):
    """P(a < Z < b) for a standard normal Z, accurate in both tails.

    Upper-tail complements are used when the interval lies right of zero and
    lower-tail ones when it lies left of zero, so that no difference of two
    numbers close to 1 is ever formed.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    right = 0.5 * (erfc(a * _SQRT1_2) - erfc(b * _SQRT1_2))        # a >= 0
    left = 0.5 * (erfc(-b * _SQRT1_2) - erfc(-a * _SQRT1_2))       # b <= 0
    mid = 1.0 - 0.5 * erfc(-a * _SQRT1_2) - 0.5 * erfc(b * _SQRT1_2)  # a < 0 < b
    out = np.where(a >= 0.0, right, np.where(b <= 0.0, left, mid))
    return np.maximum(out, 0.0)


def bin_edges(nbins: int) -> np.ndarray:
    return -1.0 + np.arange(nbins + 1, dtype=np.float64) * (2.0 / nbins)


def bin_index(n, nbins: int):
    """Centre-bin index of a projected-normal component, FP64 floor rule."""
    n = np.asarray(n, dtype=np.float64)
    i = np.floor((n + 1.0) * (nbins / 2.0)).astype(np.int64)
    return np.clip(i, 0, nbins - 1)


def axis_norm(n, sigma):
    """Zn(n): the Gaussian's mass inside [-1, 1]."""
    n = np.asarray(n, dtype=np.float64)
    return gauss_interval((-1.0 - n) / sigma, (1.0 - n) / sigma)


def axis_masses(n, nbins: int, sigma: float) -> np.ndarray:
    """Normalised bin masses for every value of ``n``: shape n.shape + (nbins,).
    A non-finite component marks an absent texel: all its masses are zero."""
    n = np.asarray(n, dtype=np.float64)[..., None]
    ok = np.isfinite(n)
    n = np.where(ok, n, 0.0)
    e = bin_edges(nbins)
    m = gauss_interval((e[:-1] - n) / sigma, (e[1:] - n) / sigma)
    return np.where(ok, m / axis_norm(n, sigma), 0.0)


def texel_masses(nxy: np.ndarray, nbins: int, sigma: float):
    """Per-texel masses along s (from n_x) and t (from n_y): two [nu][nv][N] arrays."""
    nxy = np.asarray(nxy, dtype=np.float64)
    return axis_masses(nxy[..., 0], nbins, sigma), axis_masses(nxy[..., 1], nbins, sigma)


def footprint_offsets(k: int) -> np.ndarray:
    """Texel offsets of a k-wide footprint relative to its centre index."""
    return np.arange(k) - k // 2


def ndf_bruteforce(nxy: np.ndarray, nbins: int, sigma: float, nlevels: int) -> np.ndarray:
    """T[u, v, l, s, t] by iterating every texel of every footprint (FP64).

    For each level the footprint's k^2 texels are visited one offset at a time;
    each visit adds the texel's outer product m_s (x) m_t to every centre.
    """
    ms, mt = texel_masses(nxy, nbins, sigma)
    nu, nv = nxy.shape[:2]
    T = np.zeros((nu, nv, nlevels, nbins, nbins), dtype=np.float64)
    for l in range(nlevels):
        k = 1 << l
        acc = np.zeros((nu, nv, nbins, nbins), dtype=np.float64)
        for di in footprint_offsets(k):
            ms_i = np.roll(ms, -di, axis=0)          # ms_i[u] = ms[u + di]
            mt_i = np.roll(mt, -di, axis=0)
            for dj in footprint_offsets(k):
                a = np.roll(ms_i, -dj, axis=1)       # texel (u + di, v + dj)
                b = np.roll(mt_i, -dj, axis=1)
                acc += a[:, :, :, None] * b[:, :, None, :]
        T[:, :, l] = acc / float(k * k)
    return T


def canonical_query(q: np.ndarray, nu: int, nv: int, nlevels: int, nbins: int) -> np.ndarray:
    """Apply the boundary rules to query records: wrap u, v; clamp l to the
    built levels (larger footprints clamp to the coarsest level, Sec. 5.1);
    clamp bin bounds to [0, N]."""
    q = np.asarray(q, dtype=np.int64).copy()
    q[:, 0] = np.mod(q[:, 0], nu)
    q[:, 1] = np.mod(q[:, 1], nv)
    q[:, 2] = np.clip(q[:, 2], 0, nlevels - 1)
    q[:, 3:7] = np.clip(q[:, 3:7], 0, nbins)
    return q


def range_bruteforce(nxy: np.ndarray, nbins: int, sigma: float, nlevels: int,
                     q: np.ndarray) -> np.ndarray:
    """Exact box sum of T over [s_lo, s_hi) x [t_lo, t_hi) for each query (FP64).

    Each footprint texel contributes the product of its two per-axis masses
    over the box, each a single Gaussian interval probability (the telescoped
    sum of its bin masses); the texels are summed with weight 1/k^2.
    Empty boxes (lo >= hi on either axis) give 0.
    """
    nxy = np.asarray(nxy, dtype=np.float64)
    nu, nv = nxy.shape[:2]
    q = canonical_query(q, nu, nv, nlevels, nbins)
    e = bin_edges(nbins)
    out = np.zeros(q.shape[0], dtype=np.float64)
    for i, (u, v, l, slo, shi, tlo, thi) in enumerate(q):
        if slo >= shi or tlo >= thi:
            continue
        k = 1 << int(l)
        xs = np.mod(u + footprint_offsets(k), nu)
        ys = np.mod(v + footprint_offsets(k), nv)
        n = nxy[np.ix_(xs, ys)]                       # [k][k][2]
        present = np.isfinite(n[..., 0]) & np.isfinite(n[..., 1])     # absent texels contribute 0
        nx = np.where(present, n[..., 0], 0.0)
        ny = np.where(present, n[..., 1], 0.0)
        Ms = gauss_interval((e[slo] - nx) / sigma, (e[shi] - nx) / sigma) / axis_norm(nx, sigma)
        Mt = gauss_interval((e[tlo] - ny) / sigma, (e[thi] - ny) / sigma) / axis_norm(ny, sigma)
        out[i] = float(np.sum(np.where(present, Ms * Mt, 0.0))) / float(k * k)
    return out


def box_sum(T: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Explicit sum of tensor entries over each query's box (any T[u,v,l,s,t])."""
    nu, nv, nl, ns, _ = T.shape
    q = canonical_query(q, nu, nv, nl, ns)
    out = np.zeros(q.shape[0], dtype=np.float64)
    for i, (u, v, l, slo, shi, tlo, thi) in enumerate(q):
        if slo < shi and tlo < thi:
            out[i] = float(T[u, v, l, slo:shi, tlo:thi].sum())
    return out
