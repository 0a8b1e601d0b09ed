"""Oracle: cumulative tables, point and range query, gradient (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed:
  * Point query (Sec. 4.3, Eq. decompress): one tensor entry from the
    factors, sum_r U_r[u] V_r[v] L_r[l] S_r[s] T_r[t].
  * Range query (Sec. 4.4, Eq. rangeDecom; Appendix proposition): for a
    rank-one term the box total over [s_lo, s_hi) x [t_lo, t_hi) is the product
    of the per-axis segment totals, so
        q = sum_r U_r[u] V_r[v] L_r[l] (CS_r[s_hi] - CS_r[s_lo]) (CT_r[t_hi] - CT_r[t_lo]),
    where CS_r[j] = sum_{s<j} S_r[s] is the 1D summed-area table of S_r
    (two look-ups per axis, exact).
Readings:
  * The query returns the box SUM of bin masses; the paper's average is
    sum / ((s_hi - s_lo) (t_hi - t_lo)).
  * Boundary rules: u, v wrap; l clamps to [0, nl-1]; bin bounds clamp to
    [0, N]; an empty box (lo >= hi on either axis) gives exactly 0.
  * Off-grid footprints: trilinear blend of the eight surrounding
    precomputed footprints' range queries (see range_query_trilinear).
"""
from __future__ import annotations

import numpy as np

from .ndf import canonical_query


def cumulative(S: np.ndarray) -> np.ndarray:
    """CS[j] = sum_{s<j} S[s], j = 0..N, shape [N+1][R], FP64."""
    S = np.asarray(S, dtype=np.float64)
    out = np.zeros((S.shape[0] + 1, S.shape[1]))
    out[1:] = np.cumsum(S, axis=0)
    return out


def point_query(U, V, L, S, Tf, u, v, l, s, t) -> float:
    return float(np.sum(U[u] * V[v] * L[l] * S[s] * Tf[t]))


def range_query(U, V, L, CS, CT, q, scale=None) -> np.ndarray:
    """q[i] per query record (u, v, l, s_lo, s_hi, t_lo, t_hi); FP64.

    ``scale`` is an optional per-rank multiplier (dequantisation scales).
    """
    U, V, L, CS, CT = (np.asarray(x, dtype=np.float64) for x in (U, V, L, CS, CT))
    nu, nv, nl, N = U.shape[0], V.shape[0], L.shape[0], CS.shape[0] - 1
    q = canonical_query(q, nu, nv, nl, N)
    u, v, l, slo, shi, tlo, thi = q.T
    dS = CS[shi] - CS[slo]
    dT = CT[thi] - CT[tlo]
    P = U[u] * V[v] * L[l] * dS * dT
    if scale is not None:
        P = P * np.asarray(scale, dtype=np.float64)[None, :]
    out = P.sum(axis=1)
    empty = (slo >= shi) | (tlo >= thi)
    out[empty] = 0.0
    return out


# Off-grid footprints (Sec. 4.1 and Sec. 4.3): a footprint between the
# precomputed centres and levels takes the trilinear blend of the NDF values
# of the eight surrounding precomputed footprints.  Coordinates are in index
# units: x, y continuous footprint centres (u = floor(x) wraps, fraction
# x - floor(x)); lam a continuous level clamped to [0, nl - 1].  Reading: a
# non-finite coordinate counts as 0, and |x|, |y| are clamped to 2^24 (where
# FP32 has no fraction left).
COORD_LIMIT = float(1 << 24)


def trilinear_corners(xyl, nu, nv, nl):
    """Corner indices [n][8][3] (u, v, l) and blend weights [n][8] (FP64)."""
    xyl = np.asarray(xyl, dtype=np.float32).astype(np.float64)
    xyl = np.where(np.isfinite(xyl), xyl, 0.0)
    x = np.clip(xyl[:, 0], -COORD_LIMIT, COORD_LIMIT)
    y = np.clip(xyl[:, 1], -COORD_LIMIT, COORD_LIMIT)
    lam = np.clip(xyl[:, 2], 0.0, nl - 1.0)
    fx0, fy0, fl0 = np.floor(x), np.floor(y), np.floor(lam)
    fx, fy, fl = x - fx0, y - fy0, lam - fl0
    u0, v0, l0 = fx0.astype(np.int64), fy0.astype(np.int64), fl0.astype(np.int64)
    corners = np.empty((x.shape[0], 8, 3), dtype=np.int64)
    weights = np.empty((x.shape[0], 8))
    c = 0
    for a in (0, 1):
        for b in (0, 1):
            for d in (0, 1):
                corners[:, c, 0] = np.mod(u0 + a, nu)
                corners[:, c, 1] = np.mod(v0 + b, nv)
                corners[:, c, 2] = np.minimum(l0 + d, nl - 1)
                weights[:, c] = (fx if a else 1.0 - fx) * (fy if b else 1.0 - fy) * (fl if d else 1.0 - fl)
                c += 1
    return corners, weights


def range_query_trilinear(U, V, L, CS, CT, xyl, boxes, scale=None, magnitude=False) -> np.ndarray:
    """Trilinear blend over the 8 surrounding footprints of the range query of
    each box (boxes [n][4] = s_lo, s_hi, t_lo, t_hi); FP64.  With
    ``magnitude`` the blend of the corners' rank-term magnitudes instead: an
    evaluation that interpolates the factor rows first has its error scaled
    by sum_r (sum_c w_c |U_c|)(sum_c w_c |V_c|)(sum_c w_c |L_c|) |dS dT|,
    which is this blend."""
    nu, nv, nl = U.shape[0], V.shape[0], L.shape[0]
    corners, w = trilinear_corners(xyl, nu, nv, nl)
    boxes = np.asarray(boxes, dtype=np.int64)
    fn = range_query_term_magnitude if magnitude else range_query
    out = np.zeros(corners.shape[0])
    for c in range(8):
        rec = np.concatenate([corners[:, c, :], boxes], axis=1)
        out += w[:, c] * fn(U, V, L, CS, CT, rec, scale=scale)
    return out


def range_query_magnitude(U, V, L, CS, CT, q, scale=None) -> np.ndarray:
    """Condition magnitude of the cumulative-difference evaluation:
    N_q = sum_r |U V L| (|CS_hi| + |CS_lo|) (|CT_hi| + |CT_lo|)."""
    U, V, L, CS, CT = (np.abs(np.asarray(x, dtype=np.float64)) for x in (U, V, L, CS, CT))
    nu, nv, nl, N = U.shape[0], V.shape[0], L.shape[0], CS.shape[0] - 1
    q = canonical_query(q, nu, nv, nl, N)
    u, v, l, slo, shi, tlo, thi = q.T
    P = U[u] * V[v] * L[l] * (CS[shi] + CS[slo]) * (CT[thi] + CT[tlo])
    if scale is not None:
        P = P * np.abs(np.asarray(scale, dtype=np.float64))[None, :]
    out = P.sum(axis=1)
    out[(slo >= shi) | (tlo >= thi)] = 0.0
    return out


def range_query_term_magnitude(U, V, L, CS, CT, q, scale=None) -> np.ndarray:
    """Sum of the magnitudes of the rank terms of Eq. rangeDecom:
    M_q = sum_r |c_r U_r[u] V_r[v] L_r[l] (CS_r[s_hi] - CS_r[s_lo]) (CT_r[t_hi] - CT_r[t_lo])|.

    An FP32 evaluation of the same stored values rounds each difference
    relative to the difference itself (a correctly rounded subtraction), then
    each product relative to the product, so every rank term is within a few
    units in the last place of its own size and the rank sum is within a
    rank-dependent multiple of M_q: M_q is the scale of a query's arithmetic
    error.  (N_q above bounds it too, but loosely: for a narrow box the
    summed-area values are much larger than their difference.)"""
    U, V, L, CS, CT = (np.asarray(x, dtype=np.float64) for x in (U, V, L, CS, CT))
    nu, nv, nl, N = U.shape[0], V.shape[0], L.shape[0], CS.shape[0] - 1
    q = canonical_query(q, nu, nv, nl, N)
    u, v, l, slo, shi, tlo, thi = q.T
    P = U[u] * V[v] * L[l] * (CS[shi] - CS[slo]) * (CT[thi] - CT[tlo])
    if scale is not None:
        P = P * np.asarray(scale, dtype=np.float64)[None, :]
    out = np.abs(P).sum(axis=1)
    out[(slo >= shi) | (tlo >= thi)] = 0.0
    return out


def range_query_grad(U, V, L, CS, CT, q, g):
    """Gradients of sum_i g[i] * q[i] with respect to U, V, L, CS, CT (FP64)."""
    U, V, L, CS, CT = (np.asarray(x, dtype=np.float64) for x in (U, V, L, CS, CT))
    nu, nv, nl, N = U.shape[0], V.shape[0], L.shape[0], CS.shape[0] - 1
    q = canonical_query(q, nu, nv, nl, N)
    u, v, l, slo, shi, tlo, thi = q.T
    g = np.asarray(g, dtype=np.float64).copy()
    g[(slo >= shi) | (tlo >= thi)] = 0.0
    dS = CS[shi] - CS[slo]
    dT = CT[thi] - CT[tlo]
    Uu, Vv, Ll = U[u], V[v], L[l]
    gc = g[:, None]
    dU = np.zeros_like(U)
    dV = np.zeros_like(V)
    dL = np.zeros_like(L)
    dCS = np.zeros_like(CS)
    dCT = np.zeros_like(CT)
    np.add.at(dU, u, gc * Vv * Ll * dS * dT)
    np.add.at(dV, v, gc * Uu * Ll * dS * dT)
    np.add.at(dL, l, gc * Uu * Vv * dS * dT)
    wS = gc * Uu * Vv * Ll * dT
    np.add.at(dCS, shi, wS)
    np.add.at(dCS, slo, -wS)
    wT = gc * Uu * Vv * Ll * dS
    np.add.at(dCT, thi, wT)
    np.add.at(dCT, tlo, -wT)
    return dU, dV, dL, dCS, dCT


def cumulative_grad(dC: np.ndarray) -> np.ndarray:
    """Chain rule through CS[j] = sum_{s<j} S[s]: dS[s] = sum_{j>s} dC[j]."""
    dC = np.asarray(dC, dtype=np.float64)
    n = dC.shape[0] - 1
    out = np.zeros((n, dC.shape[1]))
    for s in range(n):
        out[s] = dC[s + 1:].sum(axis=0)
    return out


def mse_loss(qv: np.ndarray, target: np.ndarray):
    """Refinement loss (1/Q) sum (q - target)^2 and its gradient in q."""
    qv = np.asarray(qv, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    d = qv - target
    return float(np.mean(d * d)), 2.0 * d / d.shape[0]


def count_invalid(q, nu: int, nv: int, nlevels: int, nbins: int) -> int:
    """Records the query rules would change: u or v outside the map (they
    wrap), l outside [0, nlevels) (it clamps), a bin bound outside [0, N]
    (it clamps), or a reversed box (lo > hi; lo == hi is a valid empty box)."""
    q = np.asarray(q, dtype=np.int64).reshape(-1, 7)
    bad = (q[:, 0] < 0) | (q[:, 0] >= nu) | (q[:, 1] < 0) | (q[:, 1] >= nv)
    bad |= (q[:, 2] < 0) | (q[:, 2] >= nlevels)
    bad |= np.any((q[:, 3:7] < 0) | (q[:, 3:7] > nbins), axis=1)
    bad |= (q[:, 3] > q[:, 4]) | (q[:, 5] > q[:, 6])
    return int(bad.sum())
