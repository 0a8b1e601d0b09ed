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
