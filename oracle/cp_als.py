"""Oracle: plain CP decomposition by alternating least squares (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed (Sec. 4.2, Eq. compress): T is approximated by a sum of R
rank-one terms, lambda_r * U_r (x) V_r (x) L_r (x) S_r (x) T_r, fitted by
alternating least squares: each sweep updates the five factors in the order
(u, v, l, s, t); a mode update is the exact least-squares solution with the
other four factors fixed, A_n = M_n G^-1, where M_n is the MTTKRP (T unfolded
along mode n times the Khatri-Rao product of the other factors) and G the
Hadamard product of the other factors' Gram matrices.

Readings where the paper is silent (its own setup is per-cluster 3-way
tensors stopped at an error of 1e-4 or 500 sweeps):
  * The initial factors are an input (i.i.d. U[0,1) drawn by the caller).
  * After each update the columns are scaled to unit 2-norm and the norms
    kept as lambda; a zero column is left as it is.  After the last sweep
    lambda is absorbed into the level factor L.
  * G is factored by Cholesky; it counts as failed when a pivot is not above
    1e-13 times the matching diagonal entry of G; then the eigen-decomposition
    pseudo-inverse with eigenvalues below 1e-12 * max eigenvalue dropped is
    used instead.
  * A fixed number of sweeps; optionally stop once |fit_k - fit_{k-1}| < tol.
  * fit = 1 - ||T - T^|| / ||T||, with ||T^||^2 = lambda^T (*_m A_m^T A_m) lambda
    and <T, T^> = sum_r lambda_r sum_i M_t[i, r] A_t[i, r].
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

_LETTERS = "abcde"


def mttkrp(T: np.ndarray, A, n: int) -> np.ndarray:
    """M_n[i, r] = sum over all other indices of T * prod_{m != n} A_m[i_m, r]."""
    others = [m for m in range(5) if m != n]
    spec = _LETTERS + "," + ",".join(_LETTERS[m] + "r" for m in others) + "->" + _LETTERS[n] + "r"
    return np.einsum(spec, T, *[A[m] for m in others], optimize=True)


def gram_hadamard(A, n: int) -> np.ndarray:
    R = A[0].shape[1]
    G = np.ones((R, R))
    for m in range(5):
        if m != n:
            G = G * (A[m].T @ A[m])
    return G


PIVOT_RTOL = 1e-13


def solve_gram(M: np.ndarray, G: np.ndarray):
    """X = M G^-1 (G symmetric PSD).  Returns (X, used_fallback).

    Cholesky counts as failed when a pivot is not above PIVOT_RTOL times the
    matching diagonal entry of G (a singular PSD matrix can leave a tiny
    positive pivot after rounding)."""
    try:
        c = np.linalg.cholesky(G)
        if np.any(np.diag(c) ** 2 <= PIVOT_RTOL * np.diag(G)):
            raise np.linalg.LinAlgError("relative pivot breakdown")
        X = scipy.linalg.cho_solve((c, True), M.T).T
        return X, False
    except np.linalg.LinAlgError:
        w, Q = np.linalg.eigh(G)
        keep = w > 1e-12 * max(float(w.max()), 0.0)
        winv = np.zeros_like(w)
        winv[keep] = 1.0 / w[keep]
        return M @ (Q * winv) @ Q.T, True


def normalize_columns(X: np.ndarray):
    lam = np.linalg.norm(X, axis=0)
    Y = X.copy()
    nz = lam > 0.0
    Y[:, nz] = X[:, nz] / lam[nz]
    return Y, lam


def fit_value(normT2: float, A, lam: np.ndarray, M_last: np.ndarray) -> float:
    R = lam.shape[0]
    Gall = np.ones((R, R))
    for m in range(5):
        Gall = Gall * (A[m].T @ A[m])
    inner = float(np.sum(lam * np.sum(M_last * A[4], axis=0)))
    normhat2 = float(lam @ Gall @ lam)
    resid2 = max(normT2 - 2.0 * inner + normhat2, 0.0)
    return 1.0 - np.sqrt(resid2) / np.sqrt(normT2)


def reconstruct(U, V, L, S, Tf, lam=None) -> np.ndarray:
    """Full tensor from the factors (lambda optional, else folded in L)."""
    Lw = L if lam is None else L * lam[None, :]
    return np.einsum("ar,br,cr,dr,er->abcde", U, V, Lw, S, Tf, optimize=True)


def cp_als(T: np.ndarray, init, iters: int, tol: float = 0.0, trace=None):
    """Plain CP-ALS.  ``init`` is (U, V, L, S, T) FP64, not modified.

    Returns a dict: factors (U, V, L*lambda, S, T), lam, fits (per sweep),
    sweeps run, fallbacks (count of pseudo-inverse solves), and if ``trace``
    is a list, every sweep's normalised factors and lambda are appended to it.
    """
    T = np.asarray(T, dtype=np.float64)
    return _als(lambda A, n: mttkrp(T, A, n), float(np.sum(T * T)), init, iters, tol, trace)


def cp_als_texel(ms: np.ndarray, mt: np.ndarray, nlevels: int, init, iters: int, normT2=None,
                 tol: float = 0.0):
    """The same ALS for the tensor of per-texel masses ms, mt ([nu][nv][N],
    see ndf.texel_masses), with every MTTKRP taken by mttkrp_structured so the
    tensor is never formed.  ||T||^2 is an input (it needs the tensor); when
    it is None the fits are NaN and no tolerance stop is possible."""
    ms = np.asarray(ms, dtype=np.float64)
    mt = np.asarray(mt, dtype=np.float64)
    if normT2 is None and tol > 0.0:
        raise ValueError("a tolerance stop needs ||T||^2")
    return _als(lambda A, n: mttkrp_structured(ms, mt, nlevels, A, n),
                np.nan if normT2 is None else float(normT2), init, iters, tol, None)


def _als(mttkrp_fn, normT2: float, init, iters: int, tol: float, trace):
    A = [np.array(a, dtype=np.float64, copy=True) for a in init]
    R = A[0].shape[1]
    lam = np.ones(R)
    fits = []
    fallbacks = 0
    sweeps = 0
    for it in range(iters):
        M = None
        for n in range(5):
            M = mttkrp_fn(A, n)
            G = gram_hadamard(A, n)
            X, fb = solve_gram(M, G)
            fallbacks += int(fb)
            A[n], lam = normalize_columns(X)
        fits.append(fit_value(normT2, A, lam, M))
        sweeps = it + 1
        if trace is not None:
            trace.append(([a.copy() for a in A], lam.copy()))
        if tol > 0.0 and it > 0 and abs(fits[-1] - fits[-2]) < tol:
            break
    out = [a.copy() for a in A]
    out[2] = out[2] * lam[None, :]
    return {"factors": tuple(out), "lam": lam, "fits": np.array(fits),
            "sweeps": sweeps, "fallbacks": fallbacks, "normT2": normT2}


# ----------------------------------------------------------------------------
# Texel-space MTTKRP: the same contraction for the tensor built from texel
# masses, evaluated without forming T.  Used as a pin for the dense MTTKRP.
# ----------------------------------------------------------------------------


def _window_sum(X: np.ndarray, k: int) -> np.ndarray:
    """Xbar[x] = sum of X[c] over every centre c whose k-footprint contains x.

    A footprint anchored at c covers c - k//2 + i for 0 <= i < k, so x is
    covered by the centres c = x + k//2 - i.
    """
    out = np.zeros_like(X)
    for i in range(k):
        out += np.roll(X, -(k // 2 - i), axis=0)
    return out


def mttkrp_structured(ms: np.ndarray, mt: np.ndarray, nlevels: int, A, n: int) -> np.ndarray:
    """MTTKRP of mode n for T[u,v,l,s,t] = (1/k^2) sum_{footprint} ms (x) mt.

    ms, mt: per-texel masses [nu][nv][N].  A = (U, V, L, S, T) factors.
    """
    U, V, L, S, Tf = A
    gs = np.einsum("xys,sr->xyr", ms, S)
    gt = np.einsum("xyt,tr->xyr", mt, Tf)
    nu, nv = ms.shape[:2]
    R = U.shape[1]
    if n == 2:
        out = np.zeros((nlevels, R))
    elif n == 0:
        out = np.zeros((nu, R))
    elif n == 1:
        out = np.zeros((nv, R))
    else:
        out = np.zeros((ms.shape[2], R))
    for l in range(nlevels):
        k = 1 << l
        w = L[l] / float(k * k)
        Ub = _window_sum(U, k)                 # [nu][R]
        Vb = _window_sum(V, k)                 # [nv][R]
        if n == 0:   # sum_{x in W(u)} sum_y Vb[y] gs gt
            H = np.einsum("yr,xyr,xyr->xr", Vb, gs, gt)
            Hc = np.zeros_like(H)
            for i in range(k):                 # footprint of u covers u - k//2 + i
                Hc += np.roll(H, -(i - k // 2), axis=0)
            out += w * Hc
        elif n == 1:
            H = np.einsum("xr,xyr,xyr->yr", Ub, gs, gt)
            Hc = np.zeros_like(H)
            for i in range(k):
                Hc += np.roll(H, -(i - k // 2), axis=0)
            out += w * Hc
        elif n == 2:
            out[l] = np.einsum("xr,yr,xyr,xyr->r", Ub, Vb, gs, gt) / float(k * k)
        elif n == 3:   # sum_{x,y} ms[x,y,s] gt[x,y] Ub[x] Vb[y]: a product over texels, then a matmul
            H = gt * Ub[:, None, :] * Vb[None, :, :]
            out += (ms.reshape(-1, ms.shape[2]).T @ H.reshape(-1, R)) * w
        else:
            H = gs * Ub[:, None, :] * Vb[None, :, :]
            out += (mt.reshape(-1, mt.shape[2]).T @ H.reshape(-1, R)) * w
    return out
