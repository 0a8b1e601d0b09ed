"""Oracle: the clustered layout of the paper's compression (Sec. 4.2,
Eq. compress and its practical choices), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed:
  * Each NDF image (one footprint: centre (u, v), level l) is cut into
    t x t angular blocks; footprints are grouped by the cs x cs texel region
    their centre lies in.  For a region (cluster) and an angular block, the
    blocks of all L = cs * cs * nl footprints of the region are stacked into a
    3-way tensor D[a][b][f] (a, b the bins inside the block, f the footprint:
    f = (du * cs + dv) * nl + l for centre (cu * cs + du, cv * cs + dv)).
  * Each non-blank D is fitted by a rank-R CP, D ~ sum_r X_r (x) Y_r (x) Z_r,
    by alternating least squares (modes X, Y, Z in that order; column
    weights absorbed into Z after the last sweep).
  * A range query adds, over the angular blocks the box overlaps, the
    block-local range query of that block's CP (two summed-area look-ups
    per axis inside the block, Sec. 4.4), splitting the box at block edges.
Readings:
  * Blank image blocks are thrown away before the fit (Sec. 4.2): the image
    block of footprint f is blank when the sum of its |values| is at most
    BLANK_TOL (1e-12; an NDF image has unit mass).  D is stacked from the
    L' non-blank blocks only, in footprint order, and fitted as t x t x L';
    the Z row of a blank footprint is zero, so it contributes exactly 0 to a
    query.  A (region, block) tensor with no non-blank footprint is blank
    and stores zero factors.
  * ALS initial factors: U[0, 1) from SplitMix64 used as a counter-based
    generator (the n-th output of the generator seeded with `seed`, n
    counted from 1): value(counter) = (mix(seed + (counter + 1) * gamma) >> 11)
    * 2^-53, with counter = ((tensor * 3 + mode) * max(t, L) + row) * R + r,
    tensor = ((cu * ncv + cv) * nb + zs) * nb + zt; the row of a Z entry is
    the footprint index f of its (non-blank) block.
  * Normal equations with a small ridge: A = M (G + mu I)^-1, mu = 1e-10 x
    trace(G) / R (a region-and-block tensor is often of lower rank than R,
    and its Hadamard Gram then singular); Cholesky breakdown (pivot <= 1e-13 x
    the diagonal entry) keeps that mode's previous factor and is counted;
    columns are normalised to unit length after every update (zero columns
    stay zero); fixed sweep count.
  * cs must divide the map sides and t must divide N (t = N when N < t).
  * Sampling on this layout (Sec. 5.2: start from a block chosen by the
    blocks' averaged NDF values, then the four-quad descent inside it): the
    block is drawn with probability proportional to its mass (the
    block-local query over the whole block; negative masses count as zero;
    block order zs-major), by the same running-sum rule as a quad, then
    log2(t) quad levels inside it (t a power of two) and a uniform position
    in the final bin.  Draws per sample: one for the block, log2(t) for the
    levels, two for the position.  pdf = P(bin) / (2/N)^2; a footprint
    without positive mass fails (bin (-1, -1), pdf 0, h = (0, 0)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .ndf import canonical_query, footprint_offsets, texel_masses

BLANK_TOL = 1e-12
PIVOT_RTOL = 1e-13
RIDGE_RTOL = 1e-10
_GAMMA = 0x9E3779B97F4A7C15
_MASK = (1 << 64) - 1


def splitmix64_mix(z: int) -> int:
    """The output function of SplitMix64 (Steele, Lea and Flood 2014)."""
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def splitmix64_stream(seed: int, n: int):
    """The first n outputs of SplitMix64 seeded with `seed`."""
    return [splitmix64_mix((seed + (i + 1) * _GAMMA) & _MASK) for i in range(n)]


def uniform(seed: int, counters: np.ndarray) -> np.ndarray:
    """U[0, 1) from SplitMix64 at the given counters (vectorised)."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def layout(nu, nv, nl, N, t, cs):
    """(ncu, ncv, nb, L) of the clustered layout."""
    if N < t:
        t = N
    assert nu % cs == 0 and nv % cs == 0 and N % t == 0
    return nu // cs, nv // cs, N // t, cs * cs * nl, t


def cluster_tensor(T: np.ndarray, cu: int, cv: int, zs: int, zt: int, t: int, cs: int) -> np.ndarray:
    """D[a][b][f] of region (cu, cv) and angular block (zs, zt)."""
    sub = T[cu * cs:(cu + 1) * cs, cv * cs:(cv + 1) * cs, :, zs * t:(zs + 1) * t, zt * t:(zt + 1) * t]
    # sub[du][dv][l][a][b] -> D[a][b][(du*cs + dv)*nl + l]
    return np.ascontiguousarray(sub.reshape(-1, t, t).transpose(1, 2, 0))


def region_block_tensor(nxy: np.ndarray, nbins: int, sigma: float, nlevels: int, t: int, cs: int,
                        cu: int, cv: int, zs: int, zt: int) -> np.ndarray:
    """D[a][b][f] of region (cu, cv) and angular block (zs, zt) straight from
    the normal map, for maps whose tensor is too large to form: footprint f =
    (du cs + dv) nl + l, centred at (cu cs + du, cv cs + dv), is the mean over
    its k x k texels (toroidal, the offsets of ndf_bruteforce) of
    m_s[zs t + a] m_t[zt t + b] (Sec. 3.1 Eq. geom restricted to the block's
    bins): the same entries cluster_tensor takes from the full tensor.  The
    sum over a footprint's texels is one product of its texels' s-masses and
    t-masses."""
    ms, mt = texel_masses(nxy, nbins, sigma)
    nu, nv = ms.shape[:2]
    ms = ms[:, :, zs * t:(zs + 1) * t]
    mt = mt[:, :, zt * t:(zt + 1) * t]
    D = np.zeros((t, t, cs * cs * nlevels))
    for du in range(cs):
        for dv in range(cs):
            u, v = cu * cs + du, cv * cs + dv
            for l in range(nlevels):
                k = 1 << l
                xs = (u + footprint_offsets(k)) % nu
                ys = (v + footprint_offsets(k)) % nv
                a = ms[xs][:, ys].reshape(-1, t)
                b = mt[xs][:, ys].reshape(-1, t)
                D[:, :, (du * cs + dv) * nlevels + l] = (a.T @ b) / float(k * k)
    return D


def init_factors(seed: int, tensor: int, t: int, L: int, R: int, zrows=None):
    """Initial X [t][R], Y [t][R] and Z [len(zrows)][R] (zrows: the footprint
    indices of the stacked blocks, default all L)."""
    rows_max = max(t, L)
    zrows = np.arange(L) if zrows is None else np.asarray(zrows)

    def block(mode, rows):
        i = np.asarray(rows, dtype=np.uint64)[:, None]
        r = np.arange(R, dtype=np.uint64)[None, :]
        c = ((np.uint64(tensor) * np.uint64(3) + np.uint64(mode)) * np.uint64(rows_max) + i) * np.uint64(R) + r
        return uniform(seed, c)

    return block(0, np.arange(t)), block(1, np.arange(t)), block(2, zrows)


def nonblank_footprints(D: np.ndarray) -> np.ndarray:
    """Indices f of the non-blank image blocks D[:, :, f]."""
    return np.nonzero(np.abs(D).sum(axis=(0, 1)) > BLANK_TOL)[0]


def _solve(M, G):
    """X = M (G + mu I)^-1 with mu = RIDGE_RTOL * trace(G) / R, by Cholesky
    with the relative-pivot breakdown rule; None on breakdown."""
    R = G.shape[0]
    Gr = G + (RIDGE_RTOL * float(np.trace(G)) / R) * np.eye(R)
    try:
        c = np.linalg.cholesky(Gr)
    except np.linalg.LinAlgError:
        return None
    if np.any(np.diag(c) ** 2 <= PIVOT_RTOL * np.diag(Gr)):
        return None
    return scipy.linalg.cho_solve((c, True), M.T).T


def als3(D: np.ndarray, init, iters: int):
    """Plain 3-way CP-ALS of D[a][b][f].  Returns (X, Y, Z * lambda, fails)."""
    a, b, c = D.shape
    X, Y, Z = (np.array(m, dtype=np.float64) for m in init)
    R = X.shape[1]
    lam = np.ones(R)
    fails = 0
    D1 = D.reshape(a, b * c)                        # [a][(b, f)]
    D2 = D.transpose(1, 0, 2).reshape(b, a * c)     # [b][(a, f)]
    D3 = D.transpose(2, 0, 1).reshape(c, a * b)     # [f][(a, b)]

    def kr(P, Q):                                   # Khatri-Rao, rows (p, q) with q fastest
        return (P[:, None, :] * Q[None, :, :]).reshape(-1, R)

    def upd(M, G, cur):
        nonlocal fails
        new = _solve(M, G)
        if new is None:
            fails += 1
            return cur, False
        return new, True

    for _ in range(iters):
        Xn, ok = upd(D1 @ kr(Y, Z), (Y.T @ Y) * (Z.T @ Z), X)
        if ok:
            lam = np.linalg.norm(Xn, axis=0)
            X = np.where(lam > 0, Xn / np.where(lam > 0, lam, 1.0), Xn)
        Yn, ok = upd(D2 @ kr(X, Z), (X.T @ X) * (Z.T @ Z), Y)
        if ok:
            lam = np.linalg.norm(Yn, axis=0)
            Y = np.where(lam > 0, Yn / np.where(lam > 0, lam, 1.0), Yn)
        Zn, ok = upd(D3 @ kr(X, Y), (X.T @ X) * (Y.T @ Y), Z)
        if ok:
            lam = np.linalg.norm(Zn, axis=0)
            Z = np.where(lam > 0, Zn / np.where(lam > 0, lam, 1.0), Zn)
    return X, Y, Z * lam[None, :], fails


def clustered_cp(T: np.ndarray, t: int, cs: int, R: int, iters: int, seed: int, counts: bool = False):
    """Factors of every (region, block): X, Y [ncu][ncv][nb][nb][t][R],
    Z [ncu][ncv][nb][nb][L][R] (lambda absorbed; zero rows for blank image
    blocks), blank flags, failures; with counts=True also L' per tensor."""
    nu, nv, nl, N = T.shape[:4]
    ncu, ncv, nb, L, t = layout(nu, nv, nl, N, t, cs)
    X = np.zeros((ncu, ncv, nb, nb, t, R))
    Y = np.zeros_like(X)
    Z = np.zeros((ncu, ncv, nb, nb, L, R))
    blank = np.zeros((ncu, ncv, nb, nb), dtype=bool)
    nkept = np.zeros((ncu, ncv, nb, nb), dtype=np.int64)
    fails = 0
    for cu in range(ncu):
        for cv in range(ncv):
            for zs in range(nb):
                for zt in range(nb):
                    D = cluster_tensor(T, cu, cv, zs, zt, t, cs)
                    keep = nonblank_footprints(D)
                    nkept[cu, cv, zs, zt] = len(keep)
                    if len(keep) == 0:
                        blank[cu, cv, zs, zt] = True
                        continue
                    tensor = ((cu * ncv + cv) * nb + zs) * nb + zt
                    x, y, z, f = als3(D[:, :, keep], init_factors(seed, tensor, t, L, R, keep), iters)
                    X[cu, cv, zs, zt], Y[cu, cv, zs, zt] = x, y
                    Z[cu, cv, zs, zt][keep] = z
                    fails += f
    if counts:
        return X, Y, Z, blank, fails, nkept
    return X, Y, Z, blank, fails


def reconstruct(X, Y, Z, nl: int, cs: int) -> np.ndarray:
    """The tensor T[u][v][l][s][t] the clustered factors represent."""
    ncu, ncv, nb = X.shape[:3]
    t = X.shape[4]
    out = np.zeros((ncu * cs, ncv * cs, nl, nb * t, nb * t))
    for cu in range(ncu):
        for cv in range(ncv):
            for zs in range(nb):
                for zt in range(nb):
                    D = np.einsum("ar,br,fr->abf", X[cu, cv, zs, zt], Y[cu, cv, zs, zt], Z[cu, cv, zs, zt])
                    blk = D.transpose(2, 0, 1).reshape(cs, cs, nl, t, t)
                    out[cu * cs:(cu + 1) * cs, cv * cs:(cv + 1) * cs, :, zs * t:(zs + 1) * t,
                        zt * t:(zt + 1) * t] = blk
    return out


def block_cumulative(X) -> np.ndarray:
    """Block-local summed-area tables: C[..., j, r] = sum_{a<j} X[..., a, r]
    for j = 0..t (Sec. 4.4 within each angular block), FP64."""
    X = np.asarray(X, dtype=np.float64)
    z = np.zeros(X.shape[:-2] + (1, X.shape[-1]))
    return np.concatenate([z, np.cumsum(X, axis=-2)], axis=-2)


def clustered_range_query(X, Y, Z, q, nl: int, cs: int) -> np.ndarray:
    """Box sums by splitting each box at block edges and adding the
    block-local range queries (cumulative sums of X and Y inside a block)."""
    return clustered_range_query_tables(block_cumulative(X), block_cumulative(Y), Z, q, nl, cs)


def clustered_range_query_tables(CX, CY, Z, q, nl: int, cs: int) -> np.ndarray:
    """The block-split range query on given block-local summed-area tables
    CX, CY [ncu][ncv][nb][nb][t+1][R] (e.g. stored values rounded to a
    storage type, Sec. 4.4): over the blocks the box overlaps, the term
    sum_r Z[f][r] (CX[a1][r] - CX[a0][r]) (CY[b1][r] - CY[b0][r]) with the
    box clipped to the block, in FP64."""
    ncu, ncv, nb = CX.shape[:3]
    t = CX.shape[4] - 1
    nu, nv, N = ncu * cs, ncv * cs, nb * t
    q = canonical_query(q, nu, nv, nl, N)
    out = np.zeros(q.shape[0])
    for i, (u, v, l, slo, shi, tlo, thi) in enumerate(q):
        if slo >= shi or tlo >= thi:
            continue
        cu, cv = u // cs, v // cs
        f = ((u % cs) * cs + (v % cs)) * nl + l
        acc = 0.0
        for zs in range(slo // t, (shi - 1) // t + 1):
            a0, a1 = max(slo, zs * t) - zs * t, min(shi, (zs + 1) * t) - zs * t
            for zt in range(tlo // t, (thi - 1) // t + 1):
                b0, b1 = max(tlo, zt * t) - zt * t, min(thi, (zt + 1) * t) - zt * t
                cx, cy = CX[cu, cv, zs, zt], CY[cu, cv, zs, zt]
                acc += float(np.sum(np.asarray(Z[cu, cv, zs, zt, f], dtype=np.float64)
                                    * (cx[a1] - cx[a0]) * (cy[b1] - cy[b0])))
        out[i] = acc
    return out


def _pick(m, u):
    """Index chosen by draw u from non-negative masses m (running-sum rule,
    never an empty entry at the top of the range); None if all are empty."""
    total = 0.0
    for x in m:
        total += x
    if not total > 0.0:
        return None, total
    target = u * total
    run = 0.0
    pick = len(m) - 1
    for i, x in enumerate(m):
        run += x
        if target < run:
            pick = i
            break
    while m[pick] <= 0.0:
        pick -= 1
    return pick, total


def clustered_sample(X, Y, Z, uvl, rnd, nl: int, cs: int):
    """Hierarchical samples on the clustered layout for records uvl [n][3]
    (wrapped/clamped like the query) with draws rnd [n][log2(t) + 3]."""
    ncu, ncv, nb = X.shape[:3]
    t = X.shape[4]
    levels = int(round(np.log2(t)))
    N = nb * t
    uvl = np.asarray(uvl, dtype=np.int64)
    rnd = np.asarray(rnd, dtype=np.float64)
    n = uvl.shape[0]
    h = np.zeros((n, 2))
    pdf = np.zeros(n)
    bins = np.full((n, 2), -1, dtype=np.int64)
    w = 2.0 / N
    for i in range(n):
        u = int(np.mod(uvl[i, 0], ncu * cs))
        v = int(np.mod(uvl[i, 1], ncv * cs))
        l = int(np.clip(uvl[i, 2], 0, nl - 1))
        cu, cv = u // cs, v // cs
        f = ((u % cs) * cs + (v % cs)) * nl + l
        CX = [np.concatenate([np.zeros((1, X.shape[-1])), np.cumsum(X[cu, cv, zs, zt], axis=0)])
              for zs in range(nb) for zt in range(nb)]
        CY = [np.concatenate([np.zeros((1, Y.shape[-1])), np.cumsum(Y[cu, cv, zs, zt], axis=0)])
              for zs in range(nb) for zt in range(nb)]
        zrow = [Z[cu, cv, b // nb, b % nb, f] for b in range(nb * nb)]
        bm = [max(float(np.sum(zrow[b] * (CX[b][t] - CX[b][0]) * (CY[b][t] - CY[b][0]))), 0.0)
              for b in range(nb * nb)]
        b, total = _pick(bm, rnd[i, 0])
        if b is None:
            continue
        prob = bm[b] / total
        s0, s1, t0, t1 = 0, t, 0, t
        failed = False
        for k in range(levels):
            sm, tm = (s0 + s1) // 2, (t0 + t1) // 2
            dS = (CX[b][sm] - CX[b][s0], CX[b][s1] - CX[b][sm])
            dT = (CY[b][tm] - CY[b][t0], CY[b][t1] - CY[b][tm])
            m = [max(float(np.sum(zrow[b] * dS[a] * dT[c])), 0.0) for a in (0, 1) for c in (0, 1)]
            q, qt = _pick(m, rnd[i, 1 + k])
            if q is None:
                failed = True
                break
            prob *= m[q] / qt
            s0, s1 = (sm, s1) if q >= 2 else (s0, sm)
            t0, t1 = (tm, t1) if q % 2 == 1 else (t0, tm)
        if failed:
            continue
        bs, bt = (b // nb) * t + s0, (b % nb) * t + t0
        bins[i] = (bs, bt)
        h[i] = (-1.0 + (bs + rnd[i, 1 + levels]) * w, -1.0 + (bt + rnd[i, 2 + levels]) * w)
        pdf[i] = prob / (w * w)
    return h, pdf, bins
