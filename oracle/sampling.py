"""Oracle: hierarchical NDF importance sampling by range queries (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed (Sec. 5.2, accurate NDF importance sampling): for one
footprint (u, v, l), the N x N NDF image is split evenly into four quads;
the range query of each quad gives its mass, one quad is drawn with
probability proportional to the masses, and the split repeats inside it
until a single bin remains; the sample is then placed uniformly inside that
bin.  The probability of a bin is the product of the chosen quads'
probabilities, which equals the bin's NDF mass over the image's total mass,
so the density of the sample is the normalised NDF.

Readings:
  * The descent starts from the whole image (this layout has no angular
    blocks), N a power of two, so there are log2(N) levels.
  * Quad order (s low, t low), (s low, t high), (s high, t low),
    (s high, t high); the uniform draw u picks the first quad whose running
    mass sum exceeds u times the total.
  * Masses below zero (possible for a CP approximation) count as zero; if
    all four quads of a level have no positive mass the sample fails:
    bin (-1, -1), pdf 0, h = (0, 0).
  * Random numbers are inputs: per sample log2(N) draws for the levels and
    two for the position inside the bin, all in [0, 1).
  * h = (-1 + (s + j_s) * 2/N, -1 + (t + j_t) * 2/N); pdf is the density in
    (s, t) units, P(bin) / (2/N)^2.
"""
from __future__ import annotations

import numpy as np


def quad_masses(U, V, L, CS, CT, u, v, l, s0, s1, t0, t1):
    """Masses (range queries) of the four quads of [s0, s1) x [t0, t1)."""
    W = U[u] * V[v] * L[l]
    sm, tm = (s0 + s1) // 2, (t0 + t1) // 2
    dS = (CS[sm] - CS[s0], CS[s1] - CS[sm])
    dT = (CT[tm] - CT[t0], CT[t1] - CT[tm])
    return np.array([np.sum(W * dS[a] * dT[b]) for a in (0, 1) for b in (0, 1)])


def sample_one(U, V, L, CS, CT, u, v, l, rnd):
    """One sample for footprint (u, v, l); rnd has log2(N) + 2 entries."""
    N = CS.shape[0] - 1
    levels = int(round(np.log2(N)))
    s0, s1, t0, t1 = 0, N, 0, N
    prob = 1.0
    for k in range(levels):
        m = np.maximum(quad_masses(U, V, L, CS, CT, u, v, l, s0, s1, t0, t1), 0.0)
        total = ((m[0] + m[1]) + m[2]) + m[3]
        if not total > 0.0:
            return (0.0, 0.0), 0.0, (-1, -1)
        target = rnd[k] * total
        run = 0.0
        pick = 3
        for i in range(4):
            run += m[i]
            if target < run:
                pick = i
                break
        while m[pick] <= 0.0:          # never land on an empty quad at the top of the range
            pick -= 1
        prob *= m[pick] / total
        sm, tm = (s0 + s1) // 2, (t0 + t1) // 2
        if pick >= 2:
            s0 = sm
        else:
            s1 = sm
        if pick % 2 == 1:
            t0 = tm
        else:
            t1 = tm
    w = 2.0 / N
    h = (-1.0 + (s0 + rnd[levels]) * w, -1.0 + (t0 + rnd[levels + 1]) * w)
    return h, prob / (w * w), (s0, t0)


def sample(U, V, L, CS, CT, uvl, rnd):
    """Samples for records uvl [n][3] (integer footprints, wrapped/clamped
    like the range query) with draws rnd [n][log2(N) + 2]."""
    U, V, L, CS, CT = (np.asarray(x, dtype=np.float64) for x in (U, V, L, CS, CT))
    nu, nv, nl = U.shape[0], V.shape[0], L.shape[0]
    uvl = np.asarray(uvl, dtype=np.int64)
    rnd = np.asarray(rnd, dtype=np.float64)
    n = uvl.shape[0]
    h = np.zeros((n, 2))
    pdf = np.zeros(n)
    bins = np.zeros((n, 2), dtype=np.int64)
    for i in range(n):
        u = int(np.mod(uvl[i, 0], nu))
        v = int(np.mod(uvl[i, 1], nv))
        l = int(np.clip(uvl[i, 2], 0, nl - 1))
        hh, p, b = sample_one(U, V, L, CS, CT, u, v, l, rnd[i])
        h[i], pdf[i], bins[i] = hh, p, b
    return h, pdf, bins
