"""Pins of the FP64 oracle's CP-ALS (CPU only)."""
import itertools

import numpy as np
import pytest

import gen
from oracle import cp_als, ndf


def _kruskal(factors, lam=None):
    return cp_als.reconstruct(*factors, lam=lam)


def test_mttkrp_matches_explicit_loops():
    rng = np.random.default_rng(1)
    dims = (3, 2, 2, 3, 2)
    T = rng.standard_normal(dims)
    A = [rng.standard_normal((d, 2)) for d in dims]
    for n in range(5):
        M = cp_als.mttkrp(T, A, n)
        want = np.zeros((dims[n], 2))
        for idx in itertools.product(*[range(d) for d in dims]):
            for r in range(2):
                p = T[idx]
                for m in range(5):
                    if m != n:
                        p *= A[m][idx[m], r]
                want[idx[n], r] += p
        assert np.allclose(M, want, atol=1e-13, rtol=0)


def test_rank1_recovered_in_one_sweep():
    rng = np.random.default_rng(2)
    dims = (64, 64, 5, 32, 32)
    true = [rng.random((d, 1)) + 0.1 for d in dims]
    T = _kruskal(true)
    init = tuple(rng.random((d, 1)) for d in dims)
    res = cp_als.cp_als(T, init, iters=1)
    err = np.linalg.norm(_kruskal(res["factors"]) - T) / np.linalg.norm(T)
    assert err <= 1e-13
    # the Gram-based fit cancels ||T||^2 terms, so it resolves only ~sqrt(eps)
    assert 1.0 - res["fits"][0] <= 1e-7


def _canon(factors, lam):
    """Canonical form: unit columns, largest-|S| entry positive, lambda descending."""
    F = [f.copy() for f in factors]
    lam = lam.copy()
    for r in range(lam.shape[0]):
        for m in range(5):
            nrm = np.linalg.norm(F[m][:, r])
            F[m][:, r] /= nrm
            lam[r] *= nrm
        for m in range(5):
            j = np.argmax(np.abs(F[m][:, r]))
            if F[m][j, r] < 0:
                F[m][:, r] *= -1
                lam[r] *= -1
    order = np.argsort(-np.abs(lam))
    return [f[:, order] for f in F], lam[order]


def test_rank3_recovered_and_factors_unique():
    rng = np.random.default_rng(3)
    dims = (12, 10, 5, 8, 8)
    true = [rng.random((d, 3)) + 0.05 for d in dims]
    T = _kruskal(true)
    init = tuple(rng.random((d, 3)) for d in dims)
    # positive factors are strongly collinear, so ALS needs a few hundred sweeps
    res = cp_als.cp_als(T, init, iters=300)
    err = np.linalg.norm(_kruskal(res["factors"]) - T) / np.linalg.norm(T)
    assert err <= 1e-10
    Fa, la = _canon(res["factors"], np.ones(3))
    Fb, lb = _canon(true, np.ones(3))
    assert np.allclose(la, lb, rtol=1e-8)
    for a, b in zip(Fa, Fb):
        assert np.allclose(a, b, atol=1e-8)


def test_full_rank_tiny_ndf_tensor_reaches_zero_residual():
    """4x4 map, 2 levels, N = 4: dims (4,4,2,4,4) = 512 entries; rank 128 is
    enough for an exact decomposition (the unfolding along u has rank <= 4
    and every mode product is bounded by 128)."""
    nxy = gen.flake_map(4, 4, 6, 0.4, 11)
    T = ndf.ndf_bruteforce(nxy, 4, 0.3, 2)
    init = gen.als_init((4, 4, 2, 4), rank=128, seed=5)
    res = cp_als.cp_als(T, init, iters=500)
    err = np.linalg.norm(_kruskal(res["factors"]) - T) / np.linalg.norm(T)
    assert err <= 1e-8, err


def test_residual_nonincreasing_after_every_mode_update():
    nxy = gen.flake_map(8, 8, 10, 0.3, 4)
    T = ndf.ndf_bruteforce(nxy, 8, 0.08, 3)
    A = [a.copy() for a in gen.als_init((8, 8, 3, 8), rank=6, seed=9)]
    prev = np.inf
    for _ in range(8):
        for n in range(5):
            M = cp_als.mttkrp(T, A, n)
            X, _ = cp_als.solve_gram(M, cp_als.gram_hadamard(A, n))
            A[n] = X            # unnormalised: the model is exactly the LS minimiser
            r = np.linalg.norm(_kruskal(A) - T)
            assert r <= prev * (1 + 1e-12) + 1e-15
            prev = r


def test_fit_formula_matches_explicit_residual():
    nxy = gen.flake_map(8, 8, 10, 0.3, 4)
    T = ndf.ndf_bruteforce(nxy, 8, 0.08, 3)
    init = gen.als_init((8, 8, 3, 8), rank=5, seed=10)
    res = cp_als.cp_als(T, init, iters=4)
    explicit = 1 - np.linalg.norm(_kruskal(res["factors"]) - T) / np.linalg.norm(T)
    assert abs(res["fits"][-1] - explicit) < 1e-10


def test_singular_gram_takes_the_pseudo_inverse():
    """Duplicate columns make the Hadamard Gram singular; the fallback still
    returns the minimum-norm least-squares update."""
    rng = np.random.default_rng(6)
    dims = (5, 4, 3, 4, 4)
    A = [rng.random((d, 2)) for d in dims]
    for m in range(5):
        A[m][:, 1] = A[m][:, 0]
    T = rng.random(dims)
    M = cp_als.mttkrp(T, A, 0)
    X, fb = cp_als.solve_gram(M, cp_als.gram_hadamard(A, 0))
    assert fb
    assert np.allclose(X, M @ np.linalg.pinv(cp_als.gram_hadamard(A, 0)), atol=1e-9)


def test_structured_mttkrp_equals_dense_on_c1():
    cfg = gen.config("c1")
    nxy = gen.normal_map(cfg)
    T = ndf.ndf_bruteforce(nxy, cfg.nbins, cfg.sigma, cfg.nlevels)
    ms, mt = ndf.texel_masses(nxy, cfg.nbins, cfg.sigma)
    A = gen.als_init(cfg, rank=4)
    for n in range(5):
        d = cp_als.mttkrp(T, A, n)
        s = cp_als.mttkrp_structured(ms, mt, cfg.nlevels, A, n)
        assert np.max(np.abs(d - s)) <= 1e-12 * np.max(np.abs(d)), n


def test_texel_als_equals_dense_als_on_c1():
    """The ALS driven by the structured MTTKRP follows the dense ALS on the
    materialised 64x64 tensor sweep for sweep (factors and fits)."""
    cfg = gen.config("c1")
    nxy = gen.normal_map(cfg)
    T = ndf.ndf_bruteforce(nxy, cfg.nbins, cfg.sigma, cfg.nlevels)
    ms, mt = ndf.texel_masses(nxy, cfg.nbins, cfg.sigma)
    init = gen.als_init(cfg)
    dense = cp_als.cp_als(T, init, iters=2)
    tex = cp_als.cp_als_texel(ms, mt, cfg.nlevels, init, iters=2, normT2=float(np.sum(T * T)))
    for a, b in zip(tex["factors"], dense["factors"]):
        assert np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(b))
    assert np.max(np.abs(tex["fits"] - dense["fits"])) < 1e-12
    nofit = cp_als.cp_als_texel(ms, mt, cfg.nlevels, init, iters=1)
    assert np.all(np.isnan(nofit["fits"]))
