"""GPU parity: the texel-space MTTKRP and CP-ALS (T never formed) against the
FP64 oracle on the materialised tensor, and against the dense GPU path."""
import numpy as np
import pytest
import torch

import gen
from oracle import cp_als, ndf

pytestmark = pytest.mark.gpu

import paper_2109_14807_amd as G  # noqa: E402


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _signed_factors(dims, R, seed):
    rng = np.random.default_rng(seed)
    nu, nv, nl, N = dims
    return [rng.standard_normal((n, R)) for n in (nu, nv, nl, N, N)]


@pytest.mark.parametrize("R", [16, 256])
def test_mttkrp_texel_every_mode_matches_oracle(R):
    """24 x 20 map (footprints wrap on both axes), 5 levels, N = 16, signed factors."""
    nu, nv, nl, N, sigma = 24, 20, 5, 16, 0.03
    nxy = gen.flake_map(nu, nv, 15, 0.2, 31)
    T = ndf.ndf_bruteforce(nxy, N, sigma, nl)
    A = _signed_factors((nu, nv, nl, N), R, 32 + R)
    d = G.desc_of(nu, nv, nl, N, sigma)
    ws = G.texel_workspace(d, R)
    for mode in range(5):
        print(f"mttkrp_texel R={R} mode={mode}", flush=True)
        got = G.mttkrp_texel(nxy, d, A, mode, workspace=ws).cpu().numpy()
        want = cp_als.mttkrp(T, A, mode)
        assert _rel(got, want) < 1e-12, (R, mode, _rel(got, want))


def test_mttkrp_texel_equals_dense_gpu_c1():
    """The 64 x 64, N = 32, 5-level workload: texel form against the matrix-core
    passes over the built FP64 tensor."""
    cfg = gen.config("c1")
    nxy = gen.normal_map(cfg)
    d = G.desc_of(cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.sigma)
    T = G.build_tensor(nxy, d, dtype=torch.float64)
    A = gen.als_init(cfg)
    for mode in range(5):
        dense = G.mttkrp(T, d, A, mode).cpu().numpy()
        tex = G.mttkrp_texel(nxy, d, A, mode).cpu().numpy()
        assert _rel(tex, dense) < 1e-12, (mode, _rel(tex, dense))


def test_cp_als_texel_two_sweeps_match_oracle():
    cfg = gen.config("c1")
    nxy = gen.normal_map(cfg)
    T = ndf.ndf_bruteforce(nxy, cfg.nbins, cfg.sigma, cfg.nlevels)
    init = gen.als_init(cfg)
    d = G.desc_of(cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.sigma)
    for iters in (1, 2):
        ref = cp_als.cp_als(T, init, iters=iters)
        res = G.cp_als_texel(nxy, d, init, iters, normT2=float(np.sum(T * T)))
        F = [f.cpu().numpy() for f in res.factors]
        for m in range(5):
            assert _rel(F[m], ref["factors"][m]) < 1e-10, (iters, m)
        assert np.max(np.abs(res.fits.cpu().numpy() - ref["fits"])) < 1e-10
        info = res.info.cpu().numpy()
        assert info[0] == iters and info[1] == 0


def test_cp_als_texel_fifty_sweeps_match_dense_gpu():
    """32 x 32 flake map, N = 16, 4 levels, rank 16: fit histories of the texel
    and dense GPU paths over 50 sweeps, and the stopping rule."""
    nxy = gen.flake_map(32, 32, 60, 0.15, 77)
    d = G.desc_of(32, 32, 4, 16, 0.02)
    T = G.build_tensor(nxy, d, dtype=torch.float64)
    normT2 = float((T * T).sum())
    init = gen.als_init((32, 32, 4, 16), rank=16, seed=78)
    dense = G.cp_als(T, d, init, 50).fits.cpu().numpy()
    tex = G.cp_als_texel(nxy, d, init, 50, normT2=normT2).fits.cpu().numpy()
    assert np.max(np.abs(tex - dense)) < 1e-9
    # a tolerance between two consecutive fit changes, so that the stop is early
    # and not decided by rounding
    step = np.abs(np.diff(dense))
    k = int(np.argmax(step < 0.5 * step[0]))
    assert k > 0
    tol = float(np.sqrt(step[k] * step[k - 1]))     # step[k] < tol < step[k - 1]
    stop_d = G.cp_als(T, d, init, 50, tol=tol)
    stop_t = G.cp_als_texel(nxy, d, init, 50, tol=tol, normT2=normT2)
    assert int(stop_t.info[0]) == int(stop_d.info[0]) < 50


def test_cp_als_texel_without_norm_gives_nan_fits():
    nxy = gen.flake_map(16, 16, 10, 0.2, 3)
    d = G.desc_of(16, 16, 3, 16, 0.03)
    init = gen.als_init((16, 16, 3, 16), rank=16, seed=4)
    res = G.cp_als_texel(nxy, d, init, 2)
    assert np.all(np.isnan(res.fits.cpu().numpy()))
    with pytest.raises(G.GlintError):
        G.cp_als_texel(nxy, d, init, 2, tol=1e-3)


def test_cp_als_texel_rank256_global_cholesky():
    """Rank 256 takes the Cholesky in global memory: one sweep against the oracle
    (fit and reconstruction; the factors of so wide a rank are ill-conditioned)."""
    nu, nv, nl, N, sigma = 32, 32, 4, 32, 0.02
    nxy = gen.flake_map(nu, nv, 40, 0.2, 256)
    T = ndf.ndf_bruteforce(nxy, N, sigma, nl)
    init = gen.als_init((nu, nv, nl, N), rank=256, seed=257)
    ref = cp_als.cp_als(T, init, iters=1)
    d = G.desc_of(nu, nv, nl, N, sigma)
    res = G.cp_als_texel(nxy, d, init, 1, normT2=float(np.sum(T * T)))
    info = res.info.cpu().numpy()
    assert info[1] == ref["fallbacks"]
    assert abs(float(res.fits[0]) - ref["fits"][0]) < 1e-8
    rec = cp_als.reconstruct(*[f.cpu().numpy() for f in res.factors])
    rec_ref = cp_als.reconstruct(*ref["factors"])
    assert _rel(rec, rec_ref) < 1e-6


def test_cp_als_texel_breakdown_rule_matches_oracle():
    """Duplicate initial columns make every Hadamard Gram singular: every update
    takes the eigen pseudo-inverse, in the texel path and the dense GPU path
    as in the oracle (factors to 1e-9 after two sweeps)."""
    nxy = gen.flake_map(16, 16, 9, 0.25, 5)
    d = G.desc_of(16, 16, 2, 16, 0.05)
    rng = np.random.default_rng(4)
    init = [rng.random((n, 16)) for n in (16, 16, 2, 16, 16)]
    for a in init:
        a[:, 1] = a[:, 0]
    Tn = ndf.ndf_bruteforce(nxy, 16, 0.05, 2)
    ref = cp_als.cp_als(Tn, init, iters=2)
    T = G.build_tensor(nxy, d, dtype=torch.float64)
    dense = G.cp_als(T, d, init, 2)
    tex = G.cp_als_texel(nxy, d, init, 2, normT2=float((T * T).sum()))
    assert int(tex.info[1]) == int(dense.info[1]) == ref["fallbacks"] == 10
    for a, b, c in zip(tex.factors, dense.factors, ref["factors"]):
        assert _rel(a.cpu().numpy(), c) < 1e-9 and _rel(b.cpu().numpy(), c) < 1e-9


def test_cp_als_texel_rank256_singular_gram_matches_oracle():
    """Rank 256 with a duplicated initial column: one exact null eigenvalue in
    every Hadamard Gram, the rest above 3.6e-4 of the largest (a clean gap at
    the 1e-12 cutoff, so the pseudo-inverse is well defined): one sweep of
    the texel path against the oracle."""
    nu, nv, nl, N, sigma = 32, 32, 4, 32, 0.02
    nxy = gen.flake_map(nu, nv, 40, 0.2, 256)
    T = ndf.ndf_bruteforce(nxy, N, sigma, nl)
    init = gen.als_init((nu, nv, nl, N), rank=256, seed=257)
    for a in init:
        a[:, 1] = a[:, 0]
    ref = cp_als.cp_als(T, init, iters=1)
    d = G.desc_of(nu, nv, nl, N, sigma)
    res = G.cp_als_texel(nxy, d, init, 1, normT2=float(np.sum(T * T)))
    assert int(res.info[1]) == ref["fallbacks"] == 5
    for m, f in enumerate(res.factors):
        assert _rel(f.cpu().numpy(), ref["factors"][m]) < 1e-9, m
    assert abs(float(res.fits[0]) - ref["fits"][0]) < 1e-9


# The maps the 2048^2 and 4096^2 workloads fit have 10 and 12 levels, which run
# the kernels instantiated for up to 12 levels; the tests above reach at most 8.
# A 256^2 map with 9 levels and a 512^2 map with 10 levels take those
# instantiations at the workloads' bin counts and ranks (N 64 with rank 128;
# N 128 with rank 256, the largest LDS tiles), and a 2048^2 map at rank 16
# runs all 12 levels (no padding level).
PYRAMID_CASES = [
    # (side, levels, N, R, sites)
    (256, 9, 64, 128, 1200),
    (512, 10, 64, 128, 4800),
    (256, 9, 128, 256, 1200),
    (2048, 12, 16, 16, 20000),
]


@pytest.mark.parametrize("side,nl,N,R,sites", PYRAMID_CASES)
def test_mttkrp_texel_pyramid_scale_matches_oracle(side, nl, N, R, sites):
    sigma = 0.005 if N >= 64 else 0.02
    nxy = gen.flake_map(side, side, sites, 0.2, 1000 + side + nl)
    ms, mt = ndf.texel_masses(nxy, N, sigma)
    rng = np.random.default_rng(side + R)
    A = [rng.standard_normal((n, R)) for n in (side, side, nl, N, N)]
    d = G.desc_of(side, side, nl, N, sigma)
    ws = G.texel_workspace(d, R)
    for mode in range(5):
        print(f"mttkrp_texel {side}^2 levels={nl} N={N} R={R} mode={mode}", flush=True)
        got = G.mttkrp_texel(nxy, d, A, mode, workspace=ws).cpu().numpy()
        want = cp_als.mttkrp_structured(ms, mt, nl, A, mode)
        assert _rel(got, want) < 1e-12, (mode, _rel(got, want))


def test_cp_als_texel_pyramid_scale_two_sweeps_match_oracle():
    """256^2 flake map, 9 levels, N 64, rank 128 (the 2048^2 workloads' rank and
    bins): factors after one and two sweeps against the oracle's texel-space ALS
    from the same start (perturbing that start by 1e-15 moves the oracle's own
    factors by about 1e-13 here, so 1e-10 is far above the rounding spread)."""
    side, nl, N, R, sigma = 256, 9, 64, 128, 0.005
    nxy = gen.flake_map(side, side, 1200, 0.2, 41)
    ms, mt = ndf.texel_masses(nxy, N, sigma)
    init = gen.als_init((side, side, nl, N), rank=R, seed=42)
    d = G.desc_of(side, side, nl, N, sigma)
    for iters in (1, 2):
        print(f"cp_als_texel {side}^2 levels={nl} R={R} sweeps={iters}", flush=True)
        ref = cp_als.cp_als_texel(ms, mt, nl, init, iters=iters)
        res = G.cp_als_texel(nxy, d, init, iters)
        info = res.info.cpu().numpy()
        assert info[0] == iters and info[1] == ref["fallbacks"] == 0
        for m, f in enumerate(res.factors):
            assert _rel(f.cpu().numpy(), ref["factors"][m]) < 1e-10, (iters, m)
