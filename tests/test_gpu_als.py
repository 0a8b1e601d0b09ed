"""GPU parity: CP-ALS on the matrix cores against the plain FP64 oracle from
the identical initial factors (through the C ABI)."""
import numpy as np
import pytest
import torch

import gen
from oracle import cp_als, ndf

pytestmark = pytest.mark.gpu

import paper_2109_14807_amd as G  # noqa: E402


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _run(T, dims, init, iters, dtype=torch.float64, tol=0.0):
    nu, nv, nl, N = dims
    d = G.desc_of(nu, nv, nl, N, 0.01)
    Tt = torch.tensor(np.ascontiguousarray(T), dtype=dtype, device="cuda")
    res = G.cp_als(Tt, d, init, iters, tol=tol)
    F = [f.cpu().numpy() for f in res.factors]
    return F, res.fits.cpu().numpy(), res.info.cpu().numpy()


@pytest.fixture(scope="module")
def c1_tensor():
    cfg = gen.config("c1")
    nxy = gen.normal_map(cfg)
    return cfg, ndf.ndf_bruteforce(nxy, cfg.nbins, cfg.sigma, cfg.nlevels)


def test_c1_fp64_two_sweeps_match_oracle(c1_tensor):
    cfg, T = c1_tensor
    init = gen.als_init(cfg)
    for iters in (1, 2):
        ref = cp_als.cp_als(T, init, iters=iters)
        F, fits, info = _run(T, (cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins), init, iters)
        for m in range(5):
            assert _rel(F[m], ref["factors"][m]) < 1e-10, (iters, m)
        assert np.max(np.abs(fits - ref["fits"])) < 1e-10
        assert info[0] == iters and info[1] == 0


def test_c1_fp32_mttkrp_first_sweep(c1_tensor):
    cfg, T = c1_tensor
    T32 = T.astype(np.float32)
    init = gen.als_init(cfg)
    ref = cp_als.cp_als(T32.astype(np.float64), init, iters=1)
    F, fits, _ = _run(T32, (cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins), init, 1, dtype=torch.float32)
    for m in range(5):
        assert _rel(F[m], ref["factors"][m]) < 1e-4, m
    assert abs(fits[0] - ref["fits"][0]) < 1e-4


def test_small_map_fifty_sweeps_fp32_and_fp64():
    """32x32 flake map, N = 16, 4 levels, rank 16: the whole 50-sweep fit history."""
    nxy = gen.flake_map(32, 32, 60, 0.15, 77)
    T = ndf.ndf_bruteforce(nxy, 16, 0.02, 4)
    init = gen.als_init((32, 32, 4, 16), rank=16, seed=78)
    ref = cp_als.cp_als(T, init, iters=50)
    _, fits64, _ = _run(T, (32, 32, 4, 16), init, 50)
    assert np.max(np.abs(fits64 - ref["fits"])) < 1e-8
    _, fits32, _ = _run(T.astype(np.float32), (32, 32, 4, 16), init, 50, dtype=torch.float32)
    assert np.max(np.abs(fits32 - ref["fits"])) < 1e-4


@pytest.mark.parametrize("R", [32, 64, 128])
def test_ragged_cells_and_ranks(R):
    """12 x 20 map, 3 levels: 720 cells, not a multiple of the 32-cell tiles.
    Ranks above the smaller modes make the Grams ill-conditioned, so the
    reconstructions and fits are compared rather than the factors."""
    nxy = gen.flake_map(12, 20, 9, 0.25, 5)
    T = ndf.ndf_bruteforce(nxy, 16, 0.05, 3)
    init = gen.als_init((12, 20, 3, 16), rank=R, seed=R)
    ref = cp_als.cp_als(T, init, iters=2)
    F, fits, info = _run(T, (12, 20, 3, 16), init, 2)
    assert info[1] == 0 and ref["fallbacks"] == 0
    assert _rel(cp_als.reconstruct(*F), cp_als.reconstruct(*ref["factors"])) < 1e-8
    assert np.max(np.abs(fits - ref["fits"])) < 1e-9


def test_exact_rank16_tensor_recovered_like_the_oracle():
    rng = np.random.default_rng(2)
    dims = (24, 20, 5, 16, 16)
    true = [rng.standard_normal((d, 16)) for d in dims]
    T = cp_als.reconstruct(*true)
    init = tuple(rng.random((d, 16)) for d in dims)
    ref = cp_als.cp_als(T, init, iters=150)
    F, fits, _ = _run(T, dims[:4], init, 150)
    err_ref = np.linalg.norm(cp_als.reconstruct(*ref["factors"]) - T) / np.linalg.norm(T)
    err = np.linalg.norm(cp_als.reconstruct(*F) - T) / np.linalg.norm(T)
    assert err_ref < 1e-8          # the oracle recovers it from this start
    assert err < 1e-8


def test_tolerance_stops_early(c1_tensor):
    cfg, T = c1_tensor
    init = gen.als_init(cfg)
    F, fits, info = _run(T, (cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins), init, 40, tol=1e-3)
    ref = cp_als.cp_als(T, init, iters=40, tol=1e-3)
    assert info[0] == ref["sweeps"] < 40
    assert np.all(fits[info[0]:] == fits[info[0] - 1])
    assert np.max(np.abs(fits[:info[0]] - ref["fits"])) < 1e-9


def test_singular_gram_takes_the_pseudo_inverse_like_the_oracle():
    """Duplicate initial columns make every Hadamard Gram singular: each update
    fails the Cholesky pivot test and is solved by the eigen pseudo-inverse,
    on the GPU (Jacobi in one workgroup) as in the oracle (LAPACK eigh).  The
    two columns stay equal only up to rounding, which the sweeps amplify
    (their difference grows from 1e-13 to 1e-11 over two sweeps), so the
    factors are compared to 1e-9 after one and two sweeps (a Jacobi model of
    the GPU's rule differs from the oracle by 1e-11 here)."""
    nxy = gen.flake_map(16, 16, 9, 0.25, 5)
    T = ndf.ndf_bruteforce(nxy, 16, 0.05, 2)
    rng = np.random.default_rng(4)
    init = [rng.random((d, 16)) for d in (16, 16, 2, 16, 16)]
    for a in init:
        a[:, 1] = a[:, 0]
    for iters in (1, 2):
        F, fits, info = _run(T, (16, 16, 2, 16), init, iters)
        ref = cp_als.cp_als(T, init, iters=iters)
        assert info[1] == ref["fallbacks"] == 5 * iters
        for m in range(5):
            assert _rel(F[m], ref["factors"][m]) < 1e-9, (iters, m, _rel(F[m], ref["factors"][m]))
        assert np.max(np.abs(fits - ref["fits"])) < 1e-9


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("R", [16, 64])
def test_mttkrp_every_mode_matches_oracle(dtype, R):
    nxy = gen.flake_map(16, 24, 12, 0.2, 1234)
    T = ndf.ndf_bruteforce(nxy, 16, 0.03, 3)
    if dtype == torch.float32:
        T = T.astype(np.float32).astype(np.float64)
    F = gen.als_init((16, 24, 3, 16), rank=R, seed=99)
    d = G.desc_of(16, 24, 3, 16, 0.03)
    Tt = torch.tensor(T, dtype=dtype, device="cuda")
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    for mode in range(5):
        got = G.mttkrp(Tt, d, F, mode).cpu().numpy()
        want = cp_als.mttkrp(T, F, mode)
        assert _rel(got, want) < tol, (mode, _rel(got, want))
