"""GPU parity: Wang-tile synthesis (Sec. 5.5) against the FP64 oracle - tile
tensors over a margin of absent texels, and range queries on the
synthesized plane summed over the tiles a footprint overlaps."""
import numpy as np
import pytest
import torch

import gen
from oracle import query, wang

pytestmark = pytest.mark.gpu

import paper_2109_14807_amd as G  # noqa: E402

S, M, NL, N, SIGMA, SEED, R = 16, 4, 4, 16, 0.04, 2024, 16


def _tiles(rng, n):
    return np.stack([gen.flake_map(S, S, 10, 0.3, int(rng.integers(1 << 30))) for _ in range(n)])


def _setup():
    rng = np.random.default_rng(9)
    etl = rng.permutation(16)
    tiles = _tiles(rng, 16)
    d = G.desc_of(S + 2 * M, S + 2 * M, NL, N, SIGMA)
    return rng, etl, tiles, d


def test_tile_tensors_with_absent_margins_match_oracle():
    """The build over a tile padded with NaN normals (absent texels) against
    the oracle's brute force, every tile: partial footprints near the edge."""
    rng, etl, tiles, d = _setup()
    want = wang.tile_tensors(tiles.astype(np.float64), M, N, SIGMA, NL)
    for t in range(16):
        pt = wang.padded_tile(tiles[t].astype(np.float64), M).astype(np.float32)
        T = G.build_tensor(torch.from_numpy(pt).cuda(), d, dtype=torch.float64).cpu().numpy()
        assert np.max(np.abs(T - want[t])) < 1e-12, t


def test_query_wang_matches_oracle_on_the_same_tables():
    rng, etl, tiles, d = _setup()
    fac64 = []
    for t in range(16):
        pt = wang.padded_tile(tiles[t].astype(np.float64), M).astype(np.float32)
        T = G.build_tensor(torch.from_numpy(pt).cuda(), d, dtype=torch.float64)
        init = gen.als_init((S + 2 * M, S + 2 * M, NL, N), rank=R, seed=100 + t)
        res = G.cp_als(T, d, init, 10)
        fac64.append([f.cpu().numpy() for f in res.factors])
    tab = G.wang_tables(fac64, S, M, SEED, etl)
    # the oracle on the stored values: FP32 factors, FP64 prefix sums of the FP32 S, T rounded to FP32
    fac = [(f[0].astype(np.float32).astype(np.float64), f[1].astype(np.float32).astype(np.float64),
            f[2].astype(np.float32).astype(np.float64),
            query.cumulative(f[3].astype(np.float32)).astype(np.float32).astype(np.float64),
            query.cumulative(f[4].astype(np.float32)).astype(np.float32).astype(np.float64)) for f in fac64]
    n = 3000
    q = np.stack([rng.integers(-1000, 1000, n), rng.integers(-(1 << 30), 1 << 30, n), rng.integers(-1, NL + 2, n),
                  rng.integers(-2, N // 2, n), rng.integers(N // 2, N + 3, n), rng.integers(0, N // 2, n),
                  rng.integers(N // 2, N + 1, n)], axis=1).astype(np.int32)
    q[: n // 10, 4] = q[: n // 10, 3]                       # empty boxes
    got = G.query_wang(tab, torch.from_numpy(q)).cpu().numpy().astype(np.float64)
    want = wang.wang_range_query(fac, q, S, M, SEED, etl)
    # the scale of the FP32 evaluation's error: the magnitudes of every tile's rank terms, summed
    mag = np.zeros(n)
    for i, recs in enumerate(wang.local_records(q, S, M, NL, N, SEED, etl)):
        for t, r in recs:
            mag[i] += float(query.range_query_term_magnitude(*fac[t], np.asarray([r]))[0])
    assert np.all(np.abs(got - want) <= 1e-5 * mag + 1e-30), float(np.max(np.abs(got - want) / np.maximum(mag, 1e-300)))
    assert np.all(got[: n // 10] == 0.0)
    # and the result approximates the exact implicit NDF (CP error only)
    tens = wang.tile_tensors(tiles.astype(np.float64), M, N, SIGMA, NL)
    exact = wang.wang_box_sum(tens, q[:500], S, M, SEED, etl)
    assert np.linalg.norm(got[:500] - exact) < 0.5 * np.linalg.norm(exact)


def test_query_wang_argument_errors():
    rng, etl, tiles, d = _setup()
    F = [[np.ones((S + 2 * M, 4)), np.ones((S + 2 * M, 4)), np.ones((NL, 4)), np.ones((N, 4)), np.ones((N, 4))]] * 16
    tab = G.wang_tables(F, S, M, SEED, etl)
    q = torch.zeros((1, 7), dtype=torch.int32)
    assert G.query_wang(tab, torch.zeros((0, 7), dtype=torch.int32)).numel() == 0
    bad = G.wang_tables(F, S, 1, SEED, etl)            # margin below half the largest footprint
    with pytest.raises(G.GlintError):
        G.query_wang(bad, q)
    Fs = [[np.ones((4 + 2 * M, 4)), np.ones((4 + 2 * M, 4)), np.ones((NL, 4)), np.ones((N, 4)), np.ones((N, 4))]] * 16
    bad = G.wang_tables(Fs, 4, M, SEED, etl)           # tiles narrower than the largest footprint (8)
    with pytest.raises(G.GlintError):
        G.query_wang(bad, q)
    bad = G.wang_tables(F[:4], S, M, SEED, etl)        # edge_to_tile names tiles that do not exist
    with pytest.raises(G.GlintError):
        G.query_wang(bad, q)
    F2 = [[np.ones((S + 2 * M, 2)), np.ones((S + 2 * M, 2)), np.ones((NL, 2)), np.ones((N, 2)), np.ones((N, 2))]] * 16
    with pytest.raises(G.GlintError):                  # the rank must be a multiple of 4
        G.query_wang(G.wang_tables(F2, S, M, SEED, etl), q)
