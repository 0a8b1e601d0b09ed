"""Pins of the Wang-tile oracle (Sec. 5.5): the implicit per-tile sum equals
the NDF of the explicitly assembled map (the paper's Fig. NDFwangTiles check),
neighbouring cells agree on their shared edges, the colours are balanced,
and the CP route equals box sums of the tiles' reconstructions."""
import numpy as np

import gen
from oracle import cp_als, ndf, query, wang


def _tiles(rng, n, S):
    return np.stack([gen.flake_map(S, S, 6, 0.3, int(rng.integers(1 << 30))) for _ in range(n)]).astype(np.float64)


def test_implicit_tiles_equal_the_explicit_map():
    rng = np.random.default_rng(1)
    S, m, nl, N, sigma, seed = 8, 4, 4, 8, 0.05, 12345
    etl = rng.permutation(16)
    tiles = _tiles(rng, 16, S)
    tens = wang.tile_tensors(tiles, m, N, sigma, nl)
    # a 4x4-cell window starting at cell (-2, -1); footprints kept inside it
    i0, j0, ni, nj = -2, -1, 4, 4
    window = wang.explicit_map(tiles, seed, etl, i0, ni, j0, nj)
    n = 400
    l = rng.integers(0, nl, n)
    k = 1 << l
    x = i0 * S + k // 2 + rng.integers(0, ni * S - k + 1)
    y = j0 * S + k // 2 + rng.integers(0, nj * S - k + 1)
    a = rng.integers(0, N + 1, (n, 2))
    b = rng.integers(0, N + 1, (n, 2))
    q = np.stack([x, y, l, a.min(1), a.max(1), b.min(1), b.max(1)], axis=1)
    implicit = wang.wang_box_sum(tens, q, S, m, seed, etl)
    ql = q.copy()
    ql[:, 0] -= i0 * S
    ql[:, 1] -= j0 * S
    explicit = ndf.range_bruteforce(window, N, sigma, nl, ql)
    assert np.max(np.abs(implicit - explicit)) < 1e-12
    assert np.sum(implicit > 0) > n // 2
    # footprints that straddle cells exercise the sum over tiles
    assert sum(len(wang.cells_of(int(xx), int(yy), int(ll), S)) > 1 for xx, yy, ll in zip(x, y, l)) > n // 4


def test_neighbouring_cells_share_edge_colours():
    etl = np.arange(16)                     # identity: the tile index is the edge code
    seed = 99
    for i in range(-5, 5):
        for j in range(-5, 5):
            c, r, d = (wang.cell_tile(seed, etl, i, j), wang.cell_tile(seed, etl, i + 1, j),
                       wang.cell_tile(seed, etl, i, j + 1))
            assert (c >> 2) & 1 == r & 1          # my right edge is my right neighbour's left edge
            assert (c >> 1) & 1 == (d >> 3) & 1   # my bottom edge is the top edge of the cell below


def test_colours_are_balanced_and_all_tiles_appear():
    etl = np.arange(16)
    cols = np.array([wang.vertex_colours(7, i, j) for i in range(-50, 50) for j in range(-50, 50)])
    assert abs(cols.mean() - 0.5) < 0.02
    seen = {wang.cell_tile(7, etl, i, j) for i in range(-20, 20) for j in range(-20, 20)}
    assert seen == set(range(16))


def test_cp_route_equals_box_sums_of_the_reconstructions():
    rng = np.random.default_rng(4)
    S, m, nl, N, R, seed = 8, 4, 3, 8, 3, 5
    P = S + 2 * m
    etl = rng.permutation(16)
    F = [[rng.random((P, R)), rng.random((P, R)), rng.random((nl, R)), rng.random((N, R)), rng.random((N, R))]
         for _ in range(16)]
    tens = [cp_als.reconstruct(*f) for f in F]
    fac = [(f[0], f[1], f[2], query.cumulative(f[3]), query.cumulative(f[4])) for f in F]
    n = 200
    q = np.stack([rng.integers(-40, 40, n), rng.integers(-40, 40, n), rng.integers(-1, nl + 1, n),
                  rng.integers(-2, 4, n), rng.integers(4, N + 3, n), rng.integers(0, 4, n),
                  rng.integers(4, N + 1, n)], axis=1)
    got = wang.wang_range_query(fac, q, S, m, seed, etl)
    want = wang.wang_box_sum(tens, q, S, m, seed, etl)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_absent_texels_carry_no_mass():
    """A footprint's total mass is (present texels) / k^2 exactly, however the
    absent (non-finite) texels are placed."""
    rng = np.random.default_rng(8)
    nu, nv, nl, N = 12, 10, 4, 16
    nxy = rng.uniform(-0.7, 0.7, (nu, nv, 2))
    absent = rng.random((nu, nv)) < 0.3
    nxy[absent, 0] = np.nan
    nxy[absent & (rng.random((nu, nv)) < 0.5), 1] = np.inf
    T = ndf.ndf_bruteforce(nxy, N, 0.04, nl)
    for l in range(nl):
        k = 1 << l
        for u in range(nu):
            for v in range(nv):
                xs = np.mod(u + ndf.footprint_offsets(k), nu)
                ys = np.mod(v + ndf.footprint_offsets(k), nv)
                present = k * k - absent[np.ix_(xs, ys)].sum()
                assert abs(T[u, v, l].sum() - present / (k * k)) < 1e-12
    q = np.array([[3, 4, 2, 0, N, 0, N], [0, 0, 0, 0, N, 0, N]])
    assert np.allclose(ndf.range_bruteforce(nxy, N, 0.04, nl, q), ndf.box_sum(T, q), atol=1e-13)
