"""Pins of the clustered-layout oracle (Sec. 4.2 practical choices): the
SplitMix64 generator against its published outputs, exact recovery of a
tensor that is low-rank per region and block (with blank blocks), the
block-split range query against explicit box sums of the reconstruction,
the query on stored (BF16-rounded) summed-area tables against the query of
the per-bin values those tables sum, and the accuracy gain over one global
CP on the 64x64 workload."""
import numpy as np

import gen
from oracle import cluster, cp_als, ndf, quant, query


def test_splitmix64_published_outputs():
    # first outputs of SplitMix64 seeded with 0 (the reference implementation's test vector)
    assert cluster.splitmix64_stream(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    u = cluster.uniform(0, np.arange(3))
    assert np.allclose(u, [x / 2.0 ** 64 for x in (0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F)],
                       rtol=0, atol=2.0 ** -53)


def _blockwise_low_rank(rng, nu, nv, nl, N, t, cs, R, blank_every=3, zero_rows=0):
    """A tensor that is exactly rank R in every (region, block), some blocks
    zero, and in the others `zero_rows` footprints' image blocks zero."""
    T = np.zeros((nu, nv, nl, N, N))
    ncu, ncv, nb, L, t = cluster.layout(nu, nv, nl, N, t, cs)
    k = 0
    for cu in range(ncu):
        for cv in range(ncv):
            for zs in range(nb):
                for zt in range(nb):
                    k += 1
                    if k % blank_every == 0:
                        continue
                    X, Y, Z = rng.standard_normal((t, R)), rng.standard_normal((t, R)), rng.standard_normal((L, R))
                    if zero_rows:
                        Z[rng.choice(L, zero_rows, replace=False)] = 0.0
                    D = np.einsum("ar,br,fr->fab", X, Y, Z).reshape(cs, cs, nl, t, t)
                    T[cu * cs:(cu + 1) * cs, cv * cs:(cv + 1) * cs, :, zs * t:(zs + 1) * t, zt * t:(zt + 1) * t] = D
    return T


def test_exact_recovery_per_region_and_block():
    rng = np.random.default_rng(1)
    nu, nv, nl, N, t, cs, R = 8, 8, 2, 8, 4, 4, 2
    T = _blockwise_low_rank(rng, nu, nv, nl, N, t, cs, R)
    X, Y, Z, blank, fails = cluster.clustered_cp(T, t, cs, R, iters=1000, seed=7)   # ALS swamps are slow
    assert fails == 0
    # blank exactly where the blocks are zero
    for cu in range(2):
        for cv in range(2):
            for zs in range(2):
                for zt in range(2):
                    D = cluster.cluster_tensor(T, cu, cv, zs, zt, t, cs)
                    assert blank[cu, cv, zs, zt] == (not np.any(D))
    rec = cluster.reconstruct(X, Y, Z, nl, cs)
    assert np.linalg.norm(rec - T) <= 1e-7 * np.linalg.norm(T)


def test_blank_image_blocks_are_thrown_away():
    """Sec. 4.2: only the non-blank image blocks of a cluster are stacked.
    Exact recovery still holds, the stacked count L' is the number of
    non-zero footprint blocks, and a blank footprint's Z row is exactly zero."""
    rng = np.random.default_rng(5)
    nu, nv, nl, N, t, cs, R = 8, 8, 2, 8, 4, 4, 2
    T = _blockwise_low_rank(rng, nu, nv, nl, N, t, cs, R, zero_rows=11)
    X, Y, Z, blank, fails, nkept = cluster.clustered_cp(T, t, cs, R, iters=1000, seed=7, counts=True)
    assert fails == 0
    for cu in range(2):
        for cv in range(2):
            for zs in range(2):
                for zt in range(2):
                    D = cluster.cluster_tensor(T, cu, cv, zs, zt, t, cs)
                    nz = np.abs(D).sum(axis=(0, 1)) > 0
                    assert nkept[cu, cv, zs, zt] == nz.sum() and blank[cu, cv, zs, zt] == (not nz.any())
                    if nz.any():
                        assert nz.sum() == 32 - 11
                    assert not Z[cu, cv, zs, zt][~nz].any()
    rec = cluster.reconstruct(X, Y, Z, nl, cs)
    assert np.linalg.norm(rec - T) <= 1e-7 * np.linalg.norm(T)


def test_block_split_query_equals_box_sums_of_the_reconstruction():
    rng = np.random.default_rng(2)
    nu, nv, nl, N, t, cs, R = 8, 4, 3, 16, 4, 4, 3
    T = rng.random((nu, nv, nl, N, N))
    X, Y, Z, blank, _ = cluster.clustered_cp(T, t, cs, R, iters=3, seed=3)
    rec = cluster.reconstruct(X, Y, Z, nl, cs)
    q = np.empty((500, 7), dtype=np.int64)
    q[:, 0] = rng.integers(-8, 16, 500)
    q[:, 1] = rng.integers(0, nv, 500)
    q[:, 2] = rng.integers(-1, nl + 1, 500)
    a = rng.integers(-2, N + 3, (500, 2))
    b = rng.integers(0, N + 1, (500, 2))
    q[:, 3], q[:, 4] = a.min(1), a.max(1)
    q[:, 5], q[:, 6] = b.min(1), b.max(1)
    got = cluster.clustered_range_query(X, Y, Z, q, nl, cs)
    want = ndf.box_sum(rec, q)
    assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.abs(want).max())


def test_query_on_rounded_tables_is_the_query_of_their_bin_differences():
    """Summed-area tables rounded to BF16 (Sec. 4.4 storage) are exactly the
    summed-area tables of their own first differences (BF16 values differ
    and add exactly in FP64), so the query on the stored tables equals the
    plain block-split query of those per-bin values, and both equal the box
    sums of that reconstruction; the FP32-level rounding moves the result
    away from the unrounded query."""
    rng = np.random.default_rng(4)
    nu, nv, nl, N, t, cs, R = 8, 4, 3, 16, 4, 4, 3
    T = rng.random((nu, nv, nl, N, N))
    X, Y, Z, _, _ = cluster.clustered_cp(T, t, cs, R, iters=2, seed=5)
    CXb = quant.bf16_round(cluster.block_cumulative(X)).astype(np.float64)
    CYb = quant.bf16_round(cluster.block_cumulative(Y)).astype(np.float64)
    Zb = quant.bf16_round(Z).astype(np.float64)
    assert np.all(CXb[..., 0, :] == 0.0)
    Xd, Yd = np.diff(CXb, axis=-2), np.diff(CYb, axis=-2)
    assert np.array_equal(cluster.block_cumulative(Xd), CXb)
    q = np.empty((400, 7), dtype=np.int64)
    q[:, 0] = rng.integers(-8, 16, 400)
    q[:, 1] = rng.integers(0, nv, 400)
    q[:, 2] = rng.integers(0, nl, 400)
    a = rng.integers(0, N + 1, (400, 2))
    b = rng.integers(0, N + 1, (400, 2))
    q[:, 3], q[:, 4] = a.min(1), a.max(1)
    q[:, 5], q[:, 6] = b.min(1), b.max(1)
    got = cluster.clustered_range_query_tables(CXb, CYb, Zb, q, nl, cs)
    assert np.array_equal(got, cluster.clustered_range_query(Xd, Yd, Zb, q, nl, cs))
    want = ndf.box_sum(cluster.reconstruct(Xd, Yd, Zb, nl, cs), q)
    assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.abs(want).max())
    plain = cluster.clustered_range_query(X, Y, Z, q, nl, cs)
    assert np.max(np.abs(got - plain)) > 1e-6 * np.abs(plain).max()


def test_clustered_layout_is_far_more_accurate_than_one_global_cp():
    """The 64x64 workload: rank 8 per region and block (3.4% of the tensor's
    size) against brute-force range integrals, and the global rank-16 CP."""
    cfg = gen.config("c1")
    nxy = gen.normal_map(cfg)
    T = ndf.ndf_bruteforce(nxy, cfg.nbins, cfg.sigma, cfg.nlevels)
    q = gen.make_queries(cfg, nxy)
    bf = ndf.box_sum(T, q)
    X, Y, Z, blank, _ = cluster.clustered_cp(T, 16, 8, 8, iters=20, seed=11)
    e_cl = np.linalg.norm(cluster.clustered_range_query(X, Y, Z, q, cfg.nlevels, 8) - bf) / np.linalg.norm(bf)
    res = cp_als.cp_als(T, gen.als_init(cfg), iters=20)
    F = res["factors"]
    e_gl = np.linalg.norm(query.range_query(F[0], F[1], F[2], query.cumulative(F[3]), query.cumulative(F[4]), q)
                          - bf) / np.linalg.norm(bf)
    assert e_cl < 0.01 < 0.1 < e_gl


def test_clustered_sampling_pdf_is_the_normalised_mass_and_histogram_matches():
    """Block choice by mass, then the quad descent inside the block: every
    sample's pdf is its bin's mass over the footprint's total mass (per unit
    area), and 2e5 samples bin like the reconstructed NDF image."""
    rng = np.random.default_rng(21)
    nu, nv, nl, N, t, cs, R = 8, 8, 2, 16, 8, 4, 3
    T = rng.random((nu, nv, nl, N, N)) ** 4
    X, Y, Z, blank, _ = cluster.clustered_cp(T, t, cs, R, iters=5, seed=2)
    X, Y, Z = np.abs(X), np.abs(Y), np.abs(Z)            # a non-negative NDF approximation
    rec = cluster.reconstruct(X, Y, Z, nl, cs)
    u, v, l = 5, 2, 1
    n = 200000
    rnd = rng.random((n, 3 + 3))
    uvl = np.tile([u, v, l], (n, 1))
    h, pdf, bins = cluster.clustered_sample(X, Y, Z, uvl, rnd, nl, cs)
    img = rec[u, v, l]
    p = img / img.sum()
    w = 2.0 / N
    assert np.all(bins >= 0)
    assert np.allclose(pdf, p[bins[:, 0], bins[:, 1]] / (w * w), rtol=1e-9)
    hist = np.zeros((N, N))
    np.add.at(hist, (bins[:, 0], bins[:, 1]), 1.0)
    expect = p * n
    ok = expect > 20
    chi2 = float(np.sum((hist[ok] - expect[ok]) ** 2 / expect[ok]))
    assert chi2 < ok.sum() + 6 * np.sqrt(2 * ok.sum())
    # positions lie in their bins
    assert np.all(np.floor((h + 1.0) / w).astype(int) == bins)
    # a footprint with no mass fails
    Z0 = Z.copy()
    Z0[1, 0, :, :, (2 * cs + 1) * nl + 0] = 0.0
    _, pdf0, b0 = cluster.clustered_sample(X, Y, Z0, [[6, 1, 0]], rnd[:1], nl, cs)
    assert pdf0[0] == 0.0 and tuple(b0[0]) == (-1, -1)


def test_region_block_tensor_equals_the_block_of_the_brute_force_tensor():
    """The region-and-block tensor built from the map (for maps whose T is
    too large) takes exactly the entries of the brute-force T: a 24 x 16 flake
    map, 5 levels (footprints up to 16 texels, wrapping), N = 32 in blocks of
    16 or 8, regions of 4 or 8 texels, every region and block."""
    nxy = gen.flake_map(24, 16, 12, 0.25, 8)
    T = ndf.ndf_bruteforce(nxy, 32, 0.02, 5)
    for t, cs in ((16, 8), (8, 4)):
        ncu, ncv, nb, L, t = cluster.layout(24, 16, 5, 32, t, cs)
        for cu in range(ncu):
            for cv in range(ncv):
                for zs in range(nb):
                    for zt in range(nb):
                        want = cluster.cluster_tensor(T, cu, cv, zs, zt, t, cs)
                        got = cluster.region_block_tensor(nxy, 32, 0.02, 5, t, cs, cu, cv, zs, zt)
                        assert np.max(np.abs(got - want)) <= 1e-14 * max(np.max(np.abs(want)), 1e-300)
