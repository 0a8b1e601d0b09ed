"""GPU parity: the clustered layout (Sec. 4.2 practical choices) against the
FP64 oracle -- per-(region, block) CP-ALS, blank blocks, the block-local
summed-area tables and the block-split range query."""
import numpy as np
import pytest
import torch

import gen
from oracle import cluster, ndf

pytestmark = pytest.mark.gpu

import paper_2109_14807_amd as G  # noqa: E402


def _to_dev(T, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(T)).to("cuda", dtype)


def _oracle_shaped(tab, nu, nv, N, t, cs):
    ncu, ncv, nb = nu // cs, nv // cs, N // t
    X = tab.X.cpu().numpy().astype(np.float64).reshape(ncu, ncv, nb, nb, t, -1)
    Y = tab.Y.cpu().numpy().astype(np.float64).reshape(ncu, ncv, nb, nb, t, -1)
    Z = tab.Z.cpu().numpy().astype(np.float64).reshape(ncu, ncv, nb, nb, -1, X.shape[-1])
    blank = tab.blank.cpu().numpy().reshape(ncu, ncv, nb, nb).astype(bool)
    return X, Y, Z, blank


def _block_recon(X, Y, Z):
    return np.einsum("...ar,...br,...fr->...abf", X, Y, Z)


def _fp32_output_bound(X, Y, Z):
    """Per block, a bound on how far storing the factors in FP32 moves the
    reconstruction: each stored entry is off by at most 2^-24 relative, so a
    product of three by at most 3 x 2^-24 of |x||y||z|, and the Frobenius
    norm of component r by at most 3 x 2^-24 ||x_r|| ||y_r|| ||z_r||.  Blocks
    whose components cancel (ALS on a block of rank below R makes such
    pairs) have this sum far above their reconstruction's norm.  Taken with
    4 instead of 3 for the FP64 differences of the two ALS paths."""
    comp = np.sqrt((X ** 2).sum(-2) * (Y ** 2).sum(-2) * (Z ** 2).sum(-2)).sum(-1)
    return 4.0 * 2.0 ** -24 * comp


def _random_queries(rng, n, nu, nv, nl, N):
    q = np.empty((n, 7), dtype=np.int64)
    q[:, 0] = rng.integers(-nu, 2 * nu, n)
    q[:, 1] = rng.integers(-nv, 2 * nv, n)
    q[:, 2] = rng.integers(-1, nl + 1, n)
    a = rng.integers(-3, N + 4, (n, 2))
    b = rng.integers(-3, N + 4, (n, 2))
    q[:, 3], q[:, 4] = a.min(1), a.max(1)
    q[:, 5], q[:, 6] = b.min(1), b.max(1)
    q[: n // 16, 4] = q[: n // 16, 3]          # empty boxes
    return q


def _magnitude(X, Y, Z, q, nl, cs):
    """Upper bound of the sum of |terms| of a clustered query (whole-block
    absolute column sums), the scale of its FP32 rounding."""
    ncu, ncv, nb = X.shape[:3]
    t = X.shape[4]
    qc = ndf.canonical_query(q, ncu * cs, ncv * cs, nl, nb * t)
    ax, ay = np.abs(X).sum(axis=4), np.abs(Y).sum(axis=4)
    out = np.zeros(len(q))
    for i, (u, v, l, slo, shi, tlo, thi) in enumerate(qc):
        if slo >= shi or tlo >= thi:
            continue
        f = ((u % cs) * cs + v % cs) * nl + l
        for zs in range(slo // t, (shi - 1) // t + 1):
            for zt in range(tlo // t, (thi - 1) // t + 1):
                k = (u // cs, v // cs, zs, zt)
                out[i] += float(np.sum(np.abs(Z[k][f]) * ax[k] * ay[k]))
    return out


@pytest.mark.parametrize("R", [4, 8, 16])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_cluster_als_factors_match_oracle_on_a_full_rank_tensor(R, dtype):
    """16 x 16 map, 2 levels, N = 16, blocks of 8 bins, regions of 4 texels,
    uniform random T (every block tensor is well conditioned): factors after
    three sweeps, element by element."""
    rng = np.random.default_rng(100 + R)
    nu, nv, nl, N, t, cs = 16, 16, 2, 16, 8, 4
    T = rng.random((nu, nv, nl, N, N))
    if dtype == torch.float32:
        T = T.astype(np.float32).astype(np.float64)     # the values the kernel reads
    d = G.desc_of(nu, nv, nl, N, 0.02)
    print(f"cluster als R={R} dtype={dtype}", flush=True)
    tab = G.cp_als_clustered(_to_dev(T, dtype), d, t, cs, R, iters=3, seed=5)
    X, Y, Z, blank = _oracle_shaped(tab, nu, nv, N, t, cs)
    Xo, Yo, Zo, blanko, fails = cluster.clustered_cp(T, t, cs, R, iters=3, seed=5)
    assert not blank.any() and not blanko.any()
    info = tab.info.cpu().numpy()
    assert int(info[0]) == fails and int(info[1]) == 0
    assert int(info[3]) == tab.Z.shape[0] * tab.Z.shape[1]               # no blank image block
    assert np.max(np.abs(X - Xo)) < 1e-5
    assert np.max(np.abs(Y - Yo)) < 1e-5
    assert np.max(np.abs(Z - Zo)) < 1e-5 * np.max(np.abs(Zo))


@pytest.mark.parametrize("R", [8, 32])
def test_cluster_als_reconstruction_matches_oracle_c1(R):
    """The 64 x 64 flake workload (N = 32, 5 levels), blocks of 16 bins and
    regions of 8 texels, after 3 and 10 sweeps: blank flags and failure
    counts exactly; per block, the reconstruction within the FP32 storage
    bound of its factors (the factors themselves are not unique where a
    block has rank below R).  The oracle moves by under 1e-8 of a block's
    norm when its input changes by one ulp, so the paths' FP64 differences
    stay far inside that bound.  Rank 32 does not fit the LDS at 320
    footprints and is rejected."""
    cfg = gen.config("c1")
    nxy = gen.normal_map(cfg)
    T = ndf.ndf_bruteforce(nxy, cfg.nbins, cfg.sigma, cfg.nlevels)
    d = G.desc_of(cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.sigma)
    if R == 32:
        with pytest.raises(G.GlintError):
            G.cp_als_clustered(_to_dev(T), d, 16, 8, R, iters=1)
        return
    for iters in (3, 10):
        tab = G.cp_als_clustered(_to_dev(T), d, 16, 8, R, iters=iters, seed=11)
        X, Y, Z, blank = _oracle_shaped(tab, cfg.nu, cfg.nv, cfg.nbins, 16, 8)
        Xo, Yo, Zo, blanko, fails, nkept = cluster.clustered_cp(T, 16, 8, R, iters=iters, seed=11, counts=True)
        assert np.array_equal(blank, blanko)
        info = tab.info.cpu().numpy()
        assert int(info[1]) == int(blanko.sum()) and int(info[0]) == fails
        assert int(info[3]) == int(nkept.sum()) < nkept.size * 320      # blank image blocks thrown away
        err = np.sqrt(np.sum((_block_recon(X, Y, Z) - _block_recon(Xo, Yo, Zo)) ** 2, axis=(-3, -2, -1)))
        bound = _fp32_output_bound(Xo, Yo, Zo)
        ok = ~blanko
        assert np.all(err[ok] <= bound[ok]), (iters, float(np.max(err[ok] / bound[ok])))


def test_cluster_blank_blocks_and_f32_tensor():
    """A tensor that is zero in every third region-and-block tensor and, in
    the others, in 7 of the 32 footprints' image blocks: exact blank flags
    and stacked counts, zero factors and zero Z rows there, and a rank-2 fit
    of the rest (F32 T)."""
    rng = np.random.default_rng(3)
    nu, nv, nl, N, t, cs, R = 8, 8, 2, 16, 8, 4, 4
    ncu, ncv, nb, Lr, t = cluster.layout(nu, nv, nl, N, t, cs)
    T = np.zeros((nu, nv, nl, N, N))
    k = 0
    for cu in range(ncu):
        for cv in range(ncv):
            for zs in range(nb):
                for zt in range(nb):
                    k += 1
                    if k % 3 == 0:
                        continue
                    A, B, C = rng.random((t, 2)), rng.random((t, 2)), rng.random((Lr, 2))
                    C[rng.choice(Lr, 7, replace=False)] = 0.0
                    D = np.einsum("ar,br,fr->fab", A, B, C).reshape(cs, cs, nl, t, t)
                    T[cu * cs:(cu + 1) * cs, cv * cs:(cv + 1) * cs, :, zs * t:(zs + 1) * t,
                      zt * t:(zt + 1) * t] = D
    T = T.astype(np.float32).astype(np.float64)
    d = G.desc_of(nu, nv, nl, N, 0.02)
    tab = G.cp_als_clustered(_to_dev(T, torch.float32), d, t, cs, R, iters=30, seed=9)
    X, Y, Z, blank = _oracle_shaped(tab, nu, nv, N, t, cs)
    Xo, Yo, Zo, blanko, fails, nkept = cluster.clustered_cp(T, t, cs, R, iters=30, seed=9, counts=True)
    assert np.array_equal(blank, blanko) and blank.sum() == k // 3
    assert int(tab.info[1]) == k // 3
    assert int(tab.info[3]) == int(nkept.sum()) == (k - k // 3) * (Lr - 7)
    assert not X[blank].any() and not Y[blank].any() and not Z[blank].any()
    assert np.array_equal(Z == 0, Zo == 0)       # the zero rows of the thrown-away blocks
    err = np.sqrt(np.sum((_block_recon(X, Y, Z) - _block_recon(Xo, Yo, Zo)) ** 2, axis=(-3, -2, -1)))
    assert np.all(err <= _fp32_output_bound(Xo, Yo, Zo) + 1e-300)


@pytest.mark.parametrize("R", [4, 8, 16, 32])
def test_clustered_query_matches_oracle(R):
    """Block-split range queries on the GPU tables against the oracle's query
    over the same (downloaded) factors: wrapped texels, clamped levels and
    bins, empty boxes, boxes over one to four blocks."""
    rng = np.random.default_rng(40 + R)
    nu, nv, nl, N, t, cs = 16, 8, 3, 32, 16, 4
    T = rng.random((nu, nv, nl, N, N))
    d = G.desc_of(nu, nv, nl, N, 0.02)
    tab = G.cp_als_clustered(_to_dev(T), d, t, cs, R, iters=2, seed=1)
    X, Y, Z, _ = _oracle_shaped(tab, nu, nv, N, t, cs)
    # the summed-area tables: FP64 prefix sums of the FP32 factors, rounded once
    CX = tab.CX.cpu().numpy().reshape(X.shape[:4] + (t + 1, R))
    want_cx = np.concatenate([np.zeros(X.shape[:4] + (1, R)), np.cumsum(X, axis=4)], axis=4)
    assert np.array_equal(CX, want_cx.astype(np.float32))
    q = _random_queries(rng, 3000, nu, nv, nl, N)
    got = G.query_clustered(tab, torch.from_numpy(q.astype(np.int32))).cpu().numpy()
    want = cluster.clustered_range_query(X, Y, Z, q, nl, cs)
    mag = _magnitude(X, Y, Z, q, nl, cs)
    assert np.all(np.abs(got - want) <= 1e-5 * mag + 1e-30)
    empty = (np.clip(q[:, 3], 0, N) >= np.clip(q[:, 4], 0, N)) | (np.clip(q[:, 5], 0, N) >= np.clip(q[:, 6], 0, N))
    assert np.all(got[empty] == 0.0)


def test_clustered_layout_accuracy_c1():
    """Rank 8 per region and block on the 64 x 64 workload (20 sweeps): range
    integrals against brute force, as accurate as the oracle's own fit."""
    cfg = gen.config("c1")
    nxy = gen.normal_map(cfg)
    T = ndf.ndf_bruteforce(nxy, cfg.nbins, cfg.sigma, cfg.nlevels)
    q = gen.make_queries(cfg, nxy)
    bf = ndf.box_sum(T, q)
    d = G.desc_of(cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.sigma)
    tab = G.cp_als_clustered(_to_dev(T, torch.float32), d, 16, 8, 8, iters=20, seed=11)
    got = G.query_clustered(tab, torch.from_numpy(q.astype(np.int32))).cpu().numpy()
    e = np.linalg.norm(got - bf) / np.linalg.norm(bf)
    assert e < 0.01, e


def test_clustered_argument_errors():
    d = G.desc_of(16, 16, 2, 16, 0.02)
    T = torch.zeros((16, 16, 2, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(G.GlintError):
        G.cp_als_clustered(T, d, 8, 5, 8, iters=1)       # region side must divide the map
    with pytest.raises(G.GlintError):
        G.cp_als_clustered(T, d, 8, 4, 12, iters=1)      # rank not supported
    with pytest.raises(G.GlintError):
        G.cp_als_clustered(T, d, 6, 4, 8, iters=1)       # block side must divide N
    tab = G.cp_als_clustered(T, d, 32, 4, 8, iters=1)     # t = min(t, N) = 16: all blank
    assert tab.t == 16 and int(tab.info[1]) == tab.X.shape[0] and bool(tab.blank.all())
    out = G.query_clustered(tab, torch.tensor([[0, 0, 0, 0, 16, 0, 16]], dtype=torch.int32))
    assert float(out[0]) == 0.0


def test_clustered_sampling_matches_oracle_and_histogram():
    """Sec. 5.2 on the clustered layout (block by mass, then quads): the same
    draws give the oracle's bins (near-ties aside: at most 1% differ, each a
    sample whose pdf is its bin's normalised mass), the same pdf and
    position on identical bins, and 10^6 samples of one footprint bin like
    the reconstructed NDF image."""
    rng = np.random.default_rng(31)
    nu, nv, nl, N, t, cs, R = 16, 8, 2, 32, 8, 4, 8
    T = rng.random((nu, nv, nl, N, N)) ** 6
    d = G.desc_of(nu, nv, nl, N, 0.02)
    tab = G.cp_als_clustered(_to_dev(T), d, t, cs, R, iters=4, seed=3)
    # non-negative factors (an NDF approximation), re-tabled
    tab.X.abs_(); tab.Y.abs_(); tab.Z.abs_()
    G.clustered_cumulative(tab)
    X, Y, Z, _ = _oracle_shaped(tab, nu, nv, N, t, cs)
    n = 20000
    uvl = np.stack([rng.integers(-nu, 2 * nu, n), rng.integers(0, nv, n), rng.integers(-1, nl + 1, n)], 1)
    rnd = rng.random((n, 6)).astype(np.float32)
    h, pdf, bins = (x.cpu().numpy() for x in G.sample_clustered(tab, torch.from_numpy(uvl.astype(np.int32)),
                                                                 torch.from_numpy(rnd)))
    ho, pdfo, binso = cluster.clustered_sample(X, Y, Z, uvl, rnd.astype(np.float64), nl, cs)
    same = np.all(bins == binso, axis=1)
    assert same.mean() > 0.99, same.mean()
    assert np.allclose(pdf[same], pdfo[same], rtol=1e-4)
    assert np.allclose(h[same], ho[same], atol=1e-6)
    rec = cluster.reconstruct(X, Y, Z, nl, cs)
    w = 2.0 / N
    for i in np.nonzero(~same)[0]:
        u, v, l = int(uvl[i, 0]) % nu, int(uvl[i, 1]) % nv, int(np.clip(uvl[i, 2], 0, nl - 1))
        img = rec[u, v, l]
        assert bins[i, 0] >= 0 and abs(pdf[i] - img[bins[i, 0], bins[i, 1]] / img.sum() / (w * w)) <= 1e-3 * pdf[i]
    # histogram of one footprint
    m = 1_000_000
    one = torch.tensor([[5, 3, 1]], dtype=torch.int32).repeat(m, 1)
    r = torch.rand((m, 6), generator=torch.Generator().manual_seed(4))
    _, pdf1, b1 = (x.cpu().numpy() for x in G.sample_clustered(tab, one, r))
    img = rec[5, 3, 1]
    p = img / img.sum()
    hist = np.zeros((N, N))
    np.add.at(hist, (b1[:, 0], b1[:, 1]), 1.0)
    expect = p * m
    ok = expect > 20
    chi2 = float(np.sum((hist[ok] - expect[ok]) ** 2 / expect[ok]))
    assert chi2 < ok.sum() + 6 * np.sqrt(2 * ok.sum()), (chi2, int(ok.sum()))
    assert np.allclose(pdf1, p[b1[:, 0], b1[:, 1]] / (w * w), rtol=1e-3)
    # no mass: failure
    tab.Z.zero_()
    _, pdf0, b0 = (x.cpu().numpy() for x in G.sample_clustered(tab, torch.tensor([[1, 1, 0]], dtype=torch.int32),
                                                                 torch.rand((1, 6))))
    assert pdf0[0] == 0.0 and tuple(b0[0]) == (-1, -1)
