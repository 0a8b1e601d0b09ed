"""GPU parity: the clustered layout built straight from the normal map
(glint_cluster_map_index + glint_cp_als_clustered_map; Sec. 4.2 practical
choices) -- the angular blocks' tensors built one at a time, the Z factors
outside the LDS at rank 32, compact Z with a per-footprint row index --
against the FP64 oracle and against the stored-tensor path."""
import numpy as np
import pytest
import torch

import gen
from oracle import cluster, ndf, quant

pytestmark = pytest.mark.gpu

import paper_2109_14807_amd as G  # noqa: E402
from test_gpu_cluster import _block_recon, _fp32_output_bound, _magnitude, _random_queries  # noqa: E402


def _shaped(tab, nu, nv, N, t, cs):
    ncu, ncv, nb = nu // cs, nv // cs, N // t
    X = tab.X.cpu().numpy().astype(np.float64).reshape(ncu, ncv, nb, nb, t, -1)
    Y = tab.Y.cpu().numpy().astype(np.float64).reshape(ncu, ncv, nb, nb, t, -1)
    Z = tab.dense_z().cpu().numpy().astype(np.float64).reshape(ncu, ncv, nb, nb, -1, X.shape[-1])
    blank = tab.blank.cpu().numpy().reshape(ncu, ncv, nb, nb).astype(bool)
    return X, Y, Z, blank


def _c1():
    cfg = gen.config("c1")
    nxy = gen.normal_map(cfg)
    d = G.desc_of(cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.sigma)
    return cfg, nxy, d


def _check_index(tab, nonblank):
    """zidx: -1 exactly at the blank footprints, else base[tensor] + the
    footprint's place among the tensor's non-blank footprints; zbase the
    exclusive running count."""
    zidx = tab.zidx.cpu().numpy()
    zbase = tab.zbase.cpu().numpy()
    nb = nonblank.reshape(zidx.shape)
    assert np.array_equal(zidx >= 0, nb)
    counts = nb.sum(axis=1)
    assert np.array_equal(zbase, np.concatenate([[0], np.cumsum(counts)]))
    want = np.where(nb, zbase[:-1, None] + np.cumsum(nb, axis=1) - 1, -1)
    assert np.array_equal(zidx, want)
    assert tab.Z.shape[0] == max(int(zbase[-1]), 1)


@pytest.mark.parametrize("R", [8, 32])
def test_map_path_matches_oracle_c1(R):
    """The 64 x 64 flake workload (N = 32, 5 levels), blocks of 16 bins,
    regions of 8 texels (320 footprints), FP64 block tensors, 3 sweeps:
    the blank image blocks and the compact index exactly, the blank tensors
    and failure counts exactly, and per block the reconstruction within the
    FP32 storage bound of its factors (as for the stored-tensor path).  At
    rank 32 the Z factors do not fit the LDS and live in the workspace.
    Rank 32 is above the block side (16), so the X and Y Grams are singular
    and only the ridge (1e-10 of the trace) fixes each solve: the oracle
    itself then moves by up to 2.5e-6 of a block's norm when its input
    changes by one ulp (measured on this workload), and the GPU's block
    tensors (level 0 products, then exact level doubling) sit a few ulps
    from the oracle's footprint sums; its reconstructions are compared
    within 1e-4 of the block's norm on top of the storage bound.  At rank 8
    the same perturbation moves the oracle by under 3e-4 of the storage
    bound."""
    cfg, nxy, d = _c1()
    T = ndf.ndf_bruteforce(nxy, cfg.nbins, cfg.sigma, cfg.nlevels)
    print(f"cluster map R={R}", flush=True)
    tab = G.cp_als_clustered_map(torch.from_numpy(nxy), d, 16, 8, R, iters=3, seed=11, dtype=torch.float64)
    X, Y, Z, blank = _shaped(tab, cfg.nu, cfg.nv, cfg.nbins, 16, 8)
    Xo, Yo, Zo, blanko, fails, nkept = cluster.clustered_cp(T, 16, 8, R, iters=3, seed=11, counts=True)
    ncu, ncv, nb, Lr, t = cluster.layout(cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, 16, 8)
    nonblank = np.zeros((ncu, ncv, nb, nb, Lr), dtype=bool)
    dnorm = np.zeros((ncu, ncv, nb, nb))
    for cu in range(ncu):
        for cv in range(ncv):
            for zs in range(nb):
                for zt in range(nb):
                    D = cluster.cluster_tensor(T, cu, cv, zs, zt, t, 8)
                    nonblank[cu, cv, zs, zt, cluster.nonblank_footprints(D)] = True
                    dnorm[cu, cv, zs, zt] = np.linalg.norm(D)
    _check_index(tab, nonblank)
    assert np.array_equal(blank, blanko)
    info = tab.info.cpu().numpy()
    assert int(info[1]) == int(blanko.sum()) and int(info[0]) == fails
    assert int(info[3]) == int(nkept.sum())
    err = np.sqrt(np.sum((_block_recon(X, Y, Z) - _block_recon(Xo, Yo, Zo)) ** 2, axis=(-3, -2, -1)))
    bound = _fp32_output_bound(Xo, Yo, Zo)
    if R > 16:
        bound = bound + 1e-4 * dnorm
    ok = ~blanko
    assert np.all(err[ok] <= bound[ok]), float(np.max(err[ok] / bound[ok]))


@pytest.mark.parametrize("R", [4, 16])
def test_map_path_equals_stored_tensor_path(R):
    """FP32 block tensors from the map against the stored FP32 tensor built
    with level 0 direct (the same kernels, each bin of level 0 one product,
    then exact doubling: the same values), fitted by the dense-layout call:
    identical factors, blank flags and counts, and Z equal to the dense Z
    row for row; queries and samples on the two layouts agree bit for bit."""
    cfg, nxy, d = _c1()
    T = G.build_tensor(nxy, d, torch.float32, direct_levels=1)
    dense = G.cp_als_clustered(T, d, 16, 8, R, iters=4, seed=7)
    del T
    tab = G.cp_als_clustered_map(torch.from_numpy(nxy), d, 16, 8, R, iters=4, seed=7)
    assert torch.equal(tab.X, dense.X) and torch.equal(tab.Y, dense.Y)
    assert torch.equal(tab.blank, dense.blank)
    assert torch.equal(tab.info[:2], dense.info[:2]) and int(tab.info[3]) == int(dense.info[3])
    assert torch.equal(tab.dense_z(), dense.Z)
    _check_index(tab, (dense.Z != 0).any(dim=-1).cpu().numpy())
    rng = np.random.default_rng(5)
    q = torch.from_numpy(_random_queries(rng, 20000, cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins).astype(np.int32))
    assert torch.equal(G.query_clustered(tab, q), G.query_clustered(dense, q))
    n = 4096
    uvl = torch.from_numpy(np.stack([rng.integers(0, cfg.nu, n), rng.integers(0, cfg.nv, n),
                                     rng.integers(0, cfg.nlevels, n)], 1).astype(np.int32))
    rnd = torch.from_numpy(rng.random((n, 4 + 3)).astype(np.float32))
    for a, b in zip(G.sample_clustered(tab, uvl, rnd), G.sample_clustered(dense, uvl, rnd)):
        assert torch.equal(a, b)


def test_map_path_compact_query_matches_oracle_r32():
    """Range queries on the compact rank-32 tables against the oracle's
    block-split query over the same (downloaded, densified) factors."""
    cfg, nxy, d = _c1()
    tab = G.cp_als_clustered_map(torch.from_numpy(nxy), d, 16, 8, 32, iters=2, seed=3)
    X, Y, Z, _ = _shaped(tab, cfg.nu, cfg.nv, cfg.nbins, 16, 8)
    rng = np.random.default_rng(8)
    q = _random_queries(rng, 4000, cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins)
    got = G.query_clustered(tab, torch.from_numpy(q.astype(np.int32))).cpu().numpy()
    want = cluster.clustered_range_query(X, Y, Z, q, cfg.nlevels, 8)
    mag = _magnitude(X, Y, Z, q, cfg.nlevels, 8)
    assert np.all(np.abs(got - want) <= 1e-5 * mag + 1e-30)


def _table_magnitude(CX, CY, Z, q, nl, cs):
    """Sum of the |rank terms| of a block-split query on given tables: the
    scale of its FP32 rounding."""
    ncu, ncv, nb = CX.shape[:3]
    t = CX.shape[4] - 1
    qc = ndf.canonical_query(q, ncu * cs, ncv * cs, nl, nb * t)
    out = np.zeros(len(q))
    for i, (u, v, l, slo, shi, tlo, thi) in enumerate(qc):
        if slo >= shi or tlo >= thi:
            continue
        f = ((u % cs) * cs + v % cs) * nl + l
        for zs in range(slo // t, (shi - 1) // t + 1):
            a0, a1 = max(slo, zs * t) - zs * t, min(shi, (zs + 1) * t) - zs * t
            for zt in range(tlo // t, (thi - 1) // t + 1):
                b0, b1 = max(tlo, zt * t) - zt * t, min(thi, (zt + 1) * t) - zt * t
                k = (u // cs, v // cs, zs, zt)
                out[i] += float(np.sum(np.abs(Z[k][f] * (CX[k][a1] - CX[k][a0]) * (CY[k][b1] - CY[k][b0]))))
    return out


@pytest.mark.parametrize("R", [4, 8, 16, 32])
def test_map_path_bf16_tables_match_oracle(R):
    """BF16 query tables of the compact layout (Sec. 4.4 storage; rank 4
    reads four ranks a lane from 8-byte loads, ranks 8 to 32 eight from
    16-byte loads, one to four lanes a query):
    the library's CX, CY and Z bit-equal to the oracle's rounding of its own
    summed-area tables of the fitted X, Y (FP64 sums, then FP32, then BF16)
    and of Z; the query on them against the oracle's block-split query on
    the same stored values within 1e-5 of the rank terms' magnitude; the
    query error against the FP32 tables within the BF16 storage bound;
    sampling refuses BF16 tables."""
    cfg, nxy, d = _c1()
    cs, t = 8, 16
    tab = G.cp_als_clustered_map(torch.from_numpy(nxy), d, t, cs, R, iters=2, seed=3)
    bt = G.clustered_bf16(tab)
    assert bt.dtype == "bf16" and bt.CX.dtype == torch.bfloat16 and bt.Z.shape == tab.Z.shape
    X, Y, Z, _ = _shaped(tab, cfg.nu, cfg.nv, cfg.nbins, t, cs)
    CXb = quant.bf16_round(cluster.block_cumulative(X)).astype(np.float64)
    CYb = quant.bf16_round(cluster.block_cumulative(Y)).astype(np.float64)
    Zb = quant.bf16_round(Z).astype(np.float64)
    assert np.array_equal(bt.CX.float().cpu().numpy().reshape(CXb.shape), CXb)
    assert np.array_equal(bt.CY.float().cpu().numpy().reshape(CYb.shape), CYb)
    assert np.array_equal(bt.Z.float().cpu().numpy(), quant.bf16_round(tab.Z.cpu().numpy()))
    rng = np.random.default_rng(9)
    q = _random_queries(rng, 4000, cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins)
    qd = torch.from_numpy(q.astype(np.int32))
    got = G.query_clustered(bt, qd).cpu().numpy().astype(np.float64)
    want = cluster.clustered_range_query_tables(CXb, CYb, Zb, q, cfg.nlevels, cs)
    mag = _table_magnitude(CXb, CYb, Zb, q, cfg.nlevels, cs)
    assert np.all(np.abs(got - want) <= 1e-5 * mag + 1e-30)
    # BF16 storage against the FP32 tables: three rounded factors of a term
    f32 = G.query_clustered(tab, qd).cpu().numpy().astype(np.float64)
    m32 = _magnitude(X, Y, Z, q, cfg.nlevels, cs)
    assert np.all(np.abs(got - f32) <= 4 * 2.0 ** -8 * m32 + 1e-30)
    uvl = torch.zeros((4, 3), dtype=torch.int32)
    rnd = torch.zeros((4, 7), dtype=torch.float32)
    with pytest.raises(G.GlintError):
        G.sample_clustered(bt, uvl, rnd)


def test_map_index_many_tensors_and_scan_chunks():
    """256 x 256 flake map, regions of 4 texels, N = 32 in blocks of 16:
    16,384 region tensors, so the row scan spans 16 chunks; the index against
    the dense-layout call's non-blank rows on the stored tensor, and one
    fitted sweep equal to it."""
    nxy = gen.flake_map(256, 256, 900, 0.2, 21)
    d = G.desc_of(256, 256, 3, 32, 0.01)
    T = G.build_tensor(nxy, d, torch.float32, direct_levels=1)
    dense = G.cp_als_clustered(T, d, 16, 4, 8, iters=1, seed=2)
    del T
    tab = G.cp_als_clustered_map(torch.from_numpy(nxy), d, 16, 4, 8, iters=1, seed=2)
    _check_index(tab, (dense.Z != 0).any(dim=-1).cpu().numpy())
    assert torch.equal(tab.dense_z(), dense.Z) and torch.equal(tab.X, dense.X)


def test_map_path_argument_errors():
    _, nxy, d = _c1()
    x = torch.from_numpy(nxy)
    with pytest.raises(G.GlintError):
        G.cp_als_clustered_map(x, d, 16, 5, 8, iters=1)        # region side must divide the map
    with pytest.raises(G.GlintError):
        G.cp_als_clustered_map(x, d, 16, 8, 12, iters=1)       # rank not supported
    with pytest.raises(G.GlintError):
        G.cp_als_clustered_map(x, d, 16, 8, 8, iters=1, dtype=torch.bfloat16)  # block tensors F32 or F64


def test_map_path_rank32_nine_levels_sampled_tensors():
    """At the paper's region size and rank on a map whose tensor is not
    formed: 256 x 256 flakes, N = 64 (16 angular blocks), 9 levels (footprints
    up to 256 texels: 576 footprints a region, so the Z factors live in the
    workspace), rank 32, FP64 block tensors, 3 sweeps.  Six region tensors
    (the three with the most non-blank image blocks, three others) against
    the oracle built from the map for that tensor alone: the non-blank
    footprints exactly, and the reconstruction within 1e-4 of the block's
    norm plus the FP32 storage bound (the rank-32 rule above)."""
    nu, nl, N, t, cs, R, seed = 256, 9, 64, 16, 8, 32, 17
    nxy = gen.flake_map(nu, nu, 1500, 0.2, 33)
    d = G.desc_of(nu, nu, nl, N, 0.005)
    print("cluster map 256^2 rank 32", flush=True)
    tab = G.cp_als_clustered_map(torch.from_numpy(nxy), d, t, cs, R, iters=3, seed=seed, dtype=torch.float64)
    ncu, ncv, nb, Lr, t = cluster.layout(nu, nu, nl, N, t, cs)
    zidx = tab.zidx.cpu().numpy()
    counts = (zidx >= 0).sum(axis=1)
    order = np.argsort(-counts, kind="stable")
    rng = np.random.default_rng(3)
    nonblank = np.flatnonzero(counts > 0)
    picks = list(order[:3]) + list(rng.choice(nonblank, 3, replace=False))
    X = tab.X.cpu().numpy().astype(np.float64)
    Y = tab.Y.cpu().numpy().astype(np.float64)
    Zc = tab.Z.cpu().numpy().astype(np.float64)
    for tensor in picks:
        tensor = int(tensor)
        zt, zs = tensor % nb, (tensor // nb) % nb
        cv, cu = (tensor // (nb * nb)) % ncv, tensor // (nb * nb * ncv)
        D = cluster.region_block_tensor(nxy, N, 0.005, nl, t, cs, cu, cv, zs, zt)
        keep = cluster.nonblank_footprints(D)
        assert np.array_equal(np.flatnonzero(zidx[tensor] >= 0), keep), tensor
        xo, yo, zo, _ = cluster.als3(D[:, :, keep], cluster.init_factors(seed, tensor, t, Lr, R, keep), 3)
        z = Zc[zidx[tensor][keep]]
        rec = np.einsum("ar,br,fr->abf", X[tensor], Y[tensor], z)
        reco = np.einsum("ar,br,fr->abf", xo, yo, zo)
        bound = _fp32_output_bound(xo[None], yo[None], zo[None])[0] + 1e-4 * np.linalg.norm(D)
        assert np.linalg.norm(rec - reco) <= bound, (tensor, float(np.linalg.norm(rec - reco) / bound))
