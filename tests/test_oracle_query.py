"""Pins of the FP64 oracle's query, gradient, quantisation and Adam (CPU only)."""
import numpy as np
import pytest
import torch

import gen
from oracle import adam, cp_als, ndf, quant, query


def _rand_factors(rng, dims, R):
    return [rng.standard_normal((d, R)) for d in dims]


def _rand_queries(rng, n, nu, nv, nl, N):
    q = np.empty((n, 7), dtype=np.int64)
    q[:, 0] = rng.integers(0, nu, n)
    q[:, 1] = rng.integers(0, nv, n)
    q[:, 2] = rng.integers(0, nl, n)
    a = rng.integers(0, N + 1, (n, 2))
    b = rng.integers(0, N + 1, (n, 2))
    q[:, 3], q[:, 4] = a.min(1), a.max(1)
    q[:, 5], q[:, 6] = b.min(1), b.max(1)
    return q


def test_cumulative_table():
    S = np.array([[1.0, 2.0], [3.0, -1.0], [0.5, 0.25]])
    assert np.array_equal(query.cumulative(S), [[0, 0], [1, 2], [4, 1], [4.5, 1.25]])


def test_appendix_identity_range_equals_explicit_box_sum():
    """Appendix proposition: for a CP tensor the box total is the rank sum of
    products of per-axis segment totals."""
    rng = np.random.default_rng(7)
    dims = (5, 4, 3, 6, 6)
    U, V, L, S, Tf = _rand_factors(rng, dims, 4)
    That = cp_als.reconstruct(U, V, L, S, Tf)
    q = _rand_queries(rng, 300, 5, 4, 3, 6)
    got = query.range_query(U, V, L, query.cumulative(S), query.cumulative(Tf), q)
    want = ndf.box_sum(That, q)
    assert np.max(np.abs(got - want)) <= 1e-13 * max(1.0, np.abs(want).max())


def test_range_equals_sum_of_point_queries():
    rng = np.random.default_rng(8)
    dims = (4, 4, 2, 8, 8)
    U, V, L, S, Tf = _rand_factors(rng, dims, 3)
    q = np.array([[1, 2, 1, 2, 7, 0, 3], [3, 0, 0, 0, 8, 5, 6]])
    got = query.range_query(U, V, L, query.cumulative(S), query.cumulative(Tf), q)
    for i, (u, v, l, slo, shi, tlo, thi) in enumerate(q):
        pts = sum(query.point_query(U, V, L, S, Tf, u, v, l, s, t)
                  for s in range(slo, shi) for t in range(tlo, thi))
        assert abs(got[i] - pts) < 1e-12


def test_rank1_is_product_of_segment_sums():
    U = np.array([[2.0]]); V = np.array([[3.0]]); L = np.array([[0.5]])
    S = np.array([[1.0], [2.0], [4.0], [8.0]])
    Tf = np.array([[1.0], [10.0], [100.0], [1000.0]])
    q = np.array([[0, 0, 0, 1, 3, 0, 2]])
    got = query.range_query(U, V, L, query.cumulative(S), query.cumulative(Tf), q)
    assert got[0] == 2.0 * 3.0 * 0.5 * (2.0 + 4.0) * (1.0 + 10.0)


def test_empty_and_clamped_boxes():
    rng = np.random.default_rng(9)
    U, V, L, S, Tf = _rand_factors(rng, (4, 4, 3, 5, 5), 2)
    CS, CT = query.cumulative(S), query.cumulative(Tf)
    q = np.array([[0, 0, 0, 3, 3, 0, 5],      # empty s
                  [0, 0, 0, 4, 2, 0, 5],      # reversed s
                  [0, 0, 0, 0, 5, 2, 2],      # empty t
                  [-1, 9, 10, -4, 99, 0, 5],  # wrap, clamp level and bins
                  [3, 1, 2, 0, 5, 0, 5]])
    got = query.range_query(U, V, L, CS, CT, q)
    assert got[0] == 0.0 and got[1] == 0.0 and got[2] == 0.0
    assert got[3] == got[4]


def test_full_box_of_exact_factors_is_one():
    """Level-0 cells are rank one (one texel), so the CP of a single cell's
    masses is exact and its full box holds the texel's unit mass."""
    nxy = gen.flake_map(4, 4, 3, 0.3, 2)
    ms, mt = ndf.texel_masses(nxy, 8, 0.05)
    U = np.ones((1, 1)); V = np.ones((1, 1)); L = np.ones((1, 1))
    S = ms[2, 3][:, None]; Tf = mt[2, 3][:, None]
    q = np.array([[0, 0, 0, 0, 8, 0, 8]])
    got = query.range_query(U, V, L, query.cumulative(S), query.cumulative(Tf), q)
    assert abs(got[0] - 1.0) < 1e-15


@pytest.mark.slow
def test_full_rank_cp_query_matches_bruteforce_range_integral():
    nxy = gen.flake_map(4, 4, 6, 0.4, 11)
    sigma, N, nl = 0.3, 4, 2
    T = ndf.ndf_bruteforce(nxy, N, sigma, nl)
    res = cp_als.cp_als(T, gen.als_init((4, 4, nl, N), rank=128, seed=5), iters=500)
    U, V, L, S, Tf = res["factors"]
    rng = np.random.default_rng(10)
    q = _rand_queries(rng, 200, 4, 4, nl, N)
    got = query.range_query(U, V, L, query.cumulative(S), query.cumulative(Tf), q)
    want = ndf.range_bruteforce(nxy, N, sigma, nl, q)
    assert np.max(np.abs(got - want)) <= 1e-8
    full = np.array([[u, v, l, 0, N, 0, N] for u in range(4) for v in range(4) for l in range(nl)])
    assert np.max(np.abs(query.range_query(U, V, L, query.cumulative(S), query.cumulative(Tf), full) - 1)) < 1e-8


def test_gradient_against_finite_differences():
    rng = np.random.default_rng(11)
    dims = (5, 4, 3, 6, 6)
    F = _rand_factors(rng, dims, 3)
    q = _rand_queries(rng, 50, 5, 4, 3, 6)
    g = rng.standard_normal(50)

    def loss(F):
        U, V, L, S, Tf = F
        return float(g @ query.range_query(U, V, L, query.cumulative(S), query.cumulative(Tf), q))

    U, V, L, S, Tf = F
    dU, dV, dL, dCS, dCT = query.range_query_grad(U, V, L, query.cumulative(S), query.cumulative(Tf), q, g)
    grads = [dU, dV, dL, query.cumulative_grad(dCS), query.cumulative_grad(dCT)]
    for m in range(5):
        for _ in range(8):
            i = rng.integers(0, F[m].shape[0]); r = rng.integers(0, 3)
            h = 1e-6 * max(1.0, abs(F[m][i, r]))
            Fp = [f.copy() for f in F]; Fm = [f.copy() for f in F]
            Fp[m][i, r] += h; Fm[m][i, r] -= h
            fd = (loss(Fp) - loss(Fm)) / (2 * h)
            assert abs(fd - grads[m][i, r]) <= 1e-6 * max(1.0, abs(fd)), (m, i, r)


def test_magnitude_bounds_value():
    rng = np.random.default_rng(12)
    F = _rand_factors(rng, (5, 4, 3, 6, 6), 3)
    q = _rand_queries(rng, 100, 5, 4, 3, 6)
    U, V, L, S, Tf = F
    CS, CT = query.cumulative(S), query.cumulative(Tf)
    assert np.all(np.abs(query.range_query(U, V, L, CS, CT, q)) <=
                  query.range_query_magnitude(U, V, L, CS, CT, q) * (1 + 1e-14))


# ----------------------------------------------------------------------------
# quantisation: against the library conversions of the same formats
# ----------------------------------------------------------------------------

def test_bf16_matches_torch_round_to_nearest_even():
    rng = np.random.default_rng(13)
    x = np.concatenate([rng.standard_normal(100000).astype(np.float32) * 10.0,
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, -0.0,
                                  1e-40, 3.0e38], dtype=np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    got = quant.bf16_round(x)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_fp8_decode_table_matches_torch():
    codes = np.arange(256, dtype=np.uint8)
    want = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    got = quant.fp8_decode(codes)
    same = (got == want) | (np.isnan(got) & np.isnan(want))
    assert same.all()
    assert quant.fp8_decode(0x7E) == 448.0


def test_fp8_encode_matches_torch_inside_range():
    rng = np.random.default_rng(14)
    x = np.concatenate([rng.standard_normal(100000) * 50.0,
                        quant.fp8_decode(np.arange(127)) * 1.0,          # exact values
                        (quant.fp8_decode(np.arange(126)) + quant.fp8_decode(np.arange(1, 127))) / 2,  # ties
                        rng.random(1000) * 2 ** -9]).astype(np.float32)
    x = np.clip(x, -448.0, 448.0)
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(quant.fp8_encode(x), want)
    assert quant.fp8_encode(1e6) == 0x7E and quant.fp8_encode(-1e6) == 0xFE


def test_fp8_column_quantisation_roundtrip_error():
    rng = np.random.default_rng(15)
    X = rng.standard_normal((64, 8)).astype(np.float32)
    X[:, 3] = 0.0
    codes, sc = quant.fp8_quantize(X)
    assert sc[3] == 1.0
    Y = quant.fp8_dequantize(codes, sc)
    err = np.abs(Y - X) / np.max(np.abs(X), axis=0, keepdims=True).clip(1e-30)
    assert err.max() <= 2 ** -4 + 1e-12         # half an ulp at 3 mantissa bits


def test_adam_step_matches_torch():
    rng = np.random.default_rng(16)
    p0 = rng.standard_normal(20)
    grads = [rng.standard_normal(20) for _ in range(3)]
    tp = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2)
    p, m, v = p0, np.zeros(20), np.zeros(20)
    for k, g in enumerate(grads, start=1):
        opt.zero_grad(); tp.grad = torch.tensor(g); opt.step()
        p, m, v = adam.adam_step(p, g, m, v, k, 1e-2)
    assert np.allclose(p, tp.detach().numpy(), rtol=0, atol=1e-12)


def test_mse_gradient():
    qv = np.array([1.0, 2.0, 3.0]); t = np.array([0.5, 2.0, 5.0])
    loss, g = query.mse_loss(qv, t)
    assert loss == (0.25 + 0 + 4) / 3
    assert np.allclose(g, [1 / 3, 0, -4 / 3])


def _rand_coords(rng, n, nu, nv, nl):
    return np.stack([rng.uniform(-nu, 2 * nu, n), rng.uniform(-nv, 2 * nv, n),
                     rng.uniform(-0.5, nl - 0.5, n)], axis=1).astype(np.float32)


def test_trilinear_at_grid_points_is_the_plain_query():
    rng = np.random.default_rng(31)
    dims = (6, 5, 4, 8, 8)
    U, V, L, S, Tf = _rand_factors(rng, dims, 5)
    CS, CT = query.cumulative(S), query.cumulative(Tf)
    q = _rand_queries(rng, 200, 6, 5, 4, 8)
    xyl = q[:, :3].astype(np.float32)
    got = query.range_query_trilinear(U, V, L, CS, CT, xyl, q[:, 3:])
    assert np.array_equal(got, query.range_query(U, V, L, CS, CT, q))


def test_trilinear_equals_linear_interpolation_of_the_tensor():
    """Against scipy's order-1 interpolation of the reconstructed tensor over
    (u, v, l), with u, v extended periodically and l clamped, then box sums."""
    from scipy.ndimage import map_coordinates
    rng = np.random.default_rng(32)
    nu, nv, nl, N = 5, 4, 3, 6
    U, V, L, S, Tf = _rand_factors(rng, (nu, nv, nl, N, N), 3)
    T = cp_als.reconstruct(U, V, L, S, Tf)
    Tp = np.concatenate([T, T[:1]], axis=0)          # u = nu wraps to 0
    Tp = np.concatenate([Tp, Tp[:, :1]], axis=1)      # v = nv wraps to 0
    xyl = _rand_coords(rng, 60, nu, nv, nl)
    boxes = _rand_queries(rng, 60, nu, nv, nl, N)[:, 3:]
    got = query.range_query_trilinear(U, V, L, query.cumulative(S), query.cumulative(Tf), xyl, boxes)
    s_idx, t_idx = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    for i in range(xyl.shape[0]):
        x, y, lam = (float(c) for c in xyl[i])
        coords = np.stack([np.full((N, N), x % nu), np.full((N, N), y % nv),
                           np.full((N, N), min(max(lam, 0.0), nl - 1.0)), s_idx, t_idx])
        sl = map_coordinates(Tp, coords.reshape(5, -1), order=1, mode="nearest").reshape(N, N)
        slo, shi, tlo, thi = boxes[i]
        want = sl[slo:shi, tlo:thi].sum()
        assert abs(got[i] - want) <= 1e-11 * max(1.0, abs(want)), (i, got[i], want)


def test_trilinear_blend_equals_interpolated_factor_rows():
    """The CP reconstruction is multilinear, so the blend of the eight corner
    queries equals one query with linearly interpolated U, V and L rows (the
    form the GPU evaluates)."""
    rng = np.random.default_rng(33)
    nu, nv, nl, N, R = 7, 6, 5, 16, 8
    U, V, L, S, Tf = _rand_factors(rng, (nu, nv, nl, N, N), R)
    CS, CT = query.cumulative(S), query.cumulative(Tf)
    xyl = _rand_coords(rng, 500, nu, nv, nl)
    boxes = _rand_queries(rng, 500, nu, nv, nl, N)[:, 3:]
    got = query.range_query_trilinear(U, V, L, CS, CT, xyl, boxes)
    x, y = xyl[:, 0].astype(np.float64), xyl[:, 1].astype(np.float64)
    lam = np.clip(xyl[:, 2].astype(np.float64), 0, nl - 1)
    u0, v0, l0 = np.floor(x).astype(int), np.floor(y).astype(int), np.floor(lam).astype(int)
    fx, fy, fl = (x - u0)[:, None], (y - v0)[:, None], (lam - l0)[:, None]
    Ui = (1 - fx) * U[u0 % nu] + fx * U[(u0 + 1) % nu]
    Vi = (1 - fy) * V[v0 % nv] + fy * V[(v0 + 1) % nv]
    Li = (1 - fl) * L[l0] + fl * L[np.minimum(l0 + 1, nl - 1)]
    slo, shi, tlo, thi = boxes.T
    want = np.sum(Ui * Vi * Li * (CS[shi] - CS[slo]) * (CT[thi] - CT[tlo]), axis=1)
    want[(slo >= shi) | (tlo >= thi)] = 0.0
    assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.abs(want).max())


def test_trilinear_boundary_rules():
    rng = np.random.default_rng(34)
    nu, nv, nl, N = 4, 6, 3, 8
    U, V, L, S, Tf = _rand_factors(rng, (nu, nv, nl, N, N), 4)
    CS, CT = query.cumulative(S), query.cumulative(Tf)
    box = np.array([[1, 5, 2, 7]])
    f = lambda c: query.range_query_trilinear(U, V, L, CS, CT, np.array([c], dtype=np.float32), box)[0]
    assert f([1.25, 2.5, 0.75]) == pytest.approx(f([1.25 + 3 * nu, 2.5 - 2 * nv, 0.75]), rel=1e-12)
    assert f([1.0, 2.0, -3.0]) == f([1.0, 2.0, 0.0])
    assert f([1.0, 2.0, 9.0]) == f([1.0, 2.0, nl - 1.0])
    assert f([np.nan, 2.0, 1.0]) == f([0.0, 2.0, 1.0])
    assert f([1.0, np.inf, 1.0]) == f([1.0, 0.0, 1.0])
    # the level weight is linear between two levels
    a, b, m = f([1.0, 2.0, 1.0]), f([1.0, 2.0, 2.0]), f([1.0, 2.0, 1.25])
    assert m == pytest.approx(0.75 * a + 0.25 * b, rel=1e-12)


def test_count_invalid_records():
    nu, nv, nl, N = 8, 6, 3, 16
    good = [[0, 0, 0, 0, 16, 0, 16], [7, 5, 2, 3, 3, 4, 9], [1, 2, 1, 16, 16, 0, 0]]   # empty boxes are valid
    bad = [[8, 0, 0, 0, 1, 0, 1], [-1, 0, 0, 0, 1, 0, 1], [0, 6, 0, 0, 1, 0, 1], [0, 0, 3, 0, 1, 0, 1],
           [0, 0, -1, 0, 1, 0, 1], [0, 0, 0, -1, 1, 0, 1], [0, 0, 0, 0, 17, 0, 1], [0, 0, 0, 5, 4, 0, 1],
           [0, 0, 0, 0, 1, 9, 2], [9, 9, 9, 99, -9, 99, -9]]
    assert query.count_invalid(good, nu, nv, nl, N) == 0
    assert query.count_invalid(bad, nu, nv, nl, N) == len(bad)
    # a record the rules leave unchanged is exactly a valid one
    rng = np.random.default_rng(5)
    q = rng.integers(-3, 20, (2000, 7))
    canon = np.stack([np.mod(q[:, 0], nu), np.mod(q[:, 1], nv), np.clip(q[:, 2], 0, nl - 1)], 1)
    same = np.all(canon == q[:, :3], axis=1) & np.all((q[:, 3:] >= 0) & (q[:, 3:] <= N), axis=1) \
        & (q[:, 3] <= q[:, 4]) & (q[:, 5] <= q[:, 6])
    assert query.count_invalid(q, nu, nv, nl, N) == int((~same).sum())


def test_magnitudes_hand_computed():
    """Both magnitudes on a two-rank case worked by hand.

    U = [1, -2], V = [3, 1], L = [0.5, 2] (one row each), so U V L = [1.5, -4];
    S = [[1, -1], [2, 3]] gives CS = [[0, 0], [1, -1], [3, 2]];
    T = [[2, 1], [0, 3]] gives CT = [[0, 0], [2, 1], [2, 4]].
    Box s [1, 2), t [0, 2): dS = [2, 3], dT = [2, 4]; terms 6 and -48, so
    q = -42, M_q = 54, N_q = 1.5 (3 + 1)(2 + 0) + 4 (2 + 1)(4 + 0) = 60.
    Box s [0, 1), t [1, 2): dS = [1, -1], dT = [0, 3]; terms 0 and 12, so
    q = 12, M_q = 12, N_q = 1.5 (1 + 0)(2 + 2) + 4 (1 + 0)(4 + 1) = 26.
    The third record is the first one out of range (u, v wrap, l, s_hi and
    t_lo clamp); the fourth is empty.  With per-rank scales (2, 0.5) the
    first box's terms become 12 and -24."""
    U = np.array([[1.0, -2.0]])
    V = np.array([[3.0, 1.0]])
    L = np.array([[0.5, 2.0]])
    CS = query.cumulative(np.array([[1.0, -1.0], [2.0, 3.0]]))
    CT = query.cumulative(np.array([[2.0, 1.0], [0.0, 3.0]]))
    assert np.array_equal(CS, [[0, 0], [1, -1], [3, 2]])
    assert np.array_equal(CT, [[0, 0], [2, 1], [2, 4]])
    q = np.array([[0, 0, 0, 1, 2, 0, 2],
                  [0, 0, 0, 0, 1, 1, 2],
                  [5, -3, 7, 1, 9, -1, 2],
                  [0, 0, 0, 2, 2, 0, 2]])
    assert np.array_equal(query.range_query(U, V, L, CS, CT, q), [-42.0, 12.0, -42.0, 0.0])
    assert np.array_equal(query.range_query_term_magnitude(U, V, L, CS, CT, q), [54.0, 12.0, 54.0, 0.0])
    assert np.array_equal(query.range_query_magnitude(U, V, L, CS, CT, q), [60.0, 26.0, 60.0, 0.0])
    sc = np.array([2.0, 0.5])
    assert np.array_equal(query.range_query(U, V, L, CS, CT, q[:1], scale=sc), [-12.0])
    assert np.array_equal(query.range_query_term_magnitude(U, V, L, CS, CT, q[:1], scale=sc), [36.0])
    assert np.array_equal(query.range_query_magnitude(U, V, L, CS, CT, q[:1], scale=sc), [48.0])


def test_term_magnitude_between_value_and_condition_magnitude():
    """|q| <= M_q <= N_q on random signed factors (the triangle inequality twice)."""
    rng = np.random.default_rng(21)
    U, V, L, S, Tf = _rand_factors(rng, (5, 4, 3, 6, 6), 3)
    q = _rand_queries(rng, 200, 5, 4, 3, 6)
    CS, CT = query.cumulative(S), query.cumulative(Tf)
    val = np.abs(query.range_query(U, V, L, CS, CT, q))
    m = query.range_query_term_magnitude(U, V, L, CS, CT, q)
    n = query.range_query_magnitude(U, V, L, CS, CT, q)
    assert np.all(val <= m * (1 + 1e-14)) and np.all(m <= n * (1 + 1e-14))
    assert np.any(m < 0.5 * n)
