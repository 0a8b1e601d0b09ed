"""GPU parity: summed-area tables, storage conversions and the range query
against the FP64 oracle on the same stored values (through the C ABI)."""
import numpy as np
import pytest
import torch

import gen
from oracle import quant, query

pytestmark = pytest.mark.gpu

import paper_2109_14807_amd as G  # noqa: E402

# FP32 query vs the FP64 oracle CP query on the same stored values:
# |q_gpu - q_64| <= TOL * M_q, M_q = sum_r |c_r U V L dS dT| the sum of the rank
# terms' magnitudes (each difference of stored summed-area values is rounded
# relative to itself in FP32, so M_q is the scale of the arithmetic error).
TOL = 1e-5


def _rand_factors(rng, nu, nv, nl, N, R):
    U = rng.standard_normal((nu, R)) * 0.5
    V = rng.standard_normal((nv, R)) * 0.5
    L = rng.standard_normal((nl, R))
    S = np.abs(rng.standard_normal((N, R))) * 0.2 + 0.01 * rng.standard_normal((N, R))
    Tf = np.abs(rng.standard_normal((N, R))) * 0.2
    return U, V, L, S, Tf


def _rand_queries(rng, n, nu, nv, nl, N, wild=False):
    q = np.empty((n, 7), dtype=np.int64)
    q[:, 0] = rng.integers(0, nu, n)
    q[:, 1] = rng.integers(0, nv, n)
    q[:, 2] = rng.integers(0, nl, n)
    a = rng.integers(0, N + 1, (n, 2))
    b = rng.integers(0, N + 1, (n, 2))
    q[:, 3], q[:, 4] = a.min(1), a.max(1)
    q[:, 5], q[:, 6] = b.min(1), b.max(1)
    if wild:   # out-of-range records: wrapped, clamped, reversed
        m = n // 8
        q[:m, 0] += rng.integers(-3, 3, m) * nu
        q[m:2 * m, 1] -= 5 * nv
        q[2 * m:3 * m, 2] = rng.integers(-4, nl + 6, m)
        q[3 * m:4 * m, 3] = rng.integers(-9, 0, m)
        q[4 * m:5 * m, 6] = N + rng.integers(1, 50, m)
        q[5 * m:6 * m, 3], q[5 * m:6 * m, 4] = q[5 * m:6 * m, 4], q[5 * m:6 * m, 3]
    return q.astype(np.int32)


def _stored(x, dtype):
    """Oracle side: the value each storage type holds for FP64 input x
    (always reached through FP32), plus its per-column scale."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    if dtype == "f32":
        return x32.astype(np.float64), None
    if dtype == "bf16":
        return quant.bf16_round(x32).astype(np.float64), None
    codes, sc = quant.fp8_quantize(x32)
    return quant.fp8_decode(codes), sc


def _oracle(F, q, dtype, cum_dtype):
    U, V, L, S, Tf = F
    vals, scales = [], []
    for x in (U, V, L):
        v, s = _stored(x, dtype)
        vals.append(v); scales.append(s)
    for x in (S, Tf):
        v, s = _stored(query.cumulative(x), cum_dtype)
        vals.append(v); scales.append(s)
    scale = np.ones(U.shape[1])
    for s in scales:
        if s is not None:
            scale = scale * s.astype(np.float64)
    return (query.range_query(*vals, q, scale=scale),
            query.range_query_term_magnitude(*vals, q, scale=scale))


def _check(got, want, mag, tol=TOL):
    err = np.abs(got.astype(np.float64) - want)
    bad = err > tol * mag + 1e-30
    assert not bad.any(), (int(bad.sum()), float((err / np.maximum(mag, 1e-300)).max()))


def test_cumulative_tables_bit_exact():
    rng = np.random.default_rng(1)
    S = rng.standard_normal((64, 32)) * 0.3
    for dtype in ("f32", "bf16", "fp8"):
        C, sc = G.cumulative(torch.tensor(S, device="cuda"), dtype)
        want = query.cumulative(S).astype(np.float32)
        if dtype == "f32":
            assert np.array_equal(C.cpu().numpy().view(np.uint32), want.view(np.uint32))
        elif dtype == "bf16":
            assert np.array_equal(C.view(torch.int16).cpu().numpy().view(np.uint16),
                                  quant.bf16_bits(want))
        else:
            codes, scw = quant.fp8_quantize(want)
            assert np.array_equal(C.view(torch.uint8).cpu().numpy(), codes)
            assert np.array_equal(sc.cpu().numpy().view(np.uint32), scw.view(np.uint32))


def test_convert_bit_exact_including_edge_values():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((100, 16)) * np.logspace(-6, 3, 16)[None, :]
    X[0, :] = [0.0, -0.0, 448.0, -448.0, 1e-9, 2 ** -9, 3 * 2 ** -10, 1.0 + 2 ** -8,
               1.0 + 3 * 2 ** -8, 240.0, 232.0, 0.015625, 0.0146484375, -7.5, 1e5, -1e-30]
    X[:, 5] = 0.0                                   # all-zero column: scale 1
    for dtype in ("f32", "bf16", "fp8"):
        out, sc = G.convert(torch.tensor(X, device="cuda"), dtype)
        x32 = X.astype(np.float32)
        if dtype == "f32":
            assert np.array_equal(out.cpu().numpy().view(np.uint32), x32.view(np.uint32))
        elif dtype == "bf16":
            assert np.array_equal(out.view(torch.int16).cpu().numpy().view(np.uint16),
                                  quant.bf16_bits(x32))
        else:
            codes, scw = quant.fp8_quantize(x32)
            assert np.array_equal(out.view(torch.uint8).cpu().numpy(), codes)
            assert np.array_equal(sc.cpu().numpy(), scw)


def test_fp8_decode_matches_the_format_on_every_code():
    """Tables holding every FP8 code: with U = V = L = 1, CT = [0, 1, 1, ...]
    and CS[j+1] = code j, the query over s in [0, j+1), t in [0, 1) reads back
    R times the value of code j."""
    R, N = 16, 256
    ones = torch.full((1, R), 0x38, dtype=torch.uint8, device="cuda").view(torch.float8_e4m3fn)
    codes = np.arange(N).astype(np.uint8)
    codes[(codes == 0x7F) | (codes == 0xFF)] = 0                 # the two NaN codes
    cs = np.zeros((N + 1, R), dtype=np.uint8)
    cs[1:] = codes[:, None]
    ct = np.zeros((N + 1, R), dtype=np.uint8)
    ct[1:] = 0x38
    CS = torch.tensor(cs, device="cuda").view(torch.float8_e4m3fn)
    CT = torch.tensor(ct, device="cuda").view(torch.float8_e4m3fn)
    tabs = G.QueryTables(ones, ones, ones, CS, CT, (None,) * 5)
    q = np.array([[0, 0, 0, 0, j + 1, 0, 1] for j in range(N)], dtype=np.int32)
    got = G.query(tabs, q).cpu().numpy().astype(np.float64)
    want = quant.fp8_decode(codes) * R
    assert np.array_equal(got, want)


CASES = [("f32", "f32", 16), ("f32", "f32", 32), ("f32", "f32", 64), ("f32", "f32", 128),
         ("f32", "f32", 256), ("bf16", "bf16", 16), ("bf16", "bf16", 64), ("bf16", "bf16", 128), ("bf16", "f32", 64),
         ("fp8", "bf16", 256), ("fp8", "bf16", 32), ("fp8", "fp8", 64), ("f32", "bf16", 64)]


@pytest.mark.parametrize("dtype,cum_dtype,R", CASES)
def test_query_matches_oracle(dtype, cum_dtype, R):
    print(f"query parity dtype={dtype} cum={cum_dtype} R={R}", flush=True)
    rng = np.random.default_rng(R + len(dtype) * 7 + len(cum_dtype))
    nu, nv, nl, N = 37, 53, 5, 32
    F = _rand_factors(rng, nu, nv, nl, N, R)
    q = _rand_queries(rng, 20011, nu, nv, nl, N, wild=True)
    tabs = G.make_tables(*[torch.tensor(x, device="cuda") for x in F], dtype=dtype, cum_dtype=cum_dtype)
    got = G.query(tabs, q).cpu().numpy()
    want, mag = _oracle(F, q, dtype, cum_dtype)
    _check(got, want, mag)
    c = np.clip(q[:, 3:7], 0, N)
    empty = (c[:, 0] >= c[:, 1]) | (c[:, 2] >= c[:, 3])
    assert empty.any() and np.all(got[empty] == 0.0)


GLOBAL_CUM_CASES = [("f32", "f32", 256, 128), ("f32", "bf16", 256, 256), ("f32", "fp8", 128, 256),
                    ("fp8", "f32", 256, 128), ("bf16", "fp8", 128, 256)]


@pytest.mark.parametrize("dtype,cum_dtype,R,N", GLOBAL_CUM_CASES)
def test_query_tables_beyond_lds(dtype, cum_dtype, R, N):
    """Summed-area tables too large for LDS are read from global memory (8-,
    4- and 16-byte row slices among these cases): flat and grouped queries."""
    print(f"global-table query dtype={dtype} cum={cum_dtype} R={R} N={N}", flush=True)
    rng = np.random.default_rng(R + N)
    nu, nv, nl = 29, 41, 6
    F = _rand_factors(rng, nu, nv, nl, N, R)
    q = _rand_queries(rng, 8009, nu, nv, nl, N, wild=True)
    tabs = G.make_tables(*[torch.tensor(x, device="cuda") for x in F], dtype=dtype, cum_dtype=cum_dtype)
    got = G.query(tabs, q).cpu().numpy()
    want, mag = _oracle(F, q, dtype, cum_dtype)
    _check(got, want, mag)
    npts, K = 257, 8
    uvl = np.stack([rng.integers(0, nu, npts), rng.integers(0, nv, npts),
                    rng.integers(0, nl, npts)], axis=1).astype(np.int32)
    boxes = _rand_queries(rng, npts * K, nu, nv, nl, N)[:, 3:7].reshape(npts, K, 4)
    gotg = G.query_grouped(tabs, uvl, boxes).cpu().numpy().reshape(-1)
    flat = np.concatenate([np.repeat(uvl, K, axis=0), boxes.reshape(-1, 4)], axis=1).astype(np.int32)
    want, mag = _oracle(F, flat, dtype, cum_dtype)
    _check(gotg, want, mag)


@pytest.mark.parametrize("nq", [0, 1, 3, 63, 65, 1000003])
def test_query_sizes(nq):
    rng = np.random.default_rng(nq + 5)
    nu, nv, nl, N, R = 64, 64, 5, 32, 16
    F = _rand_factors(rng, nu, nv, nl, N, R)
    q = _rand_queries(rng, max(nq, 1), nu, nv, nl, N)[:nq]
    tabs = G.make_tables(*[torch.tensor(x, device="cuda") for x in F])
    out = torch.full((nq + 1,), 7.0, device="cuda")
    G._lib.glint_query(tabs.factors(), torch.tensor(q, device="cuda").reshape(nq, 7), out[:nq])
    got = out.cpu().numpy()
    assert got[nq] == 7.0          # nothing written past the end
    if nq:
        want, mag = _oracle(F, q, "f32", "f32")
        _check(got[:nq], want, mag)


@pytest.mark.parametrize("nu,nv,N", [(128, 128, 32), (129, 40, 32), (40, 129, 32), (64, 64, 256), (1, 1, 4)])
def test_rank16_replicated_lds_tables_and_fallback(nu, nv, N):
    """Rank 16 over FP32 tables keeps U and V (up to 128 rows) and the other
    tables in LDS, four copies a row; larger maps or tables take the general
    kernel.  Both sides of each limit against the oracle, wrapped and clamped
    records included."""
    print(f"rank-16 query nu={nu} nv={nv} N={N}", flush=True)
    rng = np.random.default_rng(nu * 1000 + nv + N)
    nl, R = 5, 16
    F = _rand_factors(rng, nu, nv, nl, N, R)
    q = _rand_queries(rng, 30011, nu, nv, nl, N, wild=True)
    tabs = G.make_tables(*[torch.tensor(x, device="cuda") for x in F])
    got = G.query(tabs, q).cpu().numpy()
    want, mag = _oracle(F, q, "f32", "f32")
    _check(got, want, mag)


def test_grouped_equals_flat():
    rng = np.random.default_rng(9)
    nu, nv, nl, N, R = 64, 64, 12, 128, 64
    F = _rand_factors(rng, nu, nv, nl, N, R)
    npts, K = 3001, 32
    uvl = np.stack([rng.integers(-10, 80, npts), rng.integers(0, nv, npts),
                    rng.integers(0, 14, npts)], axis=1).astype(np.int32)
    boxes = _rand_queries(rng, npts * K, nu, nv, nl, N)[:, 3:7].reshape(npts, K, 4)
    for dtype, cum in (("f32", "f32"), ("fp8", "bf16")):
        tabs = G.make_tables(*[torch.tensor(x, device="cuda") for x in F], dtype=dtype, cum_dtype=cum)
        got = G.query_grouped(tabs, uvl, boxes).cpu().numpy()
        flat = np.concatenate([np.repeat(uvl, K, axis=0), boxes.reshape(-1, 4)], axis=1).astype(np.int32)
        ref = G.query(tabs, flat).cpu().numpy().reshape(npts, K)
        assert np.allclose(got, ref, rtol=1e-6, atol=1e-30)
        want, mag = _oracle(F, flat, dtype, cum)
        _check(got.reshape(-1), want, mag)


def test_query_c2_full_batch_sampled():
    """The 512x512, N = 64, 8-level, rank-64 shape with the full 1920x1080x8
    frame batch in the launch the benchmark times; 10^5 outputs checked."""
    cfg = gen.config("c2")
    nxy = gen.normal_map(cfg)
    q = gen.make_queries(cfg, nxy)
    rng = np.random.default_rng(22)
    F = _rand_factors(rng, cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.rank)
    tabs = G.make_tables(*[torch.tensor(x, device="cuda") for x in F])
    got = G.query(tabs, torch.tensor(q, device="cuda")).cpu().numpy()
    idx = np.sort(rng.choice(q.shape[0], 100_000, replace=False))
    idx[-1] = q.shape[0] - 1
    want, mag = _oracle(F, q[idx], "f32", "f32")
    _check(got[idx], want, mag)


def test_query_c3_bf16_full_batch_sampled():
    """The 2048x2048, N = 64, 10-level, rank-128 shape with BF16 factors and
    BF16 summed-area tables, the whole 6.4e7-record footprint batch in one
    launch; 10^5 outputs (and the last) against the oracle on the stored values."""
    cfg = gen.config("c3")
    nxy = gen.normal_map(cfg)
    print(f"c3: generating {cfg.nqueries} records", flush=True)
    q = gen.make_queries(cfg, nxy)
    rng = np.random.default_rng(33)
    F = _rand_factors(rng, cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.rank)
    tabs = G.make_tables(*[torch.tensor(x, device="cuda") for x in F], dtype="bf16", cum_dtype="bf16")
    got = G.query(tabs, torch.tensor(q, device="cuda")).cpu().numpy()
    idx = np.sort(rng.choice(q.shape[0], 100_000, replace=False))
    idx[-1] = q.shape[0] - 1
    want, mag = _oracle(F, q[idx], "bf16", "bf16")
    _check(got[idx], want, mag)
    print(f"c3 bf16: max |err| / M_q = {np.max(np.abs(got[idx] - want) / np.maximum(mag, 1e-300)):.2e}")


def test_grouped_c5_fp8_full_batch_sampled():
    """The 4096x4096 scratch shape, N = 128, 12 levels, rank 256, FP8 factors with
    per-column scales and BF16 tables: 2^20 shading points x 32 boxes in one
    grouped launch; 10^5 outputs against the oracle on the stored values."""
    cfg = gen.config("c5")
    nxy = gen.normal_map(cfg)
    print("c5: generating 2^20 x 32 boxes", flush=True)
    uvl, boxes = gen.make_grouped_queries(cfg, nxy)
    rng = np.random.default_rng(55)
    F = _rand_factors(rng, cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.rank)
    tabs = G.make_tables(*[torch.tensor(x, device="cuda") for x in F], dtype="fp8", cum_dtype="bf16")
    got = G.query_grouped(tabs, torch.tensor(uvl, device="cuda"), torch.tensor(boxes, device="cuda"))
    got = got.cpu().numpy().reshape(-1)
    npts, K = boxes.shape[:2]
    idx = np.sort(rng.choice(npts * K, 100_000, replace=False))
    idx[-1] = npts * K - 1
    p, k = idx // K, idx % K
    flat = np.concatenate([uvl[p], boxes[p, k]], axis=1).astype(np.int32)
    want, mag = _oracle(F, flat, "fp8", "bf16")
    _check(got[idx], want, mag)
    print(f"c5 fp8/bf16: max |err| / M_q = {np.max(np.abs(got[idx] - want) / np.maximum(mag, 1e-300)):.2e}")


def _oracle_trilinear(F, xyl, boxes, dtype, cum_dtype):
    U, V, L, S, Tf = F
    vals, scales = [], []
    for x in (U, V, L):
        v, s = _stored(x, dtype)
        vals.append(v); scales.append(s)
    for x in (S, Tf):
        v, s = _stored(query.cumulative(x), cum_dtype)
        vals.append(v); scales.append(s)
    scale = np.ones(U.shape[1])
    for s in scales:
        if s is not None:
            scale = scale * s.astype(np.float64)
    return (query.range_query_trilinear(*vals, xyl, boxes, scale=scale),
            query.range_query_trilinear(*vals, xyl, boxes, scale=scale, magnitude=True))


@pytest.mark.parametrize("dtype,cum_dtype,R,N", [("f32", "f32", 16, 32), ("f32", "f32", 64, 64),
                                                 ("bf16", "bf16", 128, 64), ("fp8", "bf16", 256, 128),
                                                 ("f32", "f32", 256, 128)])
def test_trilinear_query_matches_oracle(dtype, cum_dtype, R, N):
    """Off-grid footprints: continuous centres and levels (including negative,
    wrapped, non-finite and out-of-range coordinates, and empty boxes) against
    the oracle's blend of the eight corner queries."""
    print(f"trilinear dtype={dtype} cum={cum_dtype} R={R} N={N}", flush=True)
    rng = np.random.default_rng(R * 3 + N)
    nu, nv, nl = 37, 29, 7
    F = _rand_factors(rng, nu, nv, nl, N, R)
    n = 20011
    xyl = np.stack([rng.uniform(-2 * nu, 3 * nu, n), rng.uniform(-nv, 2 * nv, n),
                    rng.uniform(-1.0, nl + 1.0, n)], axis=1).astype(np.float32)
    xyl[:50, 0] = np.nan
    xyl[50:100, 1] = np.inf
    xyl[100:150, 2] = -np.inf
    xyl[150:200, 0] = 3e9
    xyl[200:250] = np.round(xyl[200:250])          # grid points
    xyl[8000:16000] = np.repeat(xyl[8000:9000], 8, axis=0)   # 8 boxes per shading point
    boxes = _rand_queries(rng, n, nu, nv, nl, N, wild=True)[:, 3:7].copy()
    tabs = G.make_tables(*[torch.tensor(x, device="cuda") for x in F], dtype=dtype, cum_dtype=cum_dtype)
    got = G.query_trilinear(tabs, xyl, boxes).cpu().numpy()
    want, mag = _oracle_trilinear(F, xyl, boxes, dtype, cum_dtype)
    _check(got, want, mag)
    c = np.clip(boxes, 0, N)
    empty = (c[:, 0] >= c[:, 1]) | (c[:, 2] >= c[:, 3])
    assert empty.any() and np.all(got[empty] == 0.0)


@pytest.mark.parametrize("nq", [0, 1, 65, 200_003, 4_000_037])
def test_validate_queries_counts_exactly(nq):
    """The record check against the oracle's count (bit-exact): wild records
    (wrapped, clamped, reversed) mixed with valid ones, sizes past the grid
    stride of the launch, and a count buffer holding garbage beforehand."""
    rng = np.random.default_rng(nq + 77)
    nu, nv, nl, N = 37, 20, 6, 32
    q = _rand_queries(rng, max(nq, 8), nu, nv, nl, N, wild=True)[:nq]
    if nq > 8:
        q[-5:] = [[0, 0, 0, N, N, 0, 0], [nu - 1, nv - 1, nl - 1, 0, N, 0, N], [nu, 0, 0, 0, 1, 0, 1],
                  [0, 0, 0, 0, N + 1, 0, 1], [0, 0, 0, 3, 2, 0, 1]]
    F = [np.ones((nu, 1)), np.ones((nv, 1)), np.ones((nl, 1)), np.ones((N, 1)), np.ones((N, 1))]
    tabs = G.make_tables(*[torch.tensor(x, device="cuda") for x in F])
    nbad = torch.full((2,), -12345, dtype=torch.int64, device="cuda")
    G._lib.glint_validate_queries(tabs.factors(), torch.tensor(q, device="cuda").reshape(nq, 7), nbad[:1])
    got = nbad.cpu().numpy()
    assert got[0] == query.count_invalid(q, nu, nv, nl, N)
    assert got[1] == -12345
    assert G.validate_queries(tabs, q) == got[0]
    if nq > 8:
        assert got[0] > 0 and query.count_invalid(q[-5:-3], nu, nv, nl, N) == 0


def test_query_rejects_sizes_beyond_packed_records():
    """Maps wider than 2^26 texels or more than 64 levels are refused on the
    host before any launch (the output is left as it was)."""
    rng = np.random.default_rng(3)
    F = _rand_factors(rng, 8, 8, 3, 16, 16)
    tabs = G.make_tables(*[torch.tensor(x, device="cuda") for x in F])
    q = torch.tensor(_rand_queries(rng, 100, 8, 8, 3, 16), device="cuda")
    out = torch.full((100,), 7.0, device="cuda")
    for field, value in (("nu", (1 << 26) + 1), ("nl", 65)):
        f = tabs.factors()
        setattr(f, field, value)
        with pytest.raises(G.GlintError):
            G._lib.glint_query(f, q, out)
    assert torch.all(out == 7.0)
    f = tabs.factors()
    G._lib.glint_query(f, q, out)
    assert not torch.all(out == 7.0)
