"""GPU parity: query backward, the summed-area-table chain rule, the autograd
Function, the MSE gradient and Adam against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import adam, query, quant

pytestmark = pytest.mark.gpu

import paper_2109_14807_amd as G  # noqa: E402


def _rand(rng, nu, nv, nl, N, R):
    return [rng.standard_normal((d, R)) * 0.5 for d in (nu, nv, nl, N, N)]


def _queries(rng, n, nu, nv, nl, N):
    q = np.empty((n, 7), dtype=np.int64)
    q[:, 0] = rng.integers(-nu, 2 * nu, n)
    q[:, 1] = rng.integers(0, nv, n)
    q[:, 2] = rng.integers(0, nl + 2, n)
    a = rng.integers(0, N + 1, (n, 2))
    b = rng.integers(0, N + 1, (n, 2))
    q[:, 3], q[:, 4] = a.min(1), a.max(1)
    q[:, 5], q[:, 6] = b.min(1), b.max(1)
    return q.astype(np.int32)


def _close(got, want, what):
    scale = max(float(np.max(np.abs(want))), 1e-30)
    err = float(np.max(np.abs(got.astype(np.float64) - want)))
    assert err <= 1e-5 * scale, (what, err / scale)


@pytest.mark.parametrize("R,dtype", [(16, "f32"), (64, "f32"), (128, "f32"), (64, "bf16")])
def test_backward_matches_oracle_gradient(R, dtype):
    rng = np.random.default_rng(R)
    nu, nv, nl, N = 40, 24, 6, 32
    F = _rand(rng, nu, nv, nl, N, R)
    q = _queries(rng, 30001, nu, nv, nl, N)
    g = rng.standard_normal(q.shape[0]).astype(np.float32)
    Ft = [torch.tensor(x, dtype=torch.float32, device="cuda") for x in F]
    tabs = G.make_tables(*Ft, dtype=dtype, cum_dtype=dtype)
    dU, dV, dL, dCS, dCT = G.query_backward(tabs, q, torch.tensor(g, device="cuda"))
    # oracle on the stored values
    rnd = (lambda x: quant.bf16_round(np.float32(x)).astype(np.float64)) if dtype == "bf16" else \
          (lambda x: np.asarray(x, dtype=np.float32).astype(np.float64))
    F32 = [np.asarray(x, dtype=np.float32).astype(np.float64) for x in F]
    U, V, L = (rnd(x) for x in F32[:3])
    CS, CT = (rnd(query.cumulative(x)) for x in F32[3:])
    want = query.range_query_grad(U, V, L, CS, CT, q, g.astype(np.float64))
    for got, w, name in zip((dU, dV, dL, dCS, dCT), want, ("dU", "dV", "dL", "dCS", "dCT")):
        _close(got.cpu().numpy(), w, name)
    dS = G.cumulative_backward(dCS).cpu().numpy()
    _close(dS, query.cumulative_grad(want[3]), "dS")


def test_autograd_function_end_to_end():
    rng = np.random.default_rng(5)
    nu, nv, nl, N, R = 32, 32, 5, 32, 16
    F = _rand(rng, nu, nv, nl, N, R)
    q = _queries(rng, 5000, nu, nv, nl, N)
    w = rng.standard_normal(q.shape[0])
    Ft = [torch.tensor(x, dtype=torch.float32, device="cuda", requires_grad=True) for x in F]
    out = G.GlintQuery.apply(*Ft, torch.tensor(q, device="cuda"), "f32")
    (out.double() * torch.tensor(w, device="cuda")).sum().backward()
    F32 = [np.asarray(x, dtype=np.float32).astype(np.float64) for x in F]
    CS, CT = query.cumulative(F32[3]), query.cumulative(F32[4])
    dU, dV, dL, dCS, dCT = query.range_query_grad(F32[0], F32[1], F32[2], CS, CT, q, w)
    want = (dU, dV, dL, query.cumulative_grad(dCS), query.cumulative_grad(dCT))
    for t, wnt, name in zip(Ft, want, "UVLST"):
        _close(t.grad.cpu().numpy(), wnt, name)


def test_mse_gradient_and_loss():
    rng = np.random.default_rng(6)
    qv = rng.standard_normal(100003).astype(np.float32)
    tgt = rng.standard_normal(100003)
    gout = torch.empty(qv.shape[0], device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    G._lib.glint_mse_grad(torch.tensor(qv, device="cuda"), torch.tensor(tgt, device="cuda"), gout, loss)
    lw, gw = query.mse_loss(qv.astype(np.float64), tgt)
    assert abs(loss.item() - lw) <= 1e-12 * lw
    assert np.allclose(gout.cpu().numpy(), gw, rtol=1e-6, atol=0)


def test_adam_steps_match_oracle():
    rng = np.random.default_rng(7)
    p0 = rng.standard_normal(4099).astype(np.float32)
    p = torch.tensor(p0, device="cuda")
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    pw, mw, vw = p0.astype(np.float64), np.zeros(4099), np.zeros(4099)
    for k in range(1, 4):
        g = rng.standard_normal(4099).astype(np.float32)
        G._lib.glint_adam_step(p, torch.tensor(g, device="cuda"), m, v, 1e-2, 0.9, 0.999, 1e-8, k)
        pw, mw, vw = adam.adam_step(pw, g.astype(np.float64), mw, vw, k, 1e-2)
    assert np.max(np.abs(p.cpu().numpy() - pw)) < 1e-6


def test_refinement_lowers_the_loss():
    rng = np.random.default_rng(8)
    nu, nv, nl, N, R = 16, 16, 3, 16, 16
    F = _rand(rng, nu, nv, nl, N, R)
    q = _queries(rng, 4000, nu, nv, nl, N)
    target = query.range_query(*[np.float32(x).astype(np.float64) for x in F[:3]],
                               query.cumulative(np.float32(F[3]).astype(np.float64)),
                               query.cumulative(np.float32(F[4]).astype(np.float64)), q)
    noisy = [x + 0.05 * rng.standard_normal(x.shape) for x in F]
    _, losses = G.refine(*noisy, q, target, steps=60, lr=3e-3)
    losses = losses.cpu().numpy()
    assert losses[-1] < 0.5 * losses[0]


def test_backward_c4_full_batch_sparse_gout():
    """The 2048x2048, N = 64, 10-level, rank-128 FP32 shape with the whole
    2^24-record batch in one backward launch; gout is zero except on 10^4
    sampled records, so by linearity the gradients equal the oracle gradient
    of those records alone."""
    import gen
    cfg = gen.config("c4")
    nxy = gen.normal_map(cfg)
    q = gen.make_queries(cfg, nxy)
    rng = np.random.default_rng(44)
    F = _rand(rng, cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.rank)
    idx = np.sort(rng.choice(q.shape[0], 10_000, replace=False))
    g = np.zeros(q.shape[0], dtype=np.float32)
    g[idx] = rng.standard_normal(idx.size).astype(np.float32)
    Ft = [torch.tensor(x, dtype=torch.float32, device="cuda") for x in F]
    tabs = G.make_tables(*Ft)
    got = G.query_backward(tabs, torch.tensor(q, device="cuda"), torch.tensor(g, device="cuda"))
    F32 = [np.asarray(x, dtype=np.float32).astype(np.float64) for x in F]
    CS, CT = (np.float32(query.cumulative(x)).astype(np.float64) for x in F32[3:])
    want = query.range_query_grad(F32[0], F32[1], F32[2], CS, CT, q[idx], g[idx].astype(np.float64))
    for a, w, name in zip(got, want, ("dU", "dV", "dL", "dCS", "dCT")):
        _close(a.cpu().numpy(), w, name)


def test_backward_c4_finite_differences_fp64():
    """FD check on 64 random factor entries at the 2048x2048, N = 64, 10-level,
    rank-128 shape: the GPU gradient of sum_i g_i q_i (10^4 records with
    nonzero g inside the 2^24 batch) against FP64 central differences of the
    oracle query.  The query is linear in each single entry, so the difference
    quotient is exact up to rounding; S and T enter through their summed-area
    tables (chain rule by glint_cumulative_backward)."""
    import gen
    cfg = gen.config("c4")
    nxy = gen.normal_map(cfg)
    q = gen.make_queries(cfg, nxy)
    rng = np.random.default_rng(4004)
    F = [np.asarray(x, dtype=np.float32).astype(np.float64)
         for x in _rand(rng, cfg.nu, cfg.nv, cfg.nlevels, cfg.nbins, cfg.rank)]
    idx = np.sort(rng.choice(q.shape[0], 10_000, replace=False))
    g = np.zeros(q.shape[0], dtype=np.float32)
    g[idx] = rng.standard_normal(idx.size).astype(np.float32)
    tabs = G.make_tables(*[torch.tensor(x, dtype=torch.float32, device="cuda") for x in F])
    dU, dV, dL, dCS, dCT = G.query_backward(tabs, torch.tensor(q, device="cuda"), torch.tensor(g, device="cuda"))
    grads = [dU.cpu().numpy(), dV.cpu().numpy(), dL.cpu().numpy(),
             G.cumulative_backward(dCS).cpu().numpy(), G.cumulative_backward(dCT).cpu().numpy()]
    qs, gs = q[idx], g[idx].astype(np.float64)

    def loss(Fx):
        CS, CT = query.cumulative(Fx[3]), query.cumulative(Fx[4])
        return float(np.dot(gs, query.range_query(Fx[0], Fx[1], Fx[2], CS, CT, qs)))

    scale = max(float(np.max(np.abs(x))) for x in grads)
    worst = 0.0
    for _ in range(64):
        m = int(rng.integers(0, 5))
        i, r = int(rng.integers(0, F[m].shape[0])), int(rng.integers(0, F[m].shape[1]))
        h = 1e-3 * max(abs(F[m][i, r]), 1.0)
        Fp = [x.copy() for x in F]
        Fm = [x.copy() for x in F]
        Fp[m][i, r] += h
        Fm[m][i, r] -= h
        fd = (loss(Fp) - loss(Fm)) / (2 * h)
        worst = max(worst, abs(grads[m][i, r] - fd) / scale)
    assert worst <= 1e-5, worst
