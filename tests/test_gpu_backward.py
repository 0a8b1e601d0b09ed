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
