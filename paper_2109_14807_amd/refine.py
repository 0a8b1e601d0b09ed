"""Gradient refinement of CP factors against brute-force range integrals.

Minimises (1/Q) sum_i (q_i - target_i)^2 over the five factor tables with Adam
(Kingma and Ba), every step on the GPU through the library: summed-area
tables, query, loss gradient, query backward, table chain rule and the Adam
update.  With dtype="bf16" the forward reads BF16 tables built from the FP32
masters each step and the gradients update the masters (straight-through).
Not part of the paper: it tunes the ALS fit for the query error directly.
"""
from __future__ import annotations

import torch

from . import _lib as L
from . import api


def refine(U, V, Lf, S, Tf, q, target, steps: int, lr: float, dtype: str = "f32",
           betas=(0.9, 0.999), eps: float = 1e-8):
    """Returns (params, losses): refined FP32 tables (U, V, L, S, T) and the
    per-step loss (FP64 device tensor, loss before each step's update)."""
    params = [api._dev(x, torch.float32).clone() for x in (U, V, Lf, S, Tf)]
    m = [torch.zeros_like(p) for p in params]
    v = [torch.zeros_like(p) for p in params]
    q = api._dev(q, torch.int32)
    target = api._dev(target, torch.float64)
    nq = q.shape[0]
    losses = torch.zeros(steps, dtype=torch.float64, device="cuda")
    gout = torch.empty(nq, dtype=torch.float32, device="cuda")
    out = torch.empty(nq, dtype=torch.float32, device="cuda")
    for k in range(1, steps + 1):
        tables = api.make_tables(*params, dtype=dtype, cum_dtype=dtype)
        api.query(tables, q, out=out)
        L.glint_mse_grad(out, target, gout, losses[k - 1:k])
        dU, dV, dL, dCS, dCT = api.query_backward(tables, q, gout)
        grads = (dU, dV, dL, api.cumulative_backward(dCS), api.cumulative_backward(dCT))
        for p, g, mm, vv in zip(params, grads, m, v):
            L.glint_adam_step(p, g, mm, vv, lr, betas[0], betas[1], eps, k)
    return tuple(params), losses
