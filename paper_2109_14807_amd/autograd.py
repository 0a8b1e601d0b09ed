"""torch.autograd.Function over the range query and its hand-written backward.

GlintQuery.apply(U, V, L, S, Tf, q, dtype="f32") takes FP32 master factors
[rows][R] on the GPU and int32 query records [nq][7].  The forward builds the
summed-area tables of S and Tf (FP64 accumulation) and runs the query kernel;
the backward runs the query-gradient kernel and the summed-area-table chain
rule.  With dtype="bf16" the tables are stored in BF16 for the forward and the
gradients with respect to the BF16 values are passed straight through to the
FP32 masters (straight-through quantisation-aware refinement).
"""
from __future__ import annotations

import torch

from . import api


class GlintQuery(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, V, Lf, S, Tf, q, dtype: str = "f32"):
        tables = api.make_tables(U, V, Lf, S, Tf, dtype=dtype, cum_dtype=dtype)
        out = api.query(tables, q)
        ctx.tables = tables
        ctx.save_for_backward(q)
        return out

    @staticmethod
    def backward(ctx, gout):
        (q,) = ctx.saved_tensors
        dU, dV, dL, dCS, dCT = api.query_backward(ctx.tables, q, gout.float())
        dS = api.cumulative_backward(dCS)
        dT = api.cumulative_backward(dCT)
        ctx.tables = None
        return dU, dV, dL, dS, dT, None, None


def glint_query_fn(U, V, Lf, S, Tf, q, dtype: str = "f32"):
    return GlintQuery.apply(U, V, Lf, S, Tf, q, dtype)
