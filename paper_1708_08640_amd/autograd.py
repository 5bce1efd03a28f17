"""torch.autograd.Function over the prediction map of a bound plan.

Forward returns the Tucker predictions x~ for every training tensor entry
(Eq 4) and u^(c).v for every entry of each coupled matrix; backward is the
library's adjoint kernel (s3_backward), so the factorisation can sit inside a
larger differentiable model.  The parameters passed in must be the tensors the
plan is bound to (``plan.U``, ``plan.G``, ``plan.V``).
"""
from __future__ import annotations

import torch


class SparseTuckerCMTF(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, *params):
        N, M = len(plan.U), len(plan.V)
        bound = plan.U + [plan.G] + plan.V
        if len(params) != N + 1 + M or any(p.data_ptr() != b.data_ptr() for p, b in zip(params, bound)):
            raise ValueError("parameters must be the plan's bound tensors (plan.U, plan.G, plan.V)")
        ctx.plan = plan
        xhat = plan.predict(plan.x_idx)
        yhat = [plan.predict_matrix(m, r, c) for m, (r, c, _) in enumerate(plan.y)]
        return (xhat, *yhat)

    @staticmethod
    def backward(ctx, gx, *gy):
        plan = ctx.plan
        dU, dG, dV = plan.backward(gx, list(gy))
        return (None, *dU, dG, *dV)


def predictions(plan):
    """(x~, [y^_m]) with autograd through the library's adjoint."""
    outs = SparseTuckerCMTF.apply(plan, *plan.U, plan.G, *plan.V)
    return outs[0], list(outs[1:])
