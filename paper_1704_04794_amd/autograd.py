"""torch.autograd.Function around the library's fixed-count forward and its
score-function backward (dOI/dp or dOI/dtheta with p = sigmoid(theta)).

The forward sets the graph's probabilities from the parameter tensor, draws
`count` IICP samples of stream X and returns OI = beta_0 * mean(Y) (Lemma 2);
the backward recomputes every sample from its Philox key on the GPU.
"""
from __future__ import annotations

import torch

from . import OI_PARAM_P, OI_PARAM_THETA, RUN_SEED, oi_backward, oi_sample_fixed


class OutwardInfluence(torch.autograd.Function):
    @staticmethod
    def forward(ctx, weights, graph, seeds, count, param=OI_PARAM_THETA, query_id=0, run_seed=RUN_SEED):
        if param == OI_PARAM_THETA:
            graph.set_theta(weights.detach())
        elif param == OI_PARAM_P:
            graph.set_probs(weights.detach())
        else:
            raise ValueError("param must be OI_PARAM_P or OI_PARAM_THETA")
        y = torch.empty(count, dtype=torch.int32, device=weights.device)
        r = oi_sample_fixed(graph.h, query_id, seeds, 0, 0, count, run_seed, y)
        ctx.graph, ctx.seeds, ctx.count = graph, seeds, count
        ctx.param, ctx.query_id, ctx.run_seed = param, query_id, run_seed
        ctx.beta0 = r["beta0"]
        ctx.save_for_backward(y)
        oi = r["beta0"] * r["sum_y"] / count if r["beta0"] > 0 else 0.0
        return torch.tensor(oi, dtype=torch.float64, device=weights.device)

    @staticmethod
    def backward(ctx, grad_out):
        (y,) = ctx.saved_tensors
        g = torch.empty(ctx.graph.m, dtype=torch.float32, device=y.device)
        oi_backward(ctx.graph.h, ctx.query_id, ctx.seeds, 0, ctx.count, ctx.run_seed,
                    y if ctx.beta0 > 0 else None, ctx.param, float(grad_out.item()), g)
        return g, None, None, None, None, None, None


def outward_influence(weights, graph, seeds, count, param=OI_PARAM_THETA, query_id=0, run_seed=RUN_SEED):
    return OutwardInfluence.apply(weights, graph, seeds, count, param, query_id, run_seed)
