"""torch.autograd.Function around the library's fixed-count forward and its
score-function backward (dOI/dp or dOI/dtheta with p = sigmoid(theta)).

The forward sets the graph's probabilities from the parameter tensor, draws
`count` IICP samples of stream X and returns the library's fixed-count
estimate OI = beta_0 * mean(Y) (Lemma 2); the backward recomputes every
sample from its Philox key on the GPU.  All estimator arithmetic happens in
the library: this module only moves tensors and scalars.
"""
from __future__ import annotations

import torch

from . import OI_PARAM_P, OI_PARAM_THETA, RUN_SEED, oi_backward, oi_sample_fixed


def _apply_weights(graph, weights, param):
    if param == OI_PARAM_THETA:
        graph.set_theta(weights)
    elif param == OI_PARAM_P:
        graph.set_probs(weights)
    else:
        raise ValueError("param must be OI_PARAM_P or OI_PARAM_THETA")


class OutwardInfluence(torch.autograd.Function):
    @staticmethod
    def forward(ctx, weights, graph, seeds, count, param=OI_PARAM_THETA, query_id=0, run_seed=RUN_SEED):
        w = weights.detach()
        _apply_weights(graph, w, param)
        y = torch.empty(count, dtype=torch.int32, device=weights.device)
        r = oi_sample_fixed(graph.h, query_id, seeds, 0, 0, count, run_seed, y)
        ctx.graph, ctx.seeds, ctx.count = graph, seeds, count
        ctx.param, ctx.query_id, ctx.run_seed = param, query_id, run_seed
        ctx.beta0 = r["beta0"]
        # the probabilities this forward sampled with: the graph may be given
        # other weights (another forward on the same graph) before backward
        ctx.version = graph.version
        ctx.save_for_backward(y, w)
        return torch.tensor(r["oi"], dtype=torch.float64, device=weights.device)

    @staticmethod
    def backward(ctx, grad_out):
        y, w = ctx.saved_tensors
        graph = ctx.graph
        if graph.version != ctx.version:
            # restore the forward's probabilities: the backward recomputes the
            # forward's samples, which only the same p reproduces
            _apply_weights(graph, w, ctx.param)
            ctx.version = graph.version
        g = torch.empty(graph.m, dtype=torch.float32, device=y.device)
        # oi_backward takes its scale as a host double and, like every library
        # call, returns only after its GPU work is done, so reading the scalar
        # upstream gradient here adds no wait the call would not make anyway
        oi_backward(graph.h, ctx.query_id, ctx.seeds, 0, ctx.count, ctx.run_seed,
                    y if ctx.beta0 > 0 else None, ctx.param, float(grad_out.item()), g)
        return g, None, None, None, None, None, None


def outward_influence(weights, graph, seeds, count, param=OI_PARAM_THETA, query_id=0, run_seed=RUN_SEED):
    return OutwardInfluence.apply(weights, graph, seeds, count, param, query_id, run_seed)
