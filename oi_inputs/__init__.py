"""Seeded synthetic inputs shared by the oracle tests, the HIP parity tests and the bench.

This package only *generates* inputs (graphs in CSR form, per-edge activation
probabilities, seed sets).  It holds none of the estimator's arithmetic: no
Philox, no Stage-1 table, no sampling, no stopping rule.  Both the CPU oracle
(`oracle/`) and the HIP library (`paper_1704_04794_amd/`) consume what it
produces; neither imports the other.
"""
from .graphs import (  # noqa: F401
    Graph,
    er_graph,
    chung_lu_graph,
    tiny16_graph,
    fig1_graph,
    star_graph,
    path_graph,
    out_tree_graph,
    graph_from_edges,
    wc_probs,
    trivalency_probs,
    sigmoid_theta_probs,
    uniform_probs,
    constant_probs,
    seed_node_outdeg_ge1,
    outdeg_ge1_nodes,
    uniform_seed_set,
    top_outdeg_seed_set,
    batched_seed_sets,
)
from .configs import ACCURACY_GRAPHS, CONFIGS, accuracy_workload, make_config  # noqa: F401
