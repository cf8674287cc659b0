"""Seeded synthetic graph generators shared by the tests, the bench and the oracle checks.

This module only produces inputs (edge lists and edge weights).  It holds none of the
arithmetic of the random-walk-centrality method, so both the CPU oracle and the HIP
path can be fed from it without sharing any of the method's code.
"""
from .graphs import (  # noqa: F401
    EdgeList,
    erdos_renyi_lcc,
    barabasi_albert,
    grid_with_deletions,
    rmat_lcc,
    uniform_weights,
    largest_component,
    complete_graph,
    star_graph,
    cycle_graph,
    path_graph,
    disjoint_union,
    batch_mix,
)
