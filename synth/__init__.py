"""Seeded synthetic inputs shared by the tests, the oracle runs and the bench.

Holds no step of the refinement method: only graph generators. Both the GPU
path and the oracle receive the same arrays from here.
"""
from .graphs import (Graph, uniform_graph, powerlaw_graph, batch_graphs, serving_stream,
                     worked_example, path_graph, cycle_graph, tree_graph, complete_graph,
                     random_small_graph, degree_graph, CONFIGS, make_config)

__all__ = ["Graph", "uniform_graph", "powerlaw_graph", "batch_graphs", "serving_stream",
           "worked_example", "path_graph", "cycle_graph", "tree_graph", "complete_graph",
           "random_small_graph", "degree_graph", "CONFIGS", "make_config"]
