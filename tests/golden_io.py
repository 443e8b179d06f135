"""Loads the JSON fixtures under tests/golden (values printed in the paper)."""
import json
import os

import numpy as np

from synth import Graph

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def graph_of(spec, name=""):
    e = np.array(spec["edges_src_label_dst"], np.int32).reshape(-1, 3)
    return Graph(int(spec["num_nodes"]), np.array(spec["node_label"], np.int32),
                 np.ascontiguousarray(e[:, 0]), np.ascontiguousarray(e[:, 1]),
                 np.ascontiguousarray(e[:, 2]), name=name)
