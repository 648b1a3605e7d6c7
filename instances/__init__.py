"""Seeded synthetic QAOA instances (random 3-regular graphs, angles, bitstrings).

This module holds no arithmetic of the contraction method: it only draws the
inputs that both the GPU path and the CPU oracle consume.  The paper evaluates
on 3-regular graphs whose edges are placed at random, with disconnected draws
discarded (Sec. IV A); the angle and bitstring distributions below are this
project's recipe for the same kind of workload.
"""
from .generate import (Instance, random_regular_graph, make_instance,
                       WORKLOADS, workload_instance, search_params, to_json, from_json)

__all__ = ["Instance", "random_regular_graph", "make_instance", "WORKLOADS",
           "workload_instance", "search_params", "to_json", "from_json"]
