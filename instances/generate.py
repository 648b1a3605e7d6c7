"""Seeded instance generator.

Recipe (stated once, used by tests, bench and the oracle's callers):
  rng = numpy.random.default_rng(seed)
  1. graph: configuration-model pairing of 3 stubs per vertex; a draw with a
     self-loop, a repeated edge or more than one connected component is
     rejected and redrawn (the paper discards disconnected graphs, Sec. IV A).
  2. gamma[0..p-1] ~ U[0, pi), then beta[0..p-1] ~ U[0, pi).
  3. n_bitstrings rows of n bits, each bit Bernoulli(1/2).
Bit i of a bitstring is the measured value of qubit i = graph vertex i.
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np


@dataclass
class Instance:
    n: int
    p: int
    edges: List[Tuple[int, int]]
    gamma: List[float]
    beta: List[float]
    bitstrings: np.ndarray  # uint8 [B, n], 0/1
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_bitstrings(self) -> int:
        return int(self.bitstrings.shape[0])

    def edge_array(self) -> np.ndarray:
        return np.asarray(self.edges, dtype=np.uint32).reshape(-1, 2)


def random_regular_graph(n: int, rng: np.random.Generator, degree: int = 3,
                         max_tries: int = 100000) -> List[Tuple[int, int]]:
    """Uniform configuration-model draw of a simple connected degree-regular graph."""
    if (n * degree) % 2:
        raise ValueError("n*degree must be even")
    for _ in range(max_tries):
        stubs = np.repeat(np.arange(n), degree)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        seen = set()
        ok = True
        for a, b in pairs:
            a, b = int(a), int(b)
            if a == b:
                ok = False
                break
            key = (a, b) if a < b else (b, a)
            if key in seen:
                ok = False
                break
            seen.add(key)
        if not ok:
            continue
        adj = [[] for _ in range(n)]
        for a, b in seen:
            adj[a].append(b)
            adj[b].append(a)
        mark = [False] * n
        mark[0] = True
        stack = [0]
        while stack:
            u = stack.pop()
            for w in adj[u]:
                if not mark[w]:
                    mark[w] = True
                    stack.append(w)
        if all(mark):
            return sorted(seen)
    raise RuntimeError("no simple connected graph drawn")


def make_instance(n: int, p: int, n_bitstrings: int, seed: int) -> Instance:
    rng = np.random.default_rng(seed)
    edges = random_regular_graph(n, rng)
    gamma = [float(g) for g in rng.uniform(0.0, math.pi, size=p)]
    beta = [float(b) for b in rng.uniform(0.0, math.pi, size=p)]
    bits = rng.integers(0, 2, size=(n_bitstrings, n), dtype=np.uint8)
    return Instance(n=n, p=p, edges=edges, gamma=gamma, beta=beta,
                    bitstrings=bits, seed=seed)


# Workloads used by tests and the benchmark.  "k" is the number of cut
# variables; None means "smallest k whose searched cut set meets max_rank".
WORKLOADS = {
    "qaoa_n16_p1_k2": dict(n=16, p=1, n_bitstrings=1, k=2, max_rank=None,
                           precision="fp64"),
    "qaoa_n40_p2_b32_k8": dict(n=40, p=2, n_bitstrings=32, k=8, max_rank=18,
                               precision="fp32"),
    "qaoa_n80_p2_k16": dict(n=80, p=2, n_bitstrings=1, k=16, max_rank=24,
                            precision="fp32", ga_pop=32, ga_iters=20),
    "qaoa_n120_p1_b8": dict(n=120, p=1, n_bitstrings=8, k=None, max_rank=26,
                            precision="fp32"),
    # the same 120-qubit instance with 16 cut variables: 65,536 slices per
    # amplitude, the binary count of the paper's 4^8 subgraphs (Sec. IV A)
    "qaoa_n120_p1_b8_k16": dict(n=120, p=1, n_bitstrings=8, k=16, max_rank=26,
                                precision="fp32"),
}


def search_params(name: str) -> dict:
    """Cut-search parameters of a workload (Algorithm 1's N and T)."""
    w = WORKLOADS[name]
    return {"ga_pop": w.get("ga_pop", 11), "ga_iters": w.get("ga_iters", 4)}


def workload_instance(name: str, seed: int = 0) -> Instance:
    w = WORKLOADS[name]
    inst = make_instance(w["n"], w["p"], w["n_bitstrings"], seed)
    inst.meta = dict(w, workload=name)
    return inst


def to_json(inst: Instance) -> str:
    return json.dumps({
        "n": inst.n, "p": inst.p, "seed": inst.seed,
        "edges": [list(e) for e in inst.edges],
        "gamma": [float(g).hex() for g in inst.gamma],
        "beta": [float(b).hex() for b in inst.beta],
        "bitstrings": ["".join(str(int(b)) for b in row) for row in inst.bitstrings],
        "meta": inst.meta,
    })


def from_json(text: str) -> Instance:
    d = json.loads(text)
    bits = np.array([[int(c) for c in s] for s in d["bitstrings"]], dtype=np.uint8)
    return Instance(n=d["n"], p=d["p"], edges=[tuple(e) for e in d["edges"]],
                    gamma=[float.fromhex(g) for g in d["gamma"]],
                    beta=[float.fromhex(b) for b in d["beta"]],
                    bitstrings=bits, seed=d.get("seed", 0), meta=d.get("meta", {}))
