"""Seeded random circuits with non-diagonal two-qubit gates.

The paper also runs random circuits (40 layers) and Shor's algorithm
(Sec. IV B) but defines neither; this is this project's recipe for the same
kind of workload, and, like the QAOA generator, it holds no arithmetic of the
contraction method: it only writes gate lists.

Recipe, with rng = numpy.random.default_rng(seed), qubits on a line:
  for each layer d = 0 .. depth-1:
    every qubit gets one of sqrt(X), sqrt(Y), sqrt(W) (W = (X + Y)/sqrt 2),
    drawn uniformly, never the one it had in the previous layer;
    then a two-qubit gate on the pairs (q, q+1) with q = d mod 2, 2 + d mod 2,
    ...: the fermionic simulation gate fSim(theta, phi) with theta, phi
    drawn from U[0, pi) per gate, or CZ when `cz` is set;
  bitstrings: n_bitstrings rows of Bernoulli(1/2) bits.
A gate is (qubits, matrix): matrix 2x2 or 4x4 complex, row = output index;
for two qubits the first listed qubit is the more significant index bit.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

Gate = Tuple[Tuple[int, ...], np.ndarray]


def _sqrt_x() -> np.ndarray:
    return 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128)


def _sqrt_y() -> np.ndarray:
    return 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]], dtype=np.complex128)


def _sqrt_w() -> np.ndarray:
    # sqrt(W) = exp(-i pi/4 W) up to a global phase, W = (X + Y) / sqrt(2)
    s = 1.0 / math.sqrt(2.0)
    W = np.array([[0, s - 1j * s], [s + 1j * s, 0]], dtype=np.complex128)
    c = math.cos(math.pi / 4)
    return c * np.eye(2, dtype=np.complex128) - 1j * math.sin(math.pi / 4) * W


def fsim(theta: float, phi: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[1, 0, 0, 0],
                     [0, c, -1j * s, 0],
                     [0, -1j * s, c, 0],
                     [0, 0, 0, complex(math.cos(phi), -math.sin(phi))]], dtype=np.complex128)


def cz() -> np.ndarray:
    return np.diag([1, 1, 1, -1]).astype(np.complex128)


@dataclass
class Circuit:
    n: int
    gates: List[Gate]
    bitstrings: np.ndarray  # uint8 [B, n]
    seed: int = 0

    @property
    def n_bitstrings(self) -> int:
        return int(self.bitstrings.shape[0])


def random_circuit(n: int, depth: int, n_bitstrings: int, seed: int, cz_gates: bool = False) -> Circuit:
    rng = np.random.default_rng(seed)
    singles = [_sqrt_x(), _sqrt_y(), _sqrt_w()]
    last = [-1] * n
    gates: List[Gate] = []
    for d in range(depth):
        for q in range(n):
            choices = [i for i in range(3) if i != last[q]]
            i = choices[int(rng.integers(len(choices)))]
            last[q] = i
            gates.append(((q,), singles[i]))
        for q in range(d % 2, n - 1, 2):
            if cz_gates:
                gates.append(((q, q + 1), cz()))
            else:
                theta, phi = rng.uniform(0.0, math.pi, size=2)
                gates.append(((q, q + 1), fsim(float(theta), float(phi))))
    bits = rng.integers(0, 2, size=(n_bitstrings, n), dtype=np.uint8)
    return Circuit(n=n, gates=gates, bitstrings=bits, seed=seed)
