"""Amplitudes of general circuits (non-diagonal two-qubit gates), complex128.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Two independent
routes, written from the definitions:
  * statevector: |psi> = U_m ... U_1 |0^n>, amplitude <x|psi>; qubit q is bit
    q of the statevector index (little-endian, as for the QAOA oracle);
  * tensor network (Sec. II A, Fig. 1, Eq. (1)): every gate is a vertex whose
    tensor has one index per input wire and one per output wire, every wire
    segment is its own binary variable (nothing merged), inputs are |0> and
    measurements project on x; the rank-0 contraction by variable
    elimination is the amplitude.  Slicing fixes wire variables (Sec. III A).
A gate is (qubits, matrix) with matrix[out, in]; for two qubits the first
listed qubit is the more significant bit of both indices.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Sequence, Tuple

import numpy as np


def statevector(n: int, gates) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    idx = np.arange(1 << n)
    for qs, U in gates:
        U = np.asarray(U, dtype=np.complex128)
        if len(qs) == 1:
            q = qs[0]
            b = (idx >> q) & 1
            partner = idx ^ (1 << q)
            new = U[b, b] * psi + U[b, 1 - b] * psi[partner]
        else:
            q1, q2 = qs
            b1 = (idx >> q1) & 1
            b2 = (idx >> q2) & 1
            row = 2 * b1 + b2
            new = np.zeros_like(psi)
            for col in range(4):
                c1, c2 = col >> 1, col & 1
                src = (idx & ~((1 << q1) | (1 << q2))) | (c1 << q1) | (c2 << q2)
                new += U[row, col] * psi[src]
        psi = new
    return psi


def amplitude_statevector(n: int, gates, x) -> complex:
    psi = statevector(n, gates)
    return complex(psi[sum(int(v) << i for i, v in enumerate(x))])


Factor = Tuple[Tuple[int, ...], np.ndarray]


def network(n: int, gates, x) -> Tuple[List[Factor], List[List[int]]]:
    """Factors over binary wire variables; also, per qubit, the variables of
    its successive wire segments (first: the input segment)."""
    factors: List[Factor] = []
    segs: List[List[int]] = [[q] for q in range(n)]
    nxt = n
    for q in range(n):
        factors.append(((q,), np.array([1.0, 0.0], dtype=np.complex128)))   # |0>
    for qs, U in gates:
        U = np.asarray(U, dtype=np.complex128)
        ins = [segs[q][-1] for q in qs]
        outs = list(range(nxt, nxt + len(qs)))
        nxt += len(qs)
        for q, o in zip(qs, outs):
            segs[q].append(o)
        k = len(qs)
        T = U.reshape((2,) * (2 * k))          # [out..., in...]
        factors.append((tuple(outs + ins), T))
    for q in range(n):
        factors.append(((segs[q][-1],), np.array([1.0 if int(x[q]) == b else 0.0 for b in (0, 1)],
                                                 dtype=np.complex128)))
    return factors, segs


def _eliminate(factors: List[Factor]) -> complex:
    letters = "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ"
    adj: Dict[int, set] = {}
    for vs, _ in factors:
        for a in vs:
            adj.setdefault(a, set()).update(b for b in vs if b != a)
    fs = list(factors)
    while adj:
        v = min(adj, key=lambda u: (len(adj[u]), u))       # min-degree, lowest id
        nb = adj.pop(v)
        for a in nb:
            adj[a] |= nb - {a}
            adj[a].discard(v)
        bucket = [f for f in fs if v in f[0]]
        fs = [f for f in fs if v not in f[0]]
        union = sorted(set().union(*[set(f[0]) for f in bucket]))
        name = {u: letters[i] for i, u in enumerate(union)}
        spec = ",".join("".join(name[u] for u in vs) for vs, _ in bucket)
        out = [u for u in union if u != v]
        fs.append((tuple(out), np.einsum(spec + "->" + "".join(name[u] for u in out),
                                         *[a for _, a in bucket])))
    return complex(np.prod([complex(a) for _, a in fs]))


def amplitude_network(n: int, gates, x) -> complex:
    factors, _ = network(n, gates, x)
    return _eliminate(factors)


def restrict(factors: List[Factor], fixed: Dict[int, int]) -> List[Factor]:
    out = []
    for vs, a in factors:
        idx = tuple(fixed[v] if v in fixed else slice(None) for v in vs)
        out.append((tuple(v for v in vs if v not in fixed), np.asarray(a[idx])))
    return out


def sliced_network(n: int, gates, x, cut_segments: Sequence[int]) -> complex:
    """Sum over the 2^m assignments of the given wire variables (Eq. (2))."""
    factors, _ = network(n, gates, x)
    tot = 0j
    for bits in itertools.product((0, 1), repeat=len(cut_segments)):
        tot += _eliminate(restrict(factors, dict(zip(cut_segments, bits))))
    return tot
