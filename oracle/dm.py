"""Density-matrix (Markov-Shi) form of the QAOA network, complex128.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written from Sec. II A:
every wire of the circuit is an edge carrying a 4-valued index over the
operator basis Pi = {|0><0|, |0><1|, |1><0|, |1><1|} (index 2a + b for
|a><b|); every gate is a vertex with a tensor
    input        T_sigma          = tr(rho_in sigma)
    one qubit    T_{sigma,tau}    = tr(tau^dagger G(sigma)),  G(s) = U s U^dagger
    two qubits   T_{s1 s2, t1 t2} = tr((t1 (x) t2)^dagger G(s1 (x) s2))
    measurement  T_tau            = tr(E tau),  E = |x><x|
and the rank-0 contraction of the network is tr(E rho_out), the probability
of bitstring x.  Nothing here is merged or factorised: every wire segment
between two gates is its own 4-valued variable, the circuit is H on |0> then
p layers of exp(-i gamma Z Z) on every edge and RX(2 beta) on every qubit.

Slicing (Sec. III A, Eq. (2), Fig. 3): fixing one 4-valued edge to each of
its four values and summing the four restricted contractions gives the
uncut result; m cut edges give 4^m subgraphs.

Pinned in tests/test_oracle_dm.py against |amplitude|^2 of the independent
2^n statevector, and by the slice identity.
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

BASIS = [np.array([[1, 0], [0, 0]], dtype=np.complex128),   # |0><0|
         np.array([[0, 1], [0, 0]], dtype=np.complex128),   # |0><1|
         np.array([[0, 0], [1, 0]], dtype=np.complex128),   # |1><0|
         np.array([[0, 0], [0, 1]], dtype=np.complex128)]   # |1><1|


def input_tensor(rho: np.ndarray) -> np.ndarray:
    """T_sigma = tr(rho sigma)."""
    return np.array([np.trace(rho @ s) for s in BASIS], dtype=np.complex128)


def gate1_tensor(U: np.ndarray) -> np.ndarray:
    """T[sigma, tau] = tr(tau^dagger U sigma U^dagger) for a one-qubit gate."""
    T = np.empty((4, 4), dtype=np.complex128)
    for i, s in enumerate(BASIS):
        g = U @ s @ U.conj().T
        for j, t in enumerate(BASIS):
            T[i, j] = np.trace(t.conj().T @ g)
    return T


def gate2_tensor(U: np.ndarray) -> np.ndarray:
    """T[s1, s2, t1, t2] = tr((t1 (x) t2)^dagger U (s1 (x) s2) U^dagger),
    qubit 1 the more significant factor of the 4x4 matrix U."""
    T = np.empty((4, 4, 4, 4), dtype=np.complex128)
    for i1, s1 in enumerate(BASIS):
        for i2, s2 in enumerate(BASIS):
            g = U @ np.kron(s1, s2) @ U.conj().T
            for j1, t1 in enumerate(BASIS):
                for j2, t2 in enumerate(BASIS):
                    T[i1, i2, j1, j2] = np.trace(np.kron(t1, t2).conj().T @ g)
    return T


def measure_tensor(bit: int) -> np.ndarray:
    """T_tau = tr(E tau) with E = |bit><bit|."""
    E = np.zeros((2, 2), dtype=np.complex128)
    E[bit, bit] = 1.0
    return np.array([np.trace(E @ t) for t in BASIS], dtype=np.complex128)


def _H() -> np.ndarray:
    return np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)


def _RX(beta: float) -> np.ndarray:
    c, s = math.cos(beta), math.sin(beta)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def _ZZ(gamma: float) -> np.ndarray:
    d = [complex(math.cos(gamma * z), -math.sin(gamma * z)) for z in (1, -1, -1, 1)]
    return np.diag(d).astype(np.complex128)


Factor = Tuple[Tuple[int, ...], np.ndarray]


def dm_network(n: int, edges, p: int, gamma, beta, x) -> Tuple[List[Factor], Dict[Tuple[int, int], int]]:
    """Factors of the density-matrix network over 4-valued wire variables.
    Returns the factors and, for each (qubit, layer l), the variable of the
    qubit's wire segment that enters the ZZ gates of layer l (the segment a
    cut of the merged ket variable v(qubit, l) corresponds to)."""
    factors: List[Factor] = []
    nxt = [0]

    def new_var() -> int:
        nxt[0] += 1
        return nxt[0] - 1

    wire = [new_var() for _ in range(n)]
    rho0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
    for q in range(n):
        factors.append(((wire[q],), input_tensor(rho0)))
    Th = gate1_tensor(_H())
    for q in range(n):
        w = new_var()
        factors.append(((wire[q], w), Th))
        wire[q] = w
    entry: Dict[Tuple[int, int], int] = {}
    for l in range(p):
        for q in range(n):
            entry[(q, l)] = wire[q]
        Tz = gate2_tensor(_ZZ(gamma[l]))
        for (i, j) in edges:
            wi, wj = new_var(), new_var()
            factors.append(((wire[i], wire[j], wi, wj), Tz))
            wire[i], wire[j] = wi, wj
        Tr = gate1_tensor(_RX(beta[l]))
        for q in range(n):
            w = new_var()
            factors.append(((wire[q], w), Tr))
            wire[q] = w
    for q in range(n):
        factors.append(((wire[q],), measure_tensor(int(x[q]))))
    return factors, entry


def _eliminate(factors: List[Factor], order: Sequence[int]) -> complex:
    """Variable elimination over 4-valued variables (Eq. (1) per bucket)."""
    letters = "abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ"
    fs = list(factors)
    for v in order:
        bucket = [f for f in fs if v in f[0]]
        fs = [f for f in fs if v not in f[0]]
        if not bucket:
            continue
        union = sorted(set().union(*[set(f[0]) for f in bucket]))
        if len(union) > len(letters):
            raise ValueError("bucket too large")
        name = {u: letters[i] for i, u in enumerate(union)}
        spec = ",".join("".join(name[u] for u in vs) for vs, _ in bucket)
        out = [u for u in union if u != v]
        t = np.einsum(spec + "->" + "".join(name[u] for u in out), *[a for _, a in bucket])
        fs.append((tuple(out), t))
    return complex(np.prod([complex(a) for _, a in fs]))


def _min_degree(factors: List[Factor]) -> List[int]:
    adj: Dict[int, set] = {}
    for vs, _ in factors:
        for a in vs:
            adj.setdefault(a, set()).update(b for b in vs if b != a)
    order = []
    while adj:
        v = min(adj, key=lambda u: (len(adj[u]), u))
        nb = adj.pop(v)
        for a in nb:
            adj[a] |= nb - {a}
            adj[a].discard(v)
        order.append(v)
    return order


def restrict(factors: List[Factor], fixed: Dict[int, int]) -> List[Factor]:
    """Fix 4-valued variables to basis indices (Fig. 3)."""
    out = []
    for vs, a in factors:
        idx = tuple(fixed[v] if v in fixed else slice(None) for v in vs)
        out.append((tuple(v for v in vs if v not in fixed), np.asarray(a[idx])))
    return out


def dm_probability(n: int, edges, p: int, gamma, beta, x) -> complex:
    """tr(E rho_out) by contracting the whole density-matrix network."""
    factors, _ = dm_network(n, edges, p, gamma, beta, x)
    return _eliminate(factors, _min_degree(factors))


def dm_slice(n: int, edges, p: int, gamma, beta, x, cut_pairs: Sequence[Tuple[int, int]],
             sigmas: Sequence[int]) -> complex:
    """Contraction with the wire segments entering layer l of qubit q fixed,
    for each (q, l) of cut_pairs, to the basis index sigmas[j] (0..3)."""
    factors, entry = dm_network(n, edges, p, gamma, beta, x)
    fixed = {entry[c]: int(s) for c, s in zip(cut_pairs, sigmas)}
    fs = restrict(factors, fixed)
    return _eliminate(fs, _min_degree(fs))


def dm_sliced_sum(n, edges, p, gamma, beta, x, cut_pairs) -> complex:
    """Sum of the 4^m slice contractions (Sec. III A)."""
    tot = 0j
    for sig in itertools.product(range(4), repeat=len(cut_pairs)):
        tot += dm_slice(n, edges, p, gamma, beta, x, cut_pairs, sig)
    return tot
