"""Plain complex128 reference for the QAOA single-amplitude tensor network.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every routine here is
written for a reader checking it against the paper by eye; nothing is blocked,
fused or reordered.

Readings of the paper used throughout (the paper gives no gate definitions
for its QAOA workload, Sec. IV A):
  * circuit: H on every qubit of |0^n>, then for each layer l = 0..p-1 the
    phase exp(-i gamma_l Z_i Z_j) on every graph edge followed by
    RX(2 beta_l) = exp(-i beta_l X) on every qubit;
  * result: the complex amplitude <x| U |0^n> of one output bitstring x
    (byte i of x = qubit i = graph vertex i); the paper's density-matrix
    quantity tr(E rho) with E = |x><x| equals |amplitude|^2 (Sec. II A);
  * network form: the ZZ phases are diagonal, so the wire of qubit i keeps one
    binary index variable v(i, l) = l*n + i through all ZZ gates of layer l.
    A cut "edge" of Sec. III A is such an index variable, fixed to 0 or 1
    (two values per variable instead of the four values of a density-matrix
    edge; one density-matrix cut equals two binary cuts).
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

Factor = Tuple[Tuple[int, ...], np.ndarray]


def variable_id(n: int, qubit: int, layer: int) -> int:
    """Index variable of qubit `qubit` during the ZZ gates of layer `layer`."""
    return layer * n + qubit


def _rx_entry(beta: float, a: int, b: int) -> complex:
    """<a| exp(-i beta X) |b>: cos(beta) on the diagonal, -i sin(beta) off it."""
    return complex(math.cos(beta), 0.0) if a == b else complex(0.0, -math.sin(beta))


def qaoa_factors(n: int, edges: Sequence[Tuple[int, int]], p: int,
                 gamma: Sequence[float], beta: Sequence[float],
                 x: Sequence[int]) -> Tuple[List[Factor], float]:
    """Factors of the undirected-graph tensor network (Sec. II A, Fig. 1).

    Vertices of the paper's graph are gates, inputs and measurements; edges are
    wires, i.e. index variables.  Returned here as (variables, array) pairs,
    array axes in the listed variable order, plus the scalar 2^{-n/2} from the
    Hadamard layer acting on |0^n>.
      ZZ  over (v(i,l), v(j,l)):  exp(-i gamma_l (-1)^{a xor b})
      RX  over (v(i,l+1), v(i,l)), l < p-1:  <a|RX(2 beta_l)|b>
      OUT over (v(i,p-1),):  <x_i|RX(2 beta_{p-1})|b>
    """
    factors: List[Factor] = []
    for l in range(p):
        for (i, j) in edges:
            t = np.empty((2, 2), dtype=np.complex128)
            for a in (0, 1):
                for b in (0, 1):
                    zz = 1.0 if a == b else -1.0
                    t[a, b] = complex(math.cos(gamma[l] * zz), -math.sin(gamma[l] * zz))
            factors.append(((variable_id(n, i, l), variable_id(n, j, l)), t))
    for l in range(p - 1):
        r = np.array([[_rx_entry(beta[l], a, b) for b in (0, 1)] for a in (0, 1)],
                     dtype=np.complex128)
        for i in range(n):
            factors.append(((variable_id(n, i, l + 1), variable_id(n, i, l)), r))
    for i in range(n):
        xi = int(x[i])
        t = np.array([_rx_entry(beta[p - 1], xi, b) for b in (0, 1)], dtype=np.complex128)
        factors.append(((variable_id(n, i, p - 1),), t))
    return factors, 2.0 ** (-n / 2.0)


# ---------------------------------------------------------------------------
# Independent pins: statevector and brute force
# ---------------------------------------------------------------------------

def statevector(n: int, edges, p: int, gamma, beta) -> np.ndarray:
    """Full 2^n state U|0^n>, index sum_i x_i 2^i (little-endian), for n <= 20."""
    if n > 22:
        raise ValueError("statevector only for small n")
    dim = 1 << n
    idx = np.arange(dim, dtype=np.int64)
    bits = [((idx >> i) & 1) for i in range(n)]
    zz_sum = np.zeros(dim, dtype=np.float64)
    for (i, j) in edges:
        zz_sum += np.where(bits[i] == bits[j], 1.0, -1.0)
    psi = np.full(dim, 2.0 ** (-n / 2.0), dtype=np.complex128)   # H^n |0^n>
    for l in range(p):
        psi = psi * np.exp(-1j * gamma[l] * zz_sum)
        rx = np.array([[_rx_entry(beta[l], a, b) for b in (0, 1)] for a in (0, 1)])
        for q in range(n):
            v = psi.reshape(dim >> (q + 1), 2, 1 << q)
            psi = np.einsum("ab,ubv->uav", rx, v).reshape(dim)
    return psi


def statevector_amplitude(n, edges, p, gamma, beta, x) -> complex:
    psi = statevector(n, edges, p, gamma, beta)
    return complex(psi[sum(int(b) << i for i, b in enumerate(x))])


def brute_force_amplitude(n, edges, p, gamma, beta, x,
                          fixed: Optional[Dict[int, int]] = None) -> complex:
    """Sum over every assignment of the n*p index variables of the factor
    product (pure Python, only for n*p <= ~18).  `fixed` pins some variables
    (a slice of Sec. III A, Eq. (2))."""
    factors, scalar = qaoa_factors(n, edges, p, gamma, beta, x)
    nv = n * p
    fixed = fixed or {}
    free = [v for v in range(nv) if v not in fixed]
    total = 0j
    for vals in itertools.product((0, 1), repeat=len(free)):
        a = dict(fixed)
        a.update(zip(free, vals))
        term = 1 + 0j
        for vs, t in factors:
            term *= t[tuple(a[v] for v in vs)]
        total += term
    return total * scalar


# ---------------------------------------------------------------------------
# Variable elimination (Eq. (1) pairwise contraction, Sec. II A)
# ---------------------------------------------------------------------------

def restrict_factors(factors: List[Factor], fixed: Dict[int, int]) -> List[Factor]:
    """Fix each cut variable to its slice bit in every factor that holds it
    (the 'additional vertices' of Fig. 3 carry the fixed value)."""
    out = []
    for vs, t in factors:
        if not any(v in fixed for v in vs):
            out.append((vs, t))
            continue
        index = tuple(fixed[v] if v in fixed else slice(None) for v in vs)
        out.append((tuple(v for v in vs if v not in fixed), np.asarray(t[index])))
    return out


def _expand(t: np.ndarray, vs: Tuple[int, ...], union: List[int]) -> np.ndarray:
    """View of t with one axis per union variable (size 1 where t lacks it)."""
    present = sorted(vs, key=union.index)
    t = np.transpose(t, [vs.index(v) for v in present])
    shape = [2 if v in vs else 1 for v in union]
    return t.reshape(shape)


def eliminate(factors: List[Factor], order: Iterable[int]) -> complex:
    """Bucket elimination: for each variable, multiply every factor that holds
    it into one array over the union of their variables and sum that variable
    out (Eq. (1) applied to a whole bucket); finally multiply the rank-0
    leftovers (Sec. II A: the contraction ends in a rank-0 tensor)."""
    pool = list(factors)
    for v in order:
        bucket = [f for f in pool if v in f[0]]
        pool = [f for f in pool if v not in f[0]]
        if not bucket:
            continue
        union = sorted(set().union(*[set(vs) for vs, _ in bucket]))
        prod = np.ones([2] * len(union), dtype=np.complex128)
        for vs, t in bucket:
            prod = prod * _expand(t, vs, union)
        summed = prod.sum(axis=union.index(v))
        pool.append((tuple(u for u in union if u != v), summed))
    result = 1 + 0j
    for vs, t in pool:
        if vs:
            raise ValueError("order does not cover variables %s" % (vs,))
        result *= complex(t)
    return result


def interaction_graph(n: int, edges, p: int,
                      removed: Iterable[int] = ()) -> List[set]:
    """Line graph of the network (Sec. II B): one vertex per index variable,
    joined when two variables meet in one factor; `removed` (cut) variables are
    dropped, as fixing them removes them from every factor."""
    removed = set(removed)
    nv = n * p
    adj = [set() for _ in range(nv)]

    def join(u, w):
        if u in removed or w in removed:
            return
        adj[u].add(w)
        adj[w].add(u)

    for l in range(p):
        for (i, j) in edges:
            join(variable_id(n, i, l), variable_id(n, j, l))
    for l in range(p - 1):
        for i in range(n):
            join(variable_id(n, i, l + 1), variable_id(n, i, l))
    return adj


def min_degree_order(adj: List[set], removed: Iterable[int] = ()) -> List[int]:
    """Greedy minimum-degree elimination order, ties to the lowest id."""
    removed = set(removed)
    g = {v: set(a) - removed for v, a in enumerate(adj) if v not in removed}
    order = []
    while g:
        v = min(g, key=lambda u: (len(g[u]), u))
        nb = g.pop(v)
        for a in nb:
            g[a] |= nb - {a}
            g[a].discard(v)
        order.append(v)
    return order


def min_fill_order(adj: List[set], removed: Iterable[int] = ()):
    """Greedy minimum-fill elimination order (stands in for the paper's QuickBB,
    Sec. II B): pick the variable adding the fewest fill edges, then the lowest
    degree, then the lowest id.  Returns (order, higher-neighbour sets)."""
    removed = set(removed)
    g = {v: set(a) - removed for v, a in enumerate(adj) if v not in removed}
    order, nplus = [], []

    def fill(u):
        nb = sorted(g[u])
        return sum(1 for a, b in itertools.combinations(nb, 2) if b not in g[a])

    while g:
        v = min(g, key=lambda u: (fill(u), len(g[u]), u))
        nb = g.pop(v)
        for a in nb:
            g[a] |= nb - {a}
            g[a].discard(v)
        order.append(v)
        nplus.append(frozenset(nb))
    return order, nplus


def elimination_cost(adj: List[set], order: Sequence[int], removed=()) -> Tuple[int, int]:
    """(width, work) of eliminating `order` on the graph: width is the largest
    neighbour set met at elimination (= max bag size - 1, Sec. II B; = largest
    tensor rank created); work is sum over variables of 2^(|N+(v)|+1), the
    size of each bucket's index space."""
    removed = set(removed)
    g = {v: set(a) - removed for v, a in enumerate(adj) if v not in removed}
    width, work = 0, 0
    for v in order:
        nb = g.pop(v)
        for a in nb:
            g[a] |= nb - {a}
            g[a].discard(v)
        width = max(width, len(nb))
        work += 1 << (len(nb) + 1)
    if g:
        raise ValueError("order incomplete")
    return width, work


def bags_from_order(adj: List[set], order: Sequence[int], removed=()):
    """Tree decomposition from an elimination order: bag(v) = {v} u N+(v); the
    parent of bag(v) is the bag of the earliest-eliminated member of N+(v)."""
    removed = set(removed)
    g = {v: set(a) - removed for v, a in enumerate(adj) if v not in removed}
    pos = {v: i for i, v in enumerate(order)}
    bags, parent = {}, {}
    for v in order:
        nb = g.pop(v)
        for a in nb:
            g[a] |= nb - {a}
            g[a].discard(v)
        bags[v] = frozenset(nb | {v})
        parent[v] = min(nb, key=lambda u: pos[u]) if nb else None
    return bags, parent


def check_tree_decomposition(adj: List[set], bags: Dict[int, frozenset],
                             parent: Dict[int, Optional[int]], removed=()) -> int:
    """Checks the three conditions of Sec. II B and returns the width
    max|B|-1: (1) the bags cover every vertex, (2) every edge lies in a bag,
    (3) the bags holding one vertex form a connected subtree."""
    removed = set(removed)
    verts = [v for v in range(len(adj)) if v not in removed]
    covered = set().union(*bags.values()) if bags else set()
    assert set(verts) <= covered, "condition (1) fails"
    for u in verts:
        for w in adj[u]:
            if w in removed:
                continue
            assert any(u in b and w in b for b in bags.values()), "condition (2) fails"
    # tree edges
    tedges = [(c, p) for c, p in parent.items() if p is not None]
    for v in verts:
        holders = {b for b, bag in bags.items() if v in bag}
        # connected within the forest restricted to holders
        start = next(iter(holders))
        seen, stack = {start}, [start]
        while stack:
            c = stack.pop()
            for a, b in tedges:
                for x, y in ((a, b), (b, a)):
                    if x == c and y in holders and y not in seen:
                        seen.add(y)
                        stack.append(y)
        assert seen == holders, "condition (3) fails for %d" % v
    return max(len(b) for b in bags.values()) - 1 if bags else -1


def exact_treewidth(adj: List[set]) -> int:
    """Exact treewidth by the subset recursion
    TW(S) = min_{v in S} max(TW(S - v), |Q(S - v, v)|), where Q(S, v) is the set
    of vertices outside S u {v} reachable from v through S.  Tiny graphs only."""
    nv = len(adj)
    full = (1 << nv) - 1
    from functools import lru_cache

    def q(s: int, v: int) -> int:
        seen = {v}
        stack = [v]
        count = 0
        while stack:
            u = stack.pop()
            for w in adj[u]:
                if w in seen:
                    continue
                seen.add(w)
                if (s >> w) & 1:
                    stack.append(w)
                else:
                    count += 1
        return count

    @lru_cache(maxsize=None)
    def tw(s: int) -> int:
        if s == 0:
            return -1
        best = nv
        for v in range(nv):
            if (s >> v) & 1:
                rest = s & ~(1 << v)
                best = min(best, max(tw(rest), q(rest, v)))
        return best

    return tw(full)


def ve_amplitude(n, edges, p, gamma, beta, x, order: Optional[Sequence[int]] = None) -> complex:
    """Uncut contraction of the whole network (rank-0 result, Sec. II A)."""
    factors, scalar = qaoa_factors(n, edges, p, gamma, beta, x)
    if order is None:
        order = min_degree_order(interaction_graph(n, edges, p))
    return eliminate(factors, order) * scalar


def slice_partial(n, edges, p, gamma, beta, x, cut: Sequence[int], s: int,
                  order: Optional[Sequence[int]] = None) -> complex:
    """Contraction of slice s: cut variable cut[b] fixed to bit b of s
    (least significant bit first) in every factor (Eq. (2), Fig. 3)."""
    fixed = {int(c): (s >> b) & 1 for b, c in enumerate(cut)}
    factors, scalar = qaoa_factors(n, edges, p, gamma, beta, x)
    factors = restrict_factors(factors, fixed)
    if order is None:
        order = min_degree_order(interaction_graph(n, edges, p), removed=fixed)
    else:
        order = [v for v in order if v not in fixed]
    return eliminate(factors, order) * scalar


def neumaier_sum(values: Iterable[float]) -> Tuple[float, float]:
    """Compensated (Neumaier) sum in the given order: returns (sum, compensation)."""
    s, c = 0.0, 0.0
    for v in values:
        t = s + v
        if abs(s) >= abs(v):
            c += (s - t) + v
        else:
            c += (v - t) + s
        s = t
    return s, c


def sliced_amplitude(n, edges, p, gamma, beta, x, cut, slices: Optional[Iterable[int]] = None,
                     order=None) -> complex:
    """Sum of slice partials in ascending slice order (Eq. (2); the master-side
    sum of one complex value per subgraph, Sec. III A)."""
    if slices is None:
        slices = range(1 << len(cut))
    parts = [slice_partial(n, edges, p, gamma, beta, x, cut, s, order) for s in slices]
    re = neumaier_sum(z.real for z in parts)
    im = neumaier_sum(z.imag for z in parts)
    return complex(re[0] + re[1], im[0] + im[1])


def closed_form_amplitude(n, edges, p, gamma, beta, x) -> Optional[complex]:
    """Closed forms that follow from the circuit's algebra, or None:
      gamma = 0 (all layers): RX(2b)|+> = e^{-ib}|+>, so amp = e^{-i n sum(beta)} 2^{-n/2};
      beta = 0 (all layers): RX = I, amp = 2^{-n/2} e^{-i G (|E| - 2 cut(x))}, G = sum(gamma);
      beta = pi/2 (all layers): RX(pi) = -iX commutes with ZZ, so
          amp = (-i)^{np} 2^{-n/2} e^{-i G (|E| - 2 cut(x))}."""
    cutx = sum(1 for (i, j) in edges if int(x[i]) != int(x[j]))
    G = float(sum(gamma))
    base = 2.0 ** (-n / 2.0)
    if all(g == 0.0 for g in gamma):
        ph = -n * float(sum(beta))
        return base * complex(math.cos(ph), math.sin(ph))
    if all(b == 0.0 for b in beta):
        ph = -G * (len(edges) - 2 * cutx)
        return base * complex(math.cos(ph), math.sin(ph))
    if all(b == math.pi / 2 for b in beta):
        ph = -G * (len(edges) - 2 * cutx)
        return base * ((-1j) ** (n * p)) * complex(math.cos(ph), math.sin(ph))
    return None
