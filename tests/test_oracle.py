"""Pins of the CPU oracle against facts that do not come from the oracle itself:
an independent statevector simulation, brute-force sums, closed forms of the
circuit, symmetries, the slice identity of Eq. (2), textbook treewidths, the
published SplitMix64 outputs and finite differences."""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from oracle import qaoa as Q
from oracle.search import splitmix64, ga_cut_search, cut_fitness, ga_min_k
from oracle.mlp import MLP64
from instances import make_instance, random_regular_graph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _inst(n, p, seed, B=1):
    return make_instance(n, p, B, seed)


def _args(inst, b=0):
    return inst.n, inst.edges, inst.p, inst.gamma, inst.beta, inst.bitstrings[b]


@pytest.mark.parametrize("n,p,seed", [(6, 1, 0), (6, 2, 1), (8, 2, 2), (10, 1, 3),
                                      (12, 2, 4), (16, 1, 5)])
def test_ve_matches_statevector(n, p, seed):
    inst = _inst(n, p, seed, B=4)
    psi = Q.statevector(inst.n, inst.edges, inst.p, inst.gamma, inst.beta)
    assert abs(np.vdot(psi, psi) - 1.0) < 1e-12
    for b in range(4):
        x = inst.bitstrings[b]
        ref = psi[sum(int(v) << i for i, v in enumerate(x))]
        got = Q.ve_amplitude(*_args(inst, b))
        assert abs(got - ref) <= 1e-12 * max(abs(ref), 2.0 ** (-n / 2))


@pytest.mark.parametrize("n,p,seed", [(6, 1, 7), (6, 2, 8), (8, 2, 9)])
def test_ve_matches_brute_force(n, p, seed):
    inst = _inst(n, p, seed, B=2)
    for b in range(2):
        bf = Q.brute_force_amplitude(*_args(inst, b))
        got = Q.ve_amplitude(*_args(inst, b))
        assert abs(got - bf) <= 1e-13 * max(abs(bf), 2.0 ** (-n / 2))


def test_zero_angles_exact():
    """gamma = beta = 0: every sum is of 0/1 terms, so 2^{-n/2} exactly."""
    inst = _inst(16, 1, 11, B=3)
    for b in range(3):
        x = inst.bitstrings[b]
        amp = Q.ve_amplitude(16, inst.edges, 1, [0.0], [0.0], x)
        assert amp == complex(2.0 ** -8, 0.0)
        # a cut slice that disagrees with x is exactly zero, the agreeing one exact
        cut = [3, 9]
        for s in range(4):
            part = Q.slice_partial(16, inst.edges, 1, [0.0], [0.0], x, cut, s)
            agree = all(((s >> k) & 1) == int(x[c]) for k, c in enumerate(cut))
            assert part == (complex(2.0 ** -8, 0.0) if agree else 0j)


@pytest.mark.parametrize("which", ["gamma0", "beta0", "betapi2"])
@pytest.mark.parametrize("n,p", [(8, 1), (10, 2), (16, 1)])
def test_closed_forms(which, n, p):
    inst = _inst(n, p, 21 + n + p, B=2)
    gamma, beta = list(inst.gamma), list(inst.beta)
    if which == "gamma0":
        gamma = [0.0] * p
    elif which == "beta0":
        beta = [0.0] * p
    else:
        beta = [math.pi / 2] * p
    for b in range(2):
        x = inst.bitstrings[b]
        ref = Q.closed_form_amplitude(n, inst.edges, p, gamma, beta, x)
        got = Q.ve_amplitude(n, inst.edges, p, gamma, beta, x)
        assert abs(got - ref) <= 1e-13 * 2.0 ** (-n / 2)
        if n <= 10:
            sv = Q.statevector_amplitude(n, inst.edges, p, gamma, beta, x)
            assert abs(sv - ref) <= 1e-13 * 2.0 ** (-n / 2)


def test_norm_over_all_bitstrings():
    n, p = 8, 2
    inst = _inst(n, p, 31)
    tot = 0.0
    order = Q.min_degree_order(Q.interaction_graph(n, inst.edges, p))
    for bits in itertools.product((0, 1), repeat=n):
        a = Q.ve_amplitude(n, inst.edges, p, inst.gamma, inst.beta, bits, order=order)
        tot += abs(a) ** 2
    assert abs(tot - 1.0) < 1e-12


def test_symmetries():
    n, p = 12, 2
    inst = _inst(n, p, 41, B=2)
    x = inst.bitstrings[0]
    a = Q.ve_amplitude(*_args(inst))
    xbar = 1 - x
    assert abs(Q.ve_amplitude(n, inst.edges, p, inst.gamma, inst.beta, xbar) - a) < 1e-14
    conj = Q.ve_amplitude(n, inst.edges, p, [-g for g in inst.gamma],
                          [-b for b in inst.beta], x)
    assert abs(conj - a.conjugate()) < 1e-14
    # p = 1: gamma -> gamma + pi multiplies by (-1)^{|E|}
    inst1 = _inst(10, 1, 42)
    a1 = Q.ve_amplitude(*_args(inst1))
    a2 = Q.ve_amplitude(10, inst1.edges, 1, [inst1.gamma[0] + math.pi], inst1.beta,
                        inst1.bitstrings[0])
    assert abs(a2 - (-1) ** len(inst1.edges) * a1) < 1e-14
    # vertex relabelling
    perm = np.random.default_rng(3).permutation(n)
    edges = [(int(perm[i]), int(perm[j])) for i, j in inst.edges]
    xp = np.zeros(n, dtype=np.uint8)
    for i in range(n):
        xp[perm[i]] = x[i]
    a3 = Q.ve_amplitude(n, edges, p, inst.gamma, inst.beta, xp)
    assert abs(a3 - a) < 1e-14


def test_order_independence():
    n, p = 12, 2
    inst = _inst(n, p, 43)
    adj = Q.interaction_graph(n, inst.edges, p)
    a = Q.ve_amplitude(*_args(inst), order=Q.min_degree_order(adj))
    b = Q.ve_amplitude(*_args(inst), order=Q.min_fill_order(adj)[0])
    c = Q.ve_amplitude(*_args(inst), order=list(range(n * p)))
    assert abs(a - b) < 1e-14 and abs(a - c) < 1e-14


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_slice_sum_equals_uncut(k):
    n, p = 8, 2
    inst = _inst(n, p, 50 + k)
    rng = np.random.default_rng(k)
    cut = sorted(int(c) for c in rng.choice(n * p, size=k, replace=False))
    uncut = Q.ve_amplitude(*_args(inst))
    total = Q.sliced_amplitude(*_args(inst), cut)
    assert abs(total - uncut) < 1e-14
    # each slice against brute force with the cut bits held fixed (pins the bit map)
    for s in range(1 << k):
        fixed = {c: (s >> b) & 1 for b, c in enumerate(cut)}
        bf = Q.brute_force_amplitude(*_args(inst), fixed=fixed)
        part = Q.slice_partial(*_args(inst), cut, s)
        assert abs(part - bf) < 1e-14


def test_neumaier():
    vals = [1.0, 1e100, 1.0, -1e100]
    s, c = Q.neumaier_sum(vals)
    assert s + c == 2.0


def _golden_graphs():
    out = []
    with open(os.path.join(GOLDEN, "treewidth.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            edges = [tuple(int(t) for t in e.split("-")) for e in parts[2:]]
            out.append((parts[0], int(parts[1]), edges))
    return out


@pytest.mark.parametrize("name,tw,edges", _golden_graphs())
def test_treewidth_and_decompositions(name, tw, edges):
    nv = 1 + max(max(e) for e in edges)
    adj = [set() for _ in range(nv)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    assert Q.exact_treewidth(adj) == tw
    order, nplus = Q.min_fill_order(adj)
    bags, parent = Q.bags_from_order(adj, order)
    width = Q.check_tree_decomposition(adj, bags, parent)
    assert width >= tw
    assert width == Q.elimination_cost(adj, order)[0] == max(len(s) for s in nplus)


def test_tree_decomposition_of_qaoa_networks():
    for n, p, seed in [(16, 1, 0), (20, 2, 1), (40, 2, 2)]:
        inst = _inst(n, p, seed)
        adj = Q.interaction_graph(n, inst.edges, p)
        cut = list(range(0, n * p, 7))[:4]
        order, _ = Q.min_fill_order(adj, removed=cut)
        bags, parent = Q.bags_from_order(adj, order, removed=cut)
        w = Q.check_tree_decomposition(adj, bags, parent, removed=cut)
        assert w == Q.elimination_cost(adj, order, removed=cut)[0]


def test_interaction_graph_shape():
    n = 10
    inst = _inst(n, 2, 5)
    adj = Q.interaction_graph(n, inst.edges, 2)
    degs = sorted(len(a) for a in adj)
    assert degs == [4] * (2 * n)            # 3 graph neighbours + the other layer
    adj1 = Q.interaction_graph(n, inst.edges, 1)
    assert all(len(a) == 3 for a in adj1)


def test_splitmix64_published_outputs():
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            seed, idx, out = (int(t) for t in line.split())
            assert splitmix64(seed, idx) == out


def test_ga_invariants():
    inst = _inst(20, 2, 60)
    adj = Q.interaction_graph(20, inst.edges, 2)
    M = 5
    cut, (w, work) = ga_cut_search(adj, M, N=11, T=4, seed=9)
    assert len(cut) == M and len(set(cut)) == M
    assert cut_fitness(adj, cut)[:2] == (w, work)
    # best is never worse than uncut-by-nothing random draws of the first generation
    again = ga_cut_search(adj, M, N=11, T=4, seed=9)
    assert again == (cut, (w, work))
    w0 = Q.elimination_cost(adj, Q.min_fill_order(adj)[0])[0]
    assert w <= w0
    res = ga_min_k(adj, max_rank=w0 - 2, k_max=8, seed=1)
    assert res is not None and res[1][0] <= w0 - 2


def test_paper_counts():
    vals = {}
    with open(os.path.join(GOLDEN, "paper_counts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            vals[k] = int(v)
    assert 4 ** vals["dm_cuts"] == vals["subgraphs"] == 2 ** (2 * vals["dm_cuts"])
    assert -(-vals["subgraphs"] // vals["cores"]) == vals["rounds"]


def test_mlp_gradients_finite_difference():
    rng = np.random.default_rng(0)
    dims = [7, 16, 16, 16, 2]
    W = [rng.normal(0, 0.4, (a, b)) for a, b in zip(dims[:-1], dims[1:])]
    bs = [rng.normal(0, 0.1, b) for b in dims[1:]]
    m = MLP64(W, bs)
    x = rng.normal(size=(9, 7))
    y = rng.normal(size=(9, 2))
    loss, gW, gb = m.loss_and_grads(x, y)
    h = 1e-6
    for li in range(4):
        for (i, j) in [(0, 0), (1, 1), (W[li].shape[0] - 1, W[li].shape[1] - 1)]:
            m.W[li][i, j] += h
            lp = m.loss_and_grads(x, y)[0]
            m.W[li][i, j] -= 2 * h
            lm = m.loss_and_grads(x, y)[0]
            m.W[li][i, j] += h
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gW[li][i, j]) <= 1e-6 * max(1.0, abs(fd))
        j = 0
        m.b[li][j] += h
        lp = m.loss_and_grads(x, y)[0]
        m.b[li][j] -= 2 * h
        lm = m.loss_and_grads(x, y)[0]
        m.b[li][j] += h
        assert abs((lp - lm) / (2 * h) - gb[li][j]) <= 1e-6
    # Adam decreases the loss on a fixed batch
    for _ in range(50):
        _, gW, gb = m.loss_and_grads(x, y)
        m.adam_step(gW, gb, lr=1e-2)
    assert m.loss_and_grads(x, y)[0] < loss


def test_min_fill_tie_rule_hand_derived():
    d = {}
    with open(os.path.join(GOLDEN, "minfill_order.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            d[k] = v
    edges = [tuple(int(t) for t in e.split("-")) for e in d["edges"]]
    adj = [set() for _ in range(6)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    order, nplus = Q.min_fill_order(adj)
    assert order == [int(t) for t in d["minfill"]]
    assert [len(s) for s in nplus] == [int(t) for t in d["minfill_nplus"]]
    assert Q.min_degree_order(adj)[0] == int(d["mindegree_first"][0])


def test_adam_step_hand_computed():
    """Pins MLP64.adam_step to three Adam updates of one scalar computed by hand
    from the published rule (tests/golden/adam_scalar.txt): a dropped bias
    correction, a misplaced eps or a wrong moment update changes the digits."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "adam_scalar.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    net = MLP64([np.array([[1.0]])], [np.array([0.0])])
    for t, g, w in rows:
        net.adam_step([np.array([[float(g)]])], [np.array([0.0])], lr=0.1, b1=0.9, b2=0.999,
                      eps=0.1)
        assert net.t == int(t)
        assert abs(net.W[0][0, 0] - float(w)) <= 2e-16, (t, net.W[0][0, 0], w)
        assert net.b[0][0] == 0.0   # a zero gradient leaves its parameter unchanged


def _golden_costs():
    out = []
    for line in open(os.path.join(GOLDEN, "elimination_cost.txt")):
        if line.strip() and not line.startswith("#"):
            f = line.split()
            order = [int(v) for v in f[3].split(",")]
            edges = [tuple(int(v) for v in e.split("-")) for e in f[4:]]
            out.append((f[0], int(f[1]), int(f[2]), order, edges))
    return out


def _adj(nv, edges):
    adj = [set() for _ in range(nv)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    return adj


@pytest.mark.parametrize("name,width,work,order,edges", _golden_costs())
def test_elimination_cost_hand_derived(name, width, work, order, edges):
    adj = _adj(len(order), edges)
    assert Q.elimination_cost(adj, order) == (width, work), name


def _bucket_recount(nv, edges, order, rng):
    """Eliminates `order` by contracting explicit random tensors bucket by
    bucket (one 2x2 factor per edge, one 2-vector per vertex) and counts the
    index space of every bucket product; returns (width, work, value)."""
    factors = [((a, b), rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))) for a, b in edges]
    factors += [((v,), rng.normal(size=2) + 1j * rng.normal(size=2)) for v in range(nv)]
    letters = "abcdefghijklmnopqrstuvwxyz"
    width, work = 0, 0
    for v in order:
        bucket = [f for f in factors if v in f[0]]
        factors = [f for f in factors if v not in f[0]]
        union = sorted(set().union(*[set(f[0]) for f in bucket]))
        spec = ",".join("".join(letters[u] for u in vs) for vs, _ in bucket)
        prod = np.einsum(spec + "->" + "".join(letters[u] for u in union), *[a for _, a in bucket])
        assert prod.size == 1 << len(union)
        work += prod.size
        width = max(width, len(union) - 1)
        out_vars = tuple(u for u in union if u != v)
        factors.append((out_vars, prod.sum(axis=union.index(v))))
    value = complex(np.prod([complex(a) for vs, a in factors]))
    return width, work, value, factors


@pytest.mark.parametrize("seed", range(6))
def test_elimination_cost_recount_by_bucket_contraction(seed):
    """The (width, work) that elimination_cost derives from the graph equals a
    recount from an explicit bucket-by-bucket contraction of random tensors on
    the same graph and order; the contraction itself equals the brute-force sum
    over all assignments, so the recount is of a correct elimination."""
    rng = np.random.default_rng(100 + seed)
    nv = 8 if seed % 2 else 10
    edges = random_regular_graph(nv, rng)
    order = [int(v) for v in rng.permutation(nv)]
    adj = _adj(nv, edges)
    rec_rng = np.random.default_rng(seed)
    width, work, value, _ = _bucket_recount(nv, edges, order, rec_rng)
    assert Q.elimination_cost(adj, order) == (width, work)
    # brute force with the same tensors
    rec_rng = np.random.default_rng(seed)
    fs = [((a, b), rec_rng.normal(size=(2, 2)) + 1j * rec_rng.normal(size=(2, 2))) for a, b in edges]
    fs += [((v,), rec_rng.normal(size=2) + 1j * rec_rng.normal(size=2)) for v in range(nv)]
    total = 0j
    for bits in itertools.product((0, 1), repeat=nv):
        term = 1 + 0j
        for vs, arr in fs:
            term *= arr[tuple(bits[u] for u in vs)]
        total += term
    assert abs(value - total) <= 1e-10 * max(1.0, abs(total))


def test_tree_decomposition_checker_rejects_each_violation():
    """check_tree_decomposition accepts a valid decomposition of the 4-cycle
    and rejects one violation of each condition of Sec. II B."""
    adj = _adj(4, [(0, 1), (1, 2), (2, 3), (3, 0)])
    bags, parent = Q.bags_from_order(adj, [0, 1, 2, 3])
    assert Q.check_tree_decomposition(adj, bags, parent) == 2
    path = {0: None, 1: 0, 2: 1}           # bag tree 0 - 1 - 2
    # (1) vertex 3 is in no bag
    with pytest.raises(AssertionError, match=r"condition \(1\)"):
        Q.check_tree_decomposition(adj, {0: frozenset({0, 1}), 1: frozenset({1, 2}),
                                         2: frozenset({2, 0})}, path)
    # (2) every vertex is covered but edge 3-0 lies in no bag
    with pytest.raises(AssertionError, match=r"condition \(2\)"):
        Q.check_tree_decomposition(adj, {0: frozenset({0, 1}), 1: frozenset({1, 2}),
                                         2: frozenset({2, 3})}, path)
    # (3) vertex 3 sits in bags 0 and 2 but not in bag 1 between them
    with pytest.raises(AssertionError, match=r"condition \(3\)"):
        Q.check_tree_decomposition(adj, {0: frozenset({0, 1, 3}), 1: frozenset({1, 2}),
                                         2: frozenset({2, 3})}, path)
    # the same bags with vertex 3 added to the middle bag are valid again
    assert Q.check_tree_decomposition(adj, {0: frozenset({0, 1, 3}), 1: frozenset({1, 2, 3}),
                                            2: frozenset({2, 3})}, path) == 2
