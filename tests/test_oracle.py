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
