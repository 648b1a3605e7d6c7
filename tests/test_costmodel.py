"""CPU tests of the learned cost model's host side: exact labels against the
oracle's min-fill cost, features against their definition re-derived from the
oracle's elimination, and the unguided search against Algorithm 1."""
import itertools
import math

import numpy as np
import pytest

from instances import make_instance
from oracle import qaoa as Q
from oracle.search import ga_cut_search
from paper_2010_14962_amd import qtn
from paper_2010_14962_amd.qtn import QtnError


def _random_sets(V, k, count, seed):
    rng = np.random.default_rng(seed)
    return np.stack([np.sort(rng.choice(V, size=k, replace=False)) for _ in range(count)])


@pytest.mark.parametrize("n,p,k,seed", [(16, 1, 3, 0), (20, 2, 5, 1), (30, 1, 6, 2), (24, 2, 0, 3)])
def test_exact_labels_match_oracle(n, p, k, seed):
    inst = make_instance(n, p, 1, seed)
    adj = Q.interaction_graph(n, inst.edges, p)
    sets = _random_sets(n * p, k, 12, seed)
    w, c = qtn.cost_exact(n, inst.edges, p, sets, threads=3)
    for i, cut in enumerate(sets):
        order, _ = Q.min_fill_order(adj, removed=cut)
        width, work = Q.elimination_cost(adj, order, removed=cut)
        assert w[i] == width
        assert c[i] == math.log2(work) + k


def test_exact_labels_independent_of_thread_count():
    inst = make_instance(40, 2, 1, 7)
    sets = _random_sets(80, 8, 40, 7)
    a = qtn.cost_exact(40, inst.edges, 2, sets, threads=1)
    b = qtn.cost_exact(40, inst.edges, 2, sets, threads=8)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def _features_by_definition(n, p, edges, cut):
    """The 32 features re-derived from the oracle's uncut min-fill elimination."""
    adj = Q.interaction_graph(n, edges, p)
    V = n * p
    order, nplus = Q.min_fill_order(adj)
    width, work = Q.elimination_cost(adj, order)
    g = {v: set(a) for v, a in enumerate(adj)}
    stats = {name: np.zeros(V) for name in ("deg", "pos", "bag", "fill", "nbags", "layer")}
    stats["nbags"][:] = 1
    in_max = np.zeros(V, dtype=bool)
    marked = False
    for i, (v, nb) in enumerate(zip(order, nplus)):
        stats["pos"][v] = i / V
        stats["bag"][v] = len(nb)
        stats["fill"][v] = sum(1 for a, b in itertools.combinations(sorted(nb), 2) if b not in g[a])
        for a, b in itertools.combinations(nb, 2):
            g[a].add(b)
            g[b].add(a)
        for u in nb:
            stats["nbags"][u] += 1
            g[u].discard(v)
        if not marked and len(nb) == width:
            marked = True
            in_max[v] = True
            for u in nb:
                in_max[u] = True
    for v in range(V):
        stats["deg"][v] = len(adj[v])
        stats["layer"][v] = (v // n) / p
    k = len(cut)
    f = []
    for name in ("deg", "pos", "bag", "fill", "nbags", "layer"):
        x = stats[name][list(cut)]
        f += [x.mean(), x.max(), x.min(), x.sum()] if k else [0, 0, 0, 0]
    inner = sum(1 for a, b in itertools.combinations(cut, 2) if b in adj[a])
    f += [n, p, k, width, math.log2(work)]
    f += [inner / k, in_max[list(cut)].sum() / k, (stats["bag"][list(cut)] >= width - 2).sum() / k] \
        if k else [0, 0, 0]
    return np.array(f, dtype=np.float64)


@pytest.mark.parametrize("n,p,k,seed", [(16, 1, 3, 0), (20, 2, 6, 4), (36, 1, 5, 5)])
def test_features_match_definition(n, p, k, seed):
    inst = make_instance(n, p, 1, seed)
    sets = _random_sets(n * p, k, 6, seed + 100)
    F = qtn.cost_features(n, inst.edges, p, sets)
    assert F.shape == (6, qtn.COST_FEATURES)
    for i, cut in enumerate(sets):
        ref = _features_by_definition(n, p, inst.edges, [int(c) for c in cut])
        np.testing.assert_allclose(F[i], ref.astype(np.float32), rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("n,p,k,seed", [(20, 1, 3, 0), (16, 2, 4, 3)])
def test_unguided_search_is_algorithm_1(n, p, k, seed):
    inst = make_instance(n, p, 1, seed)
    adj = Q.interaction_graph(n, inst.edges, p)
    ref_cut, (w, work) = ga_cut_search(adj, k, N=11, T=4, seed=seed)
    cut, st = qtn.cut_search(n, inst.edges, p, k, pop=11, iters=4, seed=seed)
    assert cut == ref_cut
    assert st["width"] == w and st["log2_cost"] == math.log2(work) + k
    assert st["model_evals"] == 0 and st["exact_evals"] >= 11


def test_cost_model_errors():
    inst = make_instance(16, 1, 1, 0)
    with pytest.raises(QtnError):
        qtn.cost_exact(16, inst.edges, 1, np.array([[0, 16]]))
    with pytest.raises(QtnError):
        qtn.cost_features(16, inst.edges, 1, np.array([[0, 99]]))
    with pytest.raises(QtnError):
        qtn.cut_search(16, inst.edges, 1, 16)
