"""Planner sweeps in the shape of the paper's experiments (Sec. IV A, Fig. 4,
Fig. 5), on small sizes: the tables are complete and consistent with the exact
evaluator, and cutting lowers the width (Sec. III A)."""
import numpy as np

from instances import make_instance
from paper_2010_14962_amd import qtn
from paper_2010_14962_amd import sweeps as W


def test_width_vs_cuts_is_exact_and_falls():
    rows = W.width_vs_cuts(50, 1, [0, 1], range(0, 7))
    assert len(rows) == 14
    for r in rows:
        inst = make_instance(50, 1, 1, r["seed"])
        w, c = qtn.cost_exact(50, inst.edges, 1, np.array([r["cut"]], dtype=np.uint32).reshape(1, -1))
        assert int(w[0]) == r["width"] and abs(float(c[0]) - r["log2_cost"]) < 1e-9
    for seed in (0, 1):
        ws = [r["width"] for r in rows if r["seed"] == seed]
        assert ws[-1] < ws[0]       # six cut variables lower the width


def test_qubit_sweep_and_cuts_to_reach():
    q = W.qubit_sweep([20, 40, 60], 1, range(5))
    assert [r["n"] for r in q] == [20, 40, 60] and all(r["samples"] == 5 for r in q)
    assert q[0]["width_mean"] <= q[-1]["width_mean"]
    c = W.cuts_to_reach(40, 1, range(4), cap=5, k_max=8)
    for r in c:
        if r["width_uncut"] <= 5:
            assert r["k_needed"] == 0
        elif r["k_needed"] is not None:
            assert r["k_needed"] >= 1


def test_ga_ablation_table():
    rows = W.ga_ablation(40, 1, 3, range(2), pops=(5, 11), iters=(0, 2))
    assert len(rows) == 4
    more = [r for r in rows if r["N"] == 11 and r["T"] == 2][0]
    less = [r for r in rows if r["N"] == 5 and r["T"] == 0][0]
    assert more["exact_evals_mean"] > less["exact_evals_mean"]
