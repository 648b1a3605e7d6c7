"""The autotuner of the launch configuration (qtn_plan_autotune): it times
the alternatives of every streaming step, keeps the fastest where a whole
contraction gains, reuses a cache of earlier choices, and leaves the
amplitudes unchanged (the block partition of
a step changes, the arithmetic of its outputs does not)."""
import pytest

from instances import workload_instance
from paper_2010_14962_amd import plan_instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autotune_keeps_results_and_caches(precision, tmp_path):
    print("case autotune", precision, flush=True)
    stream = torch.cuda.current_stream().cuda_stream
    inst = workload_instance("qaoa_n120_p1_b8", seed=0)
    plan = plan_instance(inst, k=0, precision=precision)
    plan.bind_torch(1)
    before = [p.value() for p in plan.contract(0, 1, stream)]
    cache = str(tmp_path / "tune.txt")
    st = plan.autotune(cache, stream)
    print("autotune", st, flush=True)
    assert st["steps"] > 0 and st["measured"] >= st["steps"] and st["cached"] == 0
    assert st["tuned_us"] <= st["default_us"]
    # choices stay only where a whole contraction gets faster with them
    assert st["kept"] <= st["steps"]
    if st["kept"]:
        assert st["whole_tuned_us"] < st["whole_default_us"]
    else:
        assert st["whole_tuned_us"] == st["whole_default_us"]
    tunes = [plan.step_tune(i) for i in range(plan.info()["n_steps"])]
    changed = [t for t in tunes if t["blocks"] != 1024 or t["direct"] or t["pair"]]
    assert len(changed) == st["kept"]
    assert all(t["blocks"] in (256, 512, 1024, 2048, 4096) for t in tunes)
    after = [p.value() for p in plan.contract(0, 1, stream)]
    for a, b in zip(after, before):
        assert abs(a - b) <= 1e-12 * abs(b)
    again = [p.value() for p in plan.contract(0, 1, stream)]
    assert again == after
    # the launch mode it chose was measured both ways; both give the same bits
    assert st["graphs"] in (0, 1) and st["graph_us"] > 0 and st["direct_us"] > 0
    assert (st["graph_us"] <= st["direct_us"]) == bool(st["graphs"])
    for graphs in (True, False):
        plan.set_graphs(graphs)
        assert [p.value() for p in plan.contract(0, 1, stream)] == after
    # a second plan of the same workload takes every choice from the cache
    other = plan_instance(inst, k=0, precision=precision)
    other.bind_torch(1)
    st2 = other.autotune(cache, stream)
    assert st2["measured"] == 0 and st2["cached"] == st["steps"]
    # (whether the cached choices stay is decided by timing again)
    for a, b in zip([p.value() for p in other.contract(0, 1, stream)], after):
        assert abs(a - b) <= 1e-12 * abs(b)
