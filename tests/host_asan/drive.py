"""Drives libqtn's host code (planner, layout, launch logic, autotuner,
ranges and checkpoints, the no-allocation and batched entry points, general
circuits, the density-matrix form) through the C ABI with the HIP runtime
replaced by CPU stand-ins, under AddressSanitizer (run by
tests/test_host_asan.py).  Device results are not produced here."""
import ctypes
import os
import sys
import tempfile
import types

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.modules["torch"] = types.ModuleType("torch")   # the stand-ins need no torch runtime
from paper_2010_14962_amd import qtn  # noqa: E402

qtn.LIB_PATH = sys.argv[1]
from instances import make_instance, search_params, workload_instance  # noqa: E402
from instances.circuits import random_circuit  # noqa: E402

libc = ctypes.CDLL(None)
libc.aligned_alloc.restype = ctypes.c_void_p
libc.aligned_alloc.argtypes = [ctypes.c_size_t, ctypes.c_size_t]
keep = []


def bind(plan, S):
    nb = plan.workspace_bytes(S)
    p = libc.aligned_alloc(256, (nb + 255) // 256 * 256)
    keep.append(p)
    plan.bind_workspace(p, nb, S)


def exercise(plan, S, tune=False, tmp=None):
    info = plan.info()
    nsl = 1 << info["k"]
    S = min(S, nsl)
    bind(plan, S)
    steps, _ = plan.export()
    for st in range(info["n_steps"]):
        plan.kappa(st)
        for i in range(int(steps[st, 1])):
            plan.index_table(st, i)
    for graphs in (True, False):
        plan.set_graphs(graphs)
        plan.contract(0, min(nsl, 2 * S))
    if tune:
        plan.autotune(os.path.join(tmp, "tune.txt"))
        for st in range(info["n_steps"]):
            plan.step_tune(st)
            plan.set_step_tune(st, blocks=512, pair=True)
        plan.contract(0, S)
    plan.range_state()
    # the repeat of a contraction counted as out of the 64-bit range
    os.environ["QTN_RANGE_TEST"] = "1"
    try:
        plan.contract(0, S)
        plan.contract(0, S)
    finally:
        del os.environ["QTN_RANGE_TEST"]
    plan.range_state()
    plan.set_timing(True)
    plan.contract(0, S)
    plan.timing()
    for st in range(-1, info["n_steps"]):
        plan.step_timing(st)
        if st >= 0:
            plan.step_kernel(st)
    plan.set_timing(False)
    plan.fingerprint()


def main():
    tmp = tempfile.mkdtemp()
    for name, prec, S, tune in (("qaoa_n120_p1_b8", "fp32", 1, True), ("qaoa_n120_p1_b8", "fp64", 1, False),
                                ("qaoa_n80_p2_k16", "fp32", 256, True), ("qaoa_n120_p1_b8_k16", "fp32", 1024, False)):
        inst = workload_instance(name)
        m = inst.meta
        plan = qtn.plan_instance(inst, k=m["k"] if m["k"] is not None else -1, max_rank=m["max_rank"] or 0,
                                 precision=prec, **search_params(name))
        exercise(plan, S, tune, tmp)
        print(name, prec, "ok", flush=True)
        plan.close()
    # small plans: absorbed chains, both execution modes, ranges with a
    # checkpoint and injected faults, the no-allocation entry point
    for n, p, seed, k in ((10, 2, 0, 0), (16, 1, 0, 2), (24, 2, 1, 3)):
        inst = make_instance(n, p, 2, seed)
        for mode in ("wide", "slice"):
            plan = qtn.plan_instance(inst, k=k, seed=seed, precision="fp32", exec_mode=mode)
            exercise(plan, 4)
            nsl = 1 << plan.info()["k"]
            plan.inject_faults(0, 1)
            plan.contract_ranges(max(1, nsl // 2), max_retries=1, checkpoint=os.path.join(tmp, "ck.jsonl"))
            plan.contract_ranges(max(1, nsl // 2), checkpoint=os.path.join(tmp, "ck.jsonl"))
            os.remove(os.path.join(tmp, "ck.jsonl"))
            out = (qtn.QtnPartial * 2)()
            plan.contract_noalloc(0, nsl, min(4, nsl), ctypes.addressof(out))
            plan.close()
    # several slice-mode plans in one persistent launch
    plans = []
    for seed in (0, 1):
        plan = qtn.plan_instance(make_instance(12, 1, 2, seed), k=2, seed=seed, exec_mode="slice")
        bind(plan, 4)
        plans.append(plan)
    qtn.batch_contract(plans, [(0, 4), (1, 3)])
    for plan in plans:
        plan.close()
    # a general circuit and the density-matrix form
    c = random_circuit(8, 4, 2, 0)
    plan = qtn.qtn_plan_circuit(c.n, c.gates, c.bitstrings, k=2)
    exercise(plan, 4)
    plan.close()
    plan = qtn.plan_instance(make_instance(10, 1, 1, 0), k=2, density_matrix=True)
    exercise(plan, 4)
    plan.close()
    print("done", flush=True)


main()
