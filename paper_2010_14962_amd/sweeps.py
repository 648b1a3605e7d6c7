"""Planner sweeps in the shape of the paper's experiments (Sec. IV A).

The paper's figures (time against qubits on 1 to 4096 cores, Fig. 4(a); time
and tree width against the number of cuts for a 50-qubit sample, Fig. 4(b);
the 120-qubit run of Fig. 5) survive only as captions, and its samples are not
available.  These sweeps reproduce their shape on seeded synthetic 3-regular
QAOA instances: every width and cost is the planner's exact min-fill
evaluation (qtn_cost_exact / qtn_cut_search through libqtn); with a GPU the
width-against-cuts sweep also times the contraction of all 2^k slices.

Widths here are ranks of binary slice tensors of the merged ket network; the
paper's tree widths are of its density-matrix line graph, whose units differ
(one density-matrix cut fixes two binary variables), so only trends compare.

Usage: python -m paper_2010_14962_amd.sweeps [--gpu] [--seeds 50] [--out file.json]
"""
from __future__ import annotations

import argparse
import json
import math
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import qtn


def _instance(n: int, p: int, seed: int):
    from instances import make_instance
    return make_instance(n, p, 1, seed)


def width_vs_cuts(n: int, p: int, seeds: Sequence[int], ks: Sequence[int], pop: int = 11,
                  iters: int = 4) -> List[dict]:
    """Exact (width, log2 cost) of Algorithm 1's cut set for each k (the
    Fig. 4(b) and Fig. 5 sweeps), per seed."""
    rows = []
    for seed in seeds:
        inst = _instance(n, p, seed)
        for k in ks:
            t = time.perf_counter()
            cut, st = qtn.cut_search(n, inst.edges, p, k, pop, iters, seed)
            rows.append({"n": n, "p": p, "seed": seed, "k": k, "width": st["width"],
                         "log2_cost": st["log2_cost"], "search_s": time.perf_counter() - t,
                         "cut": cut})
    return rows


def qubit_sweep(ns: Sequence[int], p: int, seeds: Sequence[int]) -> List[dict]:
    """Uncut min-fill width and log2 work against the qubit count, over many
    seeded graphs per size (the Fig. 4(a) sweep; 50 samples per size in the
    paper)."""
    rows = []
    for n in ns:
        ws, cs = [], []
        for seed in seeds:
            inst = _instance(n, p, seed)
            w, c = qtn.cost_exact(n, inst.edges, p, np.zeros((1, 0), dtype=np.uint32))
            ws.append(int(w[0]))
            cs.append(float(c[0]))
        rows.append({"n": n, "p": p, "samples": len(seeds), "width_mean": float(np.mean(ws)),
                     "width_min": int(min(ws)), "width_max": int(max(ws)),
                     "log2_cost_mean": float(np.mean(cs))})
    return rows


def ga_ablation(n: int, p: int, k: int, seeds: Sequence[int], pops=(5, 11, 21), iters=(0, 4, 10)):
    """Mean exact width and log2 cost of Algorithm 1's result against its
    population N and iterations T (the paper uses N = 11, T = 4)."""
    rows = []
    for N in pops:
        for T in iters:
            ws, cs, ev = [], [], []
            for seed in seeds:
                inst = _instance(n, p, seed)
                _, st = qtn.cut_search(n, inst.edges, p, k, N, T, seed)
                ws.append(st["width"])
                cs.append(st["log2_cost"])
                ev.append(st["exact_evals"])
            rows.append({"N": N, "T": T, "k": k, "width_mean": float(np.mean(ws)),
                         "log2_cost_mean": float(np.mean(cs)), "exact_evals_mean": float(np.mean(ev))})
    return rows


def cuts_to_reach(n: int, p: int, seeds: Sequence[int], cap: int, k_max: int = 12) -> List[dict]:
    """For each sample: its uncut width and the smallest k whose searched cut
    set brings the width to `cap` or below (the paper's 80-qubit check: some
    samples exceed what one core holds, a few cuts bring them under it)."""
    rows = []
    for seed in seeds:
        inst = _instance(n, p, seed)
        w0, _ = qtn.cost_exact(n, inst.edges, p, np.zeros((1, 0), dtype=np.uint32))
        need = None
        for k in range(0, k_max + 1):
            _, st = qtn.cut_search(n, inst.edges, p, k, 11, 4, seed)
            if st["width"] <= cap:
                need = k
                break
        rows.append({"n": n, "seed": seed, "width_uncut": int(w0[0]), "cap": cap, "k_needed": need})
    return rows


def time_vs_cuts(n: int, p: int, seed: int, ks: Sequence[int], precision: str = "fp64",
                 reps: int = 3) -> List[dict]:
    """GPU time per amplitude (all 2^k slices in one call) against k."""
    import torch
    from . import plan_instance
    inst = _instance(n, p, seed)
    stream = torch.cuda.current_stream().cuda_stream
    rows = []
    ref = None
    for k in ks:
        plan = plan_instance(inst, k=k, seed=seed, precision=precision)
        plan.bind_torch(min(1 << k, 4096))
        amp = plan.contract(0, 1 << k, stream)[0].value()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            plan.contract(0, 1 << k, stream)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t) / reps
        ref = amp if ref is None else ref
        info = plan.info()
        rows.append({"n": n, "p": p, "k": k, "width": info["width"], "ms_per_amplitude": 1e3 * el,
                     "slices_per_sec": (1 << k) / el, "rel_diff_vs_k0": abs(amp - ref) / abs(ref)})
        plan.close()
    return rows


def main(argv: Optional[Sequence[str]] = None) -> Dict[str, list]:
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, default=50)
    ap.add_argument("--gpu", action="store_true")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    seeds = list(range(a.seeds))
    res = {
        "width_vs_cuts_n50": width_vs_cuts(50, 1, seeds[:5], range(0, 13)),
        "width_vs_cuts_n120": width_vs_cuts(120, 1, seeds[:3], range(0, 17)),
        "qubit_sweep_p1": qubit_sweep(range(20, 141, 20), 1, seeds),
        "ga_ablation_n80": ga_ablation(80, 1, 4, seeds[:10]),
        "cuts_to_reach_n80": cuts_to_reach(80, 1, seeds, cap=12),
    }
    if a.gpu:
        res["time_vs_cuts_n50"] = time_vs_cuts(50, 1, 0, range(0, 11))
    text = json.dumps(res, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    else:
        print(text)
    return res


if __name__ == "__main__":
    main()
