"""Throughput benchmark of the sliced QAOA amplitude contraction on one GPU.

Workload (default): random 3-regular graph, n = 120 qubits, QAOA depth 1,
8 output bitstrings batched, cut size k = the smallest k whose searched cut
keeps every slice tensor at rank <= 26; seeded synthetic instance.  One step
is one contraction over all 2^k slices of all 8 bitstrings (the whole hot
path: slice set-up, every contraction step, the FP64 slice sum, the partials
in host memory), one synchronous qtn_contract per step, in the launch mode
(graph replay or direct launches) and per-step launch configurations that
qtn_plan_autotune chose before the timed region.  The same steps enqueued
back to back with qtn_contract_async are timed as well.  The mixed form (64-bit shared-exponent storage of the large tensors
with per-instance power-of-two rescaling, FP64 arithmetic) is the headline;
the plain FP64 GPU contraction is timed beside it.

Two sliced workloads follow in the same line ("sliced"): n = 80, p = 2 with
k = 16 (65,536 slices) and the same 120-qubit instance with k = 16 (8 x
65,536 slice contractions), each in both forms, with the error of the
[0, 1024) subset sums against the oracle and the oracle's slice rate.

Prints one JSON line.  Single GPU only.
"""
import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "slices/sec + amplitudes/sec, n=120 p=1 3-reg QAOA, mixed-prec vs FP64 GPU"
HBM_PEAK_GBS = 8000.0
# FP64 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
FP64_VECTOR_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
CSRC = os.path.join(ROOT, "paper_2010_14962_amd", "csrc")


def kernel_sources_sha256() -> str:
    """Hash of the sources that define the kernels and the schedule."""
    import hashlib
    h = hashlib.sha256()
    for name in ("runtime.hip", "planner.cpp", "planner.h"):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_file_tag(kernel: str) -> str:
    """File-name form of a kernel instance name, e.g. step_tiled_true_4_3_3."""
    import re
    return re.sub("_+", "_", "".join(c if c.isalnum() else "_" for c in kernel)).strip("_")


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE runs, copy-calibrated), or None when the
    kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.md" % (kernel_file_tag(kernel), workload))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != kernel_sources_sha256():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _oracle_worker(args):
    """One amplitude on one host core (the paper's one-subgraph-per-core scheme)."""
    n, edges, p, gamma, beta, x, cut, order, slices = args
    from oracle import qaoa as Q
    t = time.perf_counter()
    if cut:
        val = sum(Q.slice_partial(n, edges, p, gamma, beta, x, cut, s, order=order) for s in slices)
    else:
        val = Q.ve_amplitude(n, edges, p, gamma, beta, x, order=order)
    return val, time.perf_counter() - t


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_workers(max_rank: int) -> int:
    """Worker processes for the oracle: the host cores (at most 16, the CPU
    share of one GPU), and no more than 70% of the RAM holds at three
    complex128 tensors of the largest rank per worker."""
    cores = max(1, min(16, os.cpu_count() or 1))
    try:
        ram = os.sysconf("SC_PAGE_SIZE") * os.sysconf("SC_PHYS_PAGES")
        cores = max(1, min(cores, int(0.7 * ram // (3 * 16 * (1 << max(0, max_rank))))))
    except (ValueError, OSError):
        pass
    return cores


def cpu_baseline(inst, cut, order, max_rank, budget_s=20.0):
    """Times the oracle on a bounded sample of the same workload."""
    cores = oracle_workers(max_rank)
    k = len(cut)
    # one probe to size the sample
    slices_per_job = 1 if k else 0
    probe = _oracle_worker((inst.n, inst.edges, inst.p, inst.gamma, inst.beta, inst.bitstrings[0],
                            cut, order, range(slices_per_job) if k else None))
    per_job = max(probe[1], 1e-3)
    jobs = max(cores, int(budget_s / per_job))
    jobs = min(jobs, 4 * cores * 8)
    B = inst.bitstrings.shape[0]
    work = []
    for j in range(jobs):
        b = j % B
        sl = [j // B % (1 << k)] if k else None
        work.append((inst.n, inst.edges, inst.p, inst.gamma, inst.beta, inst.bitstrings[b],
                     cut, order, sl))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_worker, work)
    wall = time.perf_counter() - t0
    vals = [r[0] for r in res]
    if k:
        value = jobs / wall                     # slice-contractions per second
        unit = "slices/s"
        amps = value / (1 << k)
    else:
        value = jobs / wall
        unit = "amplitudes/s"
        amps = value
    return {"value": value, "unit": unit, "amplitudes_per_sec": amps, "cores": cores,
            "cpu_model": host_cpu_model(), "kind": "oracle", "sample": "%d %s of the workload (bitstrings cycled), complex128 "
            "variable elimination with the plan's order and cut, %d worker processes" %
            (jobs, "slices" if k else "uncut amplitudes", cores),
            "cpu_seconds": sum(r[1] for r in res), "wall_seconds": wall}, vals


def _subset_worker(args):
    """Oracle slice values of one bitstring over a range, on one host core."""
    n, edges, p, gamma, beta, x, cut, order, slices = args
    from oracle import qaoa as Q
    t = time.perf_counter()
    vals = [Q.slice_partial(n, edges, p, gamma, beta, x, cut, s, order=order) for s in slices]
    return vals, time.perf_counter() - t


# device memory a wave's workspace may take when the wave size is chosen
# automatically (one MI355X holds 288 GB)
WAVE_BUDGET_BYTES = 64 << 30


def autotune_summary(plan, stream):
    """Runs the library's autotuner (per-step launch configurations, kept
    only if a whole contraction gains, then graph replay or direct launches,
    whichever is faster) and returns what it chose."""
    st = plan.autotune(stream=stream)
    print("# autotune: kept %d (whole contraction %.1f us with the choices, %.1f us with the "
          "defaults); %s (%.1f us graph replay, %.1f us direct)" %
          (st["kept"], st["whole_tuned_us"], st["whole_default_us"],
           "graph replay" if st["graphs"] else "direct launches", st["graph_us"], st["direct_us"]),
          file=sys.stderr, flush=True)
    plan.bench_graphs = bool(st["graphs"])
    return {"kept": int(st["kept"]), "whole_tuned_us": st["whole_tuned_us"],
            "whole_default_us": st["whole_default_us"], "steps": int(st["steps"]),
            "launch_mode": "graph replay" if st["graphs"] else "direct launches",
            "graph_us": st["graph_us"], "direct_us": st["direct_us"]}


def bench_graphs(plan) -> bool:
    """Launch mode of the timed regions: the autotuner's choice, else graphs."""
    return getattr(plan, "bench_graphs", True)


def wave_size(plans, nsl, requested):
    """Slices per wave: `requested` if given, else the largest power of two
    up to all nsl slices whose workspace fits WAVE_BUDGET_BYTES in every
    plan (larger waves amortise the per-wave launches)."""
    if requested > 0:
        return min(nsl, requested)
    S = 1
    while S < nsl and max(pl.workspace_bytes(2 * S) for pl in plans) <= WAVE_BUDGET_BYTES:
        S *= 2
    return S


def sliced_row(name, seed, slices_per_wave, reps, with_cpu, autotune=True):
    """One sliced workload: every slice of every bitstring per contraction,
    mixed and FP64 with the same cut (each autotuned before its timed
    region), the error of the [0, 1024) subset sums against the oracle, and
    the oracle's slice rate on that subset."""
    import torch
    from instances import search_params, workload_instance
    from paper_2010_14962_amd import plan_instance
    inst = workload_instance(name, seed=seed)
    m = inst.meta
    t0 = time.perf_counter()
    mixed = plan_instance(inst, k=m["k"], max_rank=m["max_rank"], precision="fp32", **search_params(name))
    plan_s = time.perf_counter() - t0
    cut = mixed.cut()
    info = mixed.info()
    k, B = info["k"], inst.n_bitstrings
    nsl = 1 << k
    f64 = plan_instance(inst, cut_vars=cut, precision="fp64")
    S = wave_size((mixed, f64), nsl, slices_per_wave)
    stream = torch.cuda.current_stream().cuda_stream
    info_f = {"flops": 2.0 ** info["log2_flops"]}
    out = {"workload": name, "n": inst.n, "p": inst.p, "bitstrings": B, "k": k,
           "slices_per_amplitude": nsl, "slice_contractions_per_step": B * nsl,
           "max_slice_rank": info["width"], "slices_per_wave": S, "plan_s": plan_s,
           "log2_flops_per_slice": info["log2_flops"], "alg_bytes_per_slice": info["bytes_per_slice"]}
    sub = min(1024, nsl)
    res = {}
    for tag, plan in (("mixed", mixed), ("fp64", f64)):
        plan.bind_torch(S)
        tune = autotune_summary(plan, stream) if autotune else None
        plan.set_graphs(bench_graphs(plan))
        plan.contract(0, nsl, stream)           # capture and warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            vals = plan.contract(0, nsl, stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        res[tag] = [p.value() for p in plan.contract(0, sub, stream)]
        out[tag] = {"slices_per_sec": B * nsl * reps / el, "amplitudes_per_sec": B * reps / el,
                    "ms_per_step": 1e3 * el / reps,
                    # 1: some intermediate in the 64-bit form, rescaling kernels;
                    # 0: every tensor complex128, the FP64 kernels
                    "rescaled": int(plan.info()["rescaled"]), "autotune": tune,
                    # synchronous calls without rescaling, and calls repeated
                    # with rescaling after leaving the 64-bit range
                    "range": plan.range_state()}
        print("# %s %s: %.1f ms per contraction of %d slice instances" %
              (name, tag, 1e3 * el / reps, B * nsl), file=sys.stderr, flush=True)
        if tag == "mixed":
            # whole-contraction roofline from the plan's algorithmic work per
            # slice (flops and bytes of every step, all bitstrings) and the
            # graph-replay time
            flops = info_f["flops"] * nsl
            byts = info["bytes_per_slice"] * nsl
            tfs = flops / (el / reps) / 1e12
            gbs = byts / (el / reps) / 1e9
            f_alu, f_hbm = tfs / FP64_VECTOR_PEAK_TFLOPS, gbs / HBM_PEAK_GBS
            out["roofline"] = {
                "kernel": "whole contraction (all launches of all waves)",
                "bound": "alu" if f_alu > f_hbm else "hbm",
                "achieved": tfs if f_alu > f_hbm else gbs,
                "peak": FP64_VECTOR_PEAK_TFLOPS if f_alu > f_hbm else HBM_PEAK_GBS,
                "unit": "TFLOP/s" if f_alu > f_hbm else "GB/s",
                "frac": max(f_alu, f_hbm), "fp64_TFLOPs": tfs, "hbm_GBs": gbs,
                "alg_flops_per_step": flops, "alg_bytes_per_step": byts}
        plan.close()
    out["mixed_over_fp64"] = out["mixed"]["slices_per_sec"] / out["fp64"]["slices_per_sec"]
    if with_cpu:
        cores = oracle_workers(int(info["width"]))
        order = plan_instance(inst, cut_vars=cut).order()
        nsub = max(sub, min(nsl, 4 * cores))
        work, owner = [], []
        chunk = max(1, nsub // (4 * cores))
        for b in range(B):
            for lo in range(0, nsub, chunk):
                work.append((inst.n, inst.edges, inst.p, inst.gamma, inst.beta, inst.bitstrings[b], cut,
                             order, list(range(lo, min(nsub, lo + chunk)))))
                owner.append(b)
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(cores) as pool:
            got = pool.map(_subset_worker, work)
        wall = time.perf_counter() - t0
        from oracle.qaoa import neumaier_sum
        per_b = [[] for _ in range(B)]
        for (vals, _), b in zip(got, owner):
            per_b[b].extend(vals)
        errs = {"mixed": [], "fp64": []}
        kappa = []
        for b in range(B):
            sl = per_b[b][:sub]
            re, rc = neumaier_sum(v.real for v in sl)
            im, ic = neumaier_sum(v.imag for v in sl)
            ref = complex(re + rc, im + ic)
            kappa.append(sum(abs(v) for v in sl) / abs(ref))
            for tag in errs:
                errs[tag].append(abs(res[tag][b] - ref) / abs(ref))
        out["subset"] = {"slices": sub, "max_rel_err_mixed_vs_oracle": max(errs["mixed"]),
                         "max_rel_err_fp64_vs_oracle": max(errs["fp64"]), "max_kappa": max(kappa)}
        out["cpu_baseline"] = {"value": B * nsub / wall, "unit": "slices/s", "cores": cores,
                               "cpu_model": host_cpu_model(), "kind": "oracle",
                               "sample": "slices [0, %d) of all %d bitstrings, complex128 variable "
                                         "elimination with the plan's cut and order, %d worker "
                                         "processes" % (nsub, B, cores),
                               "cpu_seconds": sum(g[1] for g in got), "wall_seconds": wall}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="qaoa_n120_p1_b8")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--slices-per-wave", type=int, default=0,
                    help="slices per wave; 0 picks the largest power of two whose workspace "
                         "fits %d GiB" % (WAVE_BUDGET_BYTES >> 30))
    ap.add_argument("--no-sliced", action="store_true",
                    help="skip the sliced workloads (n=80 p=2 k=16, n=120 p=1 k=16)")
    ap.add_argument("--sliced-reps", type=int, default=3)
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (graph replay, default launch configurations)")
    ap.add_argument("--sliced-child", default=None,
                    help="internal: run one sliced workload and print its JSON object")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the sliced contraction shards by slice range "
              "across GPUs, which this build does not launch (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from instances import workload_instance
    from paper_2010_14962_amd import plan_instance, qtn_plan

    torch.cuda.set_device(0)
    if args.sliced_child:
        print(json.dumps(sliced_row(args.sliced_child, args.seed, args.slices_per_wave,
                                    args.sliced_reps, not args.no_cpu_baseline,
                                    not args.no_autotune)), flush=True)
        return
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("# copy calibration: %d bytes read, %d bytes written" % (n, n), file=sys.stderr, flush=True)
        del src, dst
    inst = workload_instance(args.workload, seed=args.seed)
    w = inst.meta
    t0 = time.perf_counter()
    mixed = plan_instance(inst, k=w["k"] if w["k"] is not None else -1,
                          max_rank=w["max_rank"] or 0, precision="fp32")
    plan_s = time.perf_counter() - t0
    cut = mixed.cut()
    info = mixed.info()
    k = info["k"]
    nsl = 1 << k
    B = inst.n_bitstrings
    f64 = plan_instance(inst, cut_vars=cut, precision="fp64")
    S = wave_size((mixed, f64), nsl, args.slices_per_wave)
    mixed.bind_torch(S)
    f64.bind_torch(S)
    stream = torch.cuda.current_stream().cuda_stream
    print("# workload %s k=%d width=%d steps=%d B=%d S=%d plan %.3fs" %
          (args.workload, k, info["width"], info["n_steps"], B, S, plan_s), file=sys.stderr, flush=True)
    # launch configurations and launch mode, measured before any timed region
    tune = None
    if not args.no_autotune:
        tune = {"mixed": autotune_summary(mixed, stream), "fp64": autotune_summary(f64, stream)}

    def run_pipelined(plan, steps, warmup):
        """Timed region: `steps` asynchronous contractions enqueued back to
        back on the stream, each copying its partials to its own slot of a
        pinned host buffer, then one synchronisation."""
        plan.set_graphs(bench_graphs(plan))
        buf = torch.zeros((steps + warmup, B, 4), dtype=torch.float64).pin_memory()
        for i in range(warmup):
            plan.contract_async(0, nsl, buf[i].data_ptr(), stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(steps):
            plan.contract_async(0, nsl, buf[warmup + i].data_ptr(), stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        last = buf[warmup + steps - 1].numpy()
        assert all(np.array_equal(buf[warmup + i].numpy(), last) for i in range(steps))
        return el, [complex(r[0] + r[2], r[1] + r[3]) for r in last]

    def run(plan, steps, warmup, timing):
        """Timed region: `steps` contractions bracketed by device syncs.  With
        `timing`, kernels are launched directly (no graph replay) and each
        streaming-step launch is bracketed by HIP events on its stream."""
        plan.set_graphs(bench_graphs(plan) and not timing)
        for _ in range(warmup):
            plan.contract(0, nsl, stream)
        if timing:
            plan.set_timing(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = None
        for _ in range(steps):
            out = plan.contract(0, nsl, stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        tm = plan.timing() if timing else None
        if timing:
            tm["steps"] = {st: plan.step_timing(st) for st in range(plan.info()["n_steps"])}
            plan.set_timing(False)
        plan.set_graphs(bench_graphs(plan))
        return el, [p.value() for p in out], tm

    # value: one synchronous qtn_contract per step (in the autotuned launch
    # mode), nothing else in the timed region
    el, amps, _ = run(mixed, args.steps, args.warmup, False)
    print("# mixed, synchronous calls: %.3f ms/step" % (1e3 * el / args.steps), file=sys.stderr, flush=True)
    # the same steps enqueued back to back with qtn_contract_async
    el_pipe, _ = run_pipelined(mixed, args.steps, args.warmup)
    print("# mixed, pipelined: %.3f ms/step" % (1e3 * el_pipe / args.steps), file=sys.stderr, flush=True)
    # roofline: same contraction, direct launches with per-launch events
    el_t, _, tm = run(mixed, args.steps, 1, True)
    print("# mixed, direct launches with events: %.3f ms/step; %s" %
          (1e3 * el_t / args.steps, {k: v for k, v in tm.items() if k != "steps"}),
          file=sys.stderr, flush=True)
    n64 = args.fp64_steps or max(3, args.steps // 2)
    el64, amps64, _ = run(f64, n64, 2, False)
    print("# fp64: %.3f ms/step" % (1e3 * el64 / n64), file=sys.stderr, flush=True)

    ms = 1e3 * el / args.steps
    amps_per_s = B * args.steps / el
    slices_per_s = B * nsl * args.steps / el
    err_vs_fp64 = max(abs(a - b) / max(abs(b), 1e-300) for a, b in zip(amps, amps64))

    roof = None
    if tm and tm["launches"]:
        # dominant kernel: the grid-wide step with the largest timed share
        per = [(t, st) for st, t in tm["steps"].items() if t["launches"]]
        t, st = max(per, key=lambda x: x[0]["total_ms"])
        kern = mixed.step_kernel(st)
        avg_ms = t["total_ms"] / t["launches"]
        bytes_per_launch = t["alg_bytes"] / t["launches"]
        flops_per_launch = t["alg_flops"] / t["launches"]
        gbs = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        tfs = flops_per_launch / (avg_ms * 1e-3) / 1e12
        f_hbm, f_alu = gbs / HBM_PEAK_GBS, tfs / FP64_VECTOR_PEAK_TFLOPS
        if f_alu > f_hbm:
            bound, achieved, peak, unit = "alu", tfs, FP64_VECTOR_PEAK_TFLOPS, "TFLOP/s"
        else:
            bound, achieved, peak, unit = "hbm", gbs, HBM_PEAK_GBS, "GB/s"
        traffic = measured_traffic(args.workload, kern)
        roof = {"kernel": "%s (schedule step %d, all %d instances in one launch)" % (kern, st, B),
                "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": traffic,
                "launches": t["launches"], "avg_launch_us": 1e3 * avg_ms,
                "alg_bytes_per_launch": bytes_per_launch, "alg_flops_per_launch": flops_per_launch,
                "hbm_GBs": gbs, "hbm_frac": f_hbm, "fp64_TFLOPs": tfs, "fp64_frac": f_alu,
                "traffic_over_alg_bytes": (traffic / bytes_per_launch) if traffic else None,
                "time_share": t["total_ms"] / (1e3 * el_t),
                "streaming_family": {"launches": tm["launches"],
                                     "avg_launch_us": 1e3 * tm["total_ms"] / tm["launches"],
                                     "GBs": tm["alg_bytes"] / (tm["total_ms"] * 1e-3) / 1e9,
                                     "time_share": tm["total_ms"] / (1e3 * el_t)}}

    line = {
        "metric": METRIC, "value": amps_per_s, "unit": "amplitudes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": inst.n, "p": inst.p, "bitstrings": B,
                   "k": k, "slices_per_amplitude": nsl, "max_slice_rank": info["width"],
                   "seed": args.seed, "slices_per_wave": S, "graph": "random 3-regular",
                   "rescaled": int(info["rescaled"]),
                   "precision": "mixed: large tensors stored in 8 bytes (shared 8-bit exponent, "
                                "two 28-bit mantissas); synchronous calls without rescaling while "
                                "every value stays in the form's exponent range (else repeated with "
                                "per-instance power-of-two rescaling), asynchronous calls rescaled; "
                                "fp64 arithmetic, fp64 compensated slice sum"},
        "slices_per_sec": slices_per_s,
        "range": mixed.range_state(),
        "timing": "one synchronous qtn_contract per step (%s, partials in host memory)" %
                  ("graph replay" if bench_graphs(mixed) else "direct launches"),
        "autotune": tune,
        "pipelined_ms_per_step": 1e3 * el_pipe / args.steps,
        "fp64": {"amplitudes_per_sec": B * n64 / el64, "slices_per_sec": B * nsl * n64 / el64,
                 "ms_per_step": 1e3 * el64 / n64},
        "mixed_over_fp64": (amps_per_s / (B * n64 / el64)),
        "max_rel_err_mixed_vs_fp64": err_vs_fp64,
        "plan": {"search_s": info["search_seconds"], "plan_s": plan_s,
                 "log2_flops_per_slice": info["log2_flops"],
                 "alg_bytes_per_slice": info["bytes_per_slice"]},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        order = mixed.order()
        cb, vals = cpu_baseline(inst, cut, order, int(info["width"]))
        line["cpu_baseline"] = cb
        if k == 0:
            errs = []
            for j, v in enumerate(vals[:B]):
                errs.append(abs(amps[j % B] - v) / abs(v))
            line["max_rel_err_mixed_vs_oracle"] = max(errs)
            line["max_rel_err_fp64_vs_oracle"] = max(abs(amps64[j % B] - v) / abs(v)
                                                     for j, v in enumerate(vals[:B]))
    if not args.no_sliced:
        # each sliced workload in a child process: whatever happens there, the
        # headline line above is printed
        import subprocess
        line["sliced"] = []
        for nm in ("qaoa_n80_p2_k16", "qaoa_n120_p1_b8_k16"):
            cmd = [sys.executable, os.path.abspath(__file__), "--sliced-child", nm, "--seed", str(args.seed),
                   "--slices-per-wave", str(args.slices_per_wave), "--sliced-reps", str(args.sliced_reps)]
            if args.no_cpu_baseline:
                cmd.append("--no-cpu-baseline")
            if args.no_autotune:
                cmd.append("--no-autotune")
            try:
                r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
                sys.stderr.write(r.stderr)
                rows = [l for l in r.stdout.splitlines() if l.startswith("{")]
                if r.returncode == 0 and rows:
                    line["sliced"].append(json.loads(rows[-1]))
                else:
                    line["sliced"].append({"workload": nm, "error": "exit status %d" % r.returncode})
            except subprocess.TimeoutExpired:
                line["sliced"].append({"workload": nm, "error": "time limit"})
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
