"""Learned cut-set cost model: dataset, training and evaluation drivers.

The model is not part of the paper.  It predicts, for a candidate cut set C
of a QAOA network, the two quantities the cut search of Sec. III B ranks by:
the peak tensor rank of the sliced network G - C under its min-fill order and
log2 of the total work (work per slice times 2^k).  Labels are the planner's
exact costs (qtn_cost_exact), features are qtn_cost_features, and the network
is trained on the GPU by libqtn's own forward, backward and Adam kernels
(qtn_mlp_*).  The guided search (qtn_cut_search with a model) re-scores every
set it keeps with the exact evaluator, so no amplitude ever depends on it.

Arrays live in torch device memory; every arithmetic step of training and
inference runs in libqtn.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import qtn


@dataclass
class GraphSpec:
    n: int
    p: int
    edges: list
    graph_id: int


@dataclass
class Dataset:
    X: np.ndarray        # [N, COST_FEATURES] float32
    Y: np.ndarray        # [N, 2] float32: peak rank, log2 cost
    graph: np.ndarray    # [N] graph id of each row


def candidate_sets(spec: GraphSpec, count: int, k_range: Tuple[int, int], rng: np.random.Generator,
                   threads: int = 8) -> np.ndarray:
    """Half uniform-random k-subsets, half offspring-like sets: an Algorithm 1
    cut of the same k with 1..max(1,k/3) members replaced at random."""
    V = spec.n * spec.p
    out = []
    kmin, kmax = k_range
    kmax = min(kmax, V - 1)
    base = {}
    for i in range(count):
        k = int(rng.integers(kmin, kmax + 1))
        if i % 2 == 0:
            s = rng.choice(V, size=k, replace=False)
        else:
            if k not in base:
                base[k], _ = qtn.cut_search(spec.n, spec.edges, spec.p, k,
                                            seed=int(rng.integers(1 << 62)))
            s = np.array(base[k], dtype=np.int64)
            r = int(rng.integers(1, max(1, k // 3) + 1))
            pos = rng.choice(k, size=r, replace=False)
            for q in pos:
                while True:
                    u = int(rng.integers(V))
                    if u not in s:
                        s[q] = u
                        break
        out.append(np.sort(s))
    return out


def make_dataset(specs: Sequence[GraphSpec], sets_per_graph: int, k_range=(2, 20), seed: int = 0,
                 threads: int = 8) -> Dataset:
    """Features and exact labels of sets_per_graph candidate sets per graph."""
    rng = np.random.default_rng(seed)
    Xs, Ys, Gs = [], [], []
    for spec in specs:
        sets = candidate_sets(spec, sets_per_graph, k_range, rng, threads)
        by_k = {}
        for s in sets:
            by_k.setdefault(len(s), []).append(s)
        for k, group in sorted(by_k.items()):
            arr = np.stack(group).astype(np.uint32)
            Xs.append(qtn.cost_features(spec.n, spec.edges, spec.p, arr))
            w, c = qtn.cost_exact(spec.n, spec.edges, spec.p, arr, threads=threads)
            Ys.append(np.stack([w.astype(np.float32), c.astype(np.float32)], axis=1))
            Gs.append(np.full(len(group), spec.graph_id, dtype=np.int64))
    return Dataset(np.concatenate(Xs), np.concatenate(Ys), np.concatenate(Gs))


@dataclass
class Normalization:
    x_mean: np.ndarray
    x_std: np.ndarray
    y_mean: np.ndarray
    y_std: np.ndarray

    @staticmethod
    def fit(ds: Dataset) -> "Normalization":
        xs = ds.X.std(axis=0)
        ys = ds.Y.std(axis=0)
        return Normalization(ds.X.mean(axis=0), np.where(xs > 1e-6, xs, 1.0).astype(np.float32),
                             ds.Y.mean(axis=0), np.where(ys > 1e-6, ys, 1.0).astype(np.float32))


def train(ds: Dataset, epochs: int = 20, batch: int = 1024, lr: float = 1e-3, seed: int = 0,
          hidden: int = 256, n_hidden: int = 3, device: str = "cuda", log=None):
    """Trains a CostMLP on ds (standardised features and labels).  Returns the
    model (normalisation installed) and the per-epoch mean training loss."""
    import torch
    norm = Normalization.fit(ds)
    X = torch.from_numpy(((ds.X - norm.x_mean) / norm.x_std).astype(np.float32)).to(device)
    Y = torch.from_numpy(((ds.Y - norm.y_mean) / norm.y_std).astype(np.float32)).to(device)
    model = qtn.CostMLP(qtn.COST_FEATURES, hidden, n_hidden, 2, max_batch=batch, seed=seed)
    model.set_normalization(norm.x_mean, norm.x_std, norm.y_mean, norm.y_std)
    stream = torch.cuda.current_stream().cuda_stream
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    losses = []
    N = X.shape[0]
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g).to(device)
        Xp = X[perm].contiguous()
        Yp = Y[perm].contiguous()
        tot, cnt = 0.0, 0
        for i in range(0, N - batch + 1, batch):
            loss = model.train_step(Xp[i:].data_ptr(), Yp[i:].data_ptr(), batch, lr, stream)
            tot += loss
            cnt += 1
        losses.append(tot / max(cnt, 1))
        if log:
            log("epoch %d loss %.4f" % (ep, losses[-1]))
    model.norm = norm
    return model, losses


def predict(model: "qtn.CostMLP", X: np.ndarray, device: str = "cuda") -> np.ndarray:
    """Denormalised predictions [N, 2] for raw features X."""
    import torch
    norm = model.norm
    Xn = torch.from_numpy(((X - norm.x_mean) / norm.x_std).astype(np.float32)).to(device)
    out = torch.empty((X.shape[0], 2), dtype=torch.float32, device=device)
    stream = torch.cuda.current_stream().cuda_stream
    for i in range(0, X.shape[0], model.max_batch):
        b = min(model.max_batch, X.shape[0] - i)
        model.forward(Xn[i:].data_ptr(), b, out[i:].data_ptr(), stream)
    torch.cuda.synchronize()
    return out.cpu().numpy() * norm.y_std + norm.y_mean


K_FEATURE = 26      # column of k in the feature vector


def evaluate(model, ds: Dataset) -> dict:
    """MAE of peak rank and log2 cost, the mean per-graph Spearman rho of the
    predicted log2 cost, and the same rho within (graph, k) groups (the
    ranking a search of fixed k relies on)."""
    from scipy.stats import spearmanr
    P = predict(model, ds.X)
    rho, rho_k = [], []
    for gid in np.unique(ds.graph):
        m = ds.graph == gid
        if m.sum() > 2:
            rho.append(spearmanr(P[m, 1], ds.Y[m, 1]).statistic)
        for k in np.unique(ds.X[m, K_FEATURE]):
            mk = m & (ds.X[:, K_FEATURE] == k)
            if mk.sum() > 10 and np.ptp(ds.Y[mk, 1]) > 0:
                rho_k.append(spearmanr(P[mk, 1], ds.Y[mk, 1]).statistic)
    return {"mae_rank": float(np.abs(P[:, 0] - ds.Y[:, 0]).mean()),
            "mae_log2_cost": float(np.abs(P[:, 1] - ds.Y[:, 1]).mean()),
            "spearman_log2_cost": float(np.mean(rho)),
            "spearman_log2_cost_fixed_k": float(np.mean(rho_k)) if rho_k else None,
            "rows": int(ds.X.shape[0])}


def random_search(spec: GraphSpec, k: int, count: int, seed: int, threads: int = 1):
    """Best of `count` uniform-random k-subsets, scored exactly."""
    rng = np.random.default_rng(seed)
    V = spec.n * spec.p
    t = time.perf_counter()
    sets = np.stack([np.sort(rng.choice(V, size=k, replace=False)) for _ in range(count)])
    w, c = qtn.cost_exact(spec.n, spec.edges, spec.p, sets.astype(np.uint32), threads=threads)
    i = min(range(count), key=lambda j: (w[j], c[j]))
    return [int(v) for v in sets[i]], {"seconds": time.perf_counter() - t, "exact_evals": count,
                                       "model_evals": 0, "width": int(w[i]),
                                       "log2_cost": float(c[i])}


def gain_comparison(model, specs: Sequence[GraphSpec], k: int, seeds: Sequence[int],
                    pop: int = 11, iters: int = 4, factor: int = 16) -> List[dict]:
    """(i) Algorithm 1 with exact fitness; (ii) model-guided search with
    `factor` x more offspring per generation, the model keeping the best N for
    exact scoring; (ii') the same loop with factor 1, where every offspring is
    scored and the model decides nothing (the model's own contribution is
    (ii) against (ii')); (iii) random sets with as many exact evaluations as
    (ii).  Every reported cost is an exact re-score."""
    rows = []
    for spec in specs:
        for s in seeds:
            cut1, st1 = qtn.cut_search(spec.n, spec.edges, spec.p, k, pop, iters, s)
            cut2, st2 = qtn.cut_search(spec.n, spec.edges, spec.p, k, pop, iters, s, model=model,
                                       offspring_factor=factor)
            w2, c2 = qtn.cost_exact(spec.n, spec.edges, spec.p, np.array([cut2], dtype=np.uint32))
            assert int(w2[0]) == st2["width"] and float(c2[0]) == st2["log2_cost"]
            _, st2b = qtn.cut_search(spec.n, spec.edges, spec.p, k, pop, iters, s, model=model,
                                     offspring_factor=1)
            cut3, st3 = random_search(spec, k, int(st2["exact_evals"]), s)
            rows.append({"n": spec.n, "p": spec.p, "graph": spec.graph_id, "k": k, "seed": s,
                         "alg1": st1, "guided": st2, "unscreened": st2b, "random": st3})
    return rows


def _main():
    import argparse
    import json
    import sys
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from instances import make_instance

    ap = argparse.ArgumentParser(description="train and evaluate the cut-set cost model")
    ap.add_argument("--sets", type=int, default=100000, help="labelled sets in total")
    ap.add_argument("--graphs-per-np", type=int, default=5)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--k-gain", type=int, default=14)
    ap.add_argument("--gain-seeds", type=int, default=4)
    ap.add_argument("--threads", type=int, default=16)
    args = ap.parse_args()
    t0 = time.perf_counter()
    specs = []
    gid = 0
    for n in (60, 80, 100, 120):
        for p in (1, 2):
            for g in range(args.graphs_per_np):
                inst = make_instance(n, p, 1, 1000 + gid)
                specs.append(GraphSpec(n, p, inst.edges, gid))
                gid += 1
    per = max(1, args.sets // len(specs))
    ds = make_dataset(specs, per, seed=1, threads=args.threads)
    t_data = time.perf_counter() - t0
    held = set(s.graph_id for i, s in enumerate(specs) if i % 10 == 9)
    tr = np.array([g not in held for g in ds.graph])
    train_ds = Dataset(ds.X[tr], ds.Y[tr], ds.graph[tr])
    test_ds = Dataset(ds.X[~tr], ds.Y[~tr], ds.graph[~tr])
    t1 = time.perf_counter()
    model, losses = train(train_ds, epochs=args.epochs,
                          log=lambda m: print("#", m, file=sys.stderr, flush=True))
    t_train = time.perf_counter() - t1
    ev = evaluate(model, test_ds)
    gain_specs = []
    for n in (80, 120):
        for p in (1, 2):
            inst = make_instance(n, p, 1, 5000 + n + p)
            gain_specs.append(GraphSpec(n, p, inst.edges, -1))
    rows = gain_comparison(model, gain_specs, args.k_gain, list(range(args.gain_seeds)))
    print(json.dumps({"dataset_rows": int(ds.X.shape[0]), "dataset_seconds": t_data,
                      "train_seconds": t_train, "epochs": args.epochs, "final_loss": losses[-1],
                      "held_out": ev, "gain": rows}))


if __name__ == "__main__":
    _main()
