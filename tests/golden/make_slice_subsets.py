"""Writes the oracle's slice values of the two sliced benchmark workloads to
tests/golden/ (run from the repository root; calls only oracle/ and the
input generator).

For each workload the cut set is Algorithm 1's (oracle/search.py, the
workload's N and T, seed 0), the order of every slice is the oracle's own
min-degree order, and the values are complex128 slice contractions with the
cut variables fixed (Sec. III A, Fig. 3):
  qaoa_n80_p2_k16      bitstring 0, every slice s in [0, 1024), and the
                       Neumaier sum over that range;
  qaoa_n120_p1_b8_k16  per bitstring the Neumaier sum over [0, 1024) and the
                       single slices 0, 1, 2, 511, 1023.
Usage: python tests/golden/make_slice_subsets.py [workers]
"""
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from instances import search_params, workload_instance  # noqa: E402
from oracle import qaoa as Q  # noqa: E402
from oracle.search import ga_cut_search  # noqa: E402

SUBSET = 1024
SINGLES = (0, 1, 2, 511, 1023)


def _slice(args):
    name, b, cut, s = args
    inst = workload_instance(name, seed=0)
    return Q.slice_partial(inst.n, inst.edges, inst.p, inst.gamma, inst.beta, inst.bitstrings[b], cut, s)


def _cut(name):
    inst = workload_instance(name, seed=0)
    sp = search_params(name)
    adj = Q.interaction_graph(inst.n, inst.edges, inst.p)
    cut, (w, work) = ga_cut_search(adj, inst.meta["k"], N=sp["ga_pop"], T=sp["ga_iters"], seed=0)
    return inst, cut, w


def _hex(z):
    return "%s %s" % (float(z.real).hex(), float(z.imag).hex())


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else min(8, os.cpu_count() or 1)
    with mp.get_context("spawn").Pool(workers) as pool:
        # n = 80, p = 2: every slice of the subset for bitstring 0
        name = "qaoa_n80_p2_k16"
        inst, cut, w = _cut(name)
        vals = pool.map(_slice, [(name, 0, cut, s) for s in range(SUBSET)])
        re, rc = Q.neumaier_sum(v.real for v in vals)
        im, ic = Q.neumaier_sum(v.imag for v in vals)
        with open(os.path.join(HERE, "slices_%s.txt" % name), "w") as f:
            f.write("# oracle slice values, %s seed 0, bitstring 0; written by make_slice_subsets.py\n" % name)
            f.write("cut %s\n" % " ".join(str(c) for c in cut))
            f.write("width %d\n" % w)
            f.write("sum %s\n" % _hex(complex(re + rc, im + ic)))
            for s, v in enumerate(vals):
                f.write("slice %d %s\n" % (s, _hex(v)))
        # n = 120, p = 1, 8 bitstrings: sums over the subset and a few slices
        name = "qaoa_n120_p1_b8_k16"
        inst, cut, w = _cut(name)
        with open(os.path.join(HERE, "slices_%s.txt" % name), "w") as f:
            f.write("# oracle slice values, %s seed 0; written by make_slice_subsets.py\n" % name)
            f.write("cut %s\n" % " ".join(str(c) for c in cut))
            f.write("width %d\n" % w)
            for b in range(inst.n_bitstrings):
                vals = pool.map(_slice, [(name, b, cut, s) for s in range(SUBSET)])
                re, rc = Q.neumaier_sum(v.real for v in vals)
                im, ic = Q.neumaier_sum(v.imag for v in vals)
                f.write("sum %d %s\n" % (b, _hex(complex(re + rc, im + ic))))
                for s in SINGLES:
                    f.write("slice %d %d %s\n" % (b, s, _hex(vals[s])))
                print(name, "bitstring", b, "done", flush=True)


if __name__ == "__main__":
    main()
