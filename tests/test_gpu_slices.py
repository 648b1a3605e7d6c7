"""Sliced workloads of the benchmark against stored oracle values.

tests/golden/slices_*.txt are written by tests/golden/make_slice_subsets.py,
which calls only oracle/ (Algorithm 1 for the cut set, complex128 slice
contractions, Neumaier sums).  The cut set is integer work and must agree bit
for bit; slice values and subset sums agree within the precision form's
tolerance: 1e-12 (FP64) or 1e-6 (mixed), relative to the oracle value for
sums and relative to the largest slice value for single slices (Sec. III A:
the slice values sum to the amplitude, Eq. (2)).
"""
import os

import pytest

from instances import search_params, workload_instance
from paper_2010_14962_amd import plan_instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = {"fp64": 1e-12, "fp32": 1e-6}


def _hex(a, b):
    return complex(float.fromhex(a), float.fromhex(b))


def _golden(name):
    g = {"sum": {}, "slice": {}}
    with open(os.path.join(GOLDEN, "slices_%s.txt" % name)) as f:
        for line in f:
            w = line.split()
            if not w or w[0].startswith("#"):
                continue
            if w[0] == "cut":
                g["cut"] = [int(v) for v in w[1:]]
            elif w[0] == "width":
                g["width"] = int(w[1])
            elif w[0] == "sum":
                if len(w) == 3:
                    g["sum"][0] = _hex(w[1], w[2])
                else:
                    g["sum"][int(w[1])] = _hex(w[2], w[3])
            elif w[0] == "slice":
                if len(w) == 4:
                    g["slice"][(0, int(w[1]))] = _hex(w[2], w[3])
                else:
                    g["slice"][(int(w[1]), int(w[2]))] = _hex(w[3], w[4])
    return g


def _stream():
    return torch.cuda.current_stream().cuda_stream


@pytest.mark.parametrize("name", ["qaoa_n80_p2_k16", "qaoa_n120_p1_b8_k16"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_slice_subset_against_oracle(name, precision):
    print("case", name, precision, flush=True)
    inst = workload_instance(name, seed=0)
    g = _golden(name)
    plan = plan_instance(inst, k=inst.meta["k"], max_rank=inst.meta["max_rank"], precision=precision,
                         **search_params(name))
    assert plan.cut() == g["cut"]            # Algorithm 1 with SplitMix64: bit-exact
    assert plan.info()["width"] <= inst.meta["max_rank"]
    plan.bind_torch(1024)
    sums = [p.value() for p in plan.contract(0, 1024, _stream())]
    for b, ref in g["sum"].items():
        err = abs(sums[b] - ref) / abs(ref)
        print("bitstring %d: subset sum rel err %.3e" % (b, err), flush=True)
        assert err <= TOL[precision], (b, sums[b], ref)
    # single slices, launched directly (no graph per range)
    plan.set_graphs(False)
    by_b = {}
    for (b, s), ref in g["slice"].items():
        by_b.setdefault(b, {})[s] = ref
    worst = 0.0
    for b, refs in by_b.items():
        scale = max(abs(v) for v in refs.values())
        for s, ref in refs.items():
            got = plan.contract(s, s + 1, _stream())[b].value()
            worst = max(worst, abs(got - ref) / scale)
    print("single slices: %d, worst error / largest slice value %.3e" % (len(g["slice"]), worst), flush=True)
    assert worst <= TOL[precision]
