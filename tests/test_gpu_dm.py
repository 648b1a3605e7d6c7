"""Density-matrix form (Sec. II A) on the GPU against the Markov-Shi oracle
(oracle/dm.py, contracted over unmerged 4-valued wires): the sum of all 4^m
slices is the probability |<x|U|0^n>|^2, and single slices equal the oracle's
slices with the cut edges fixed to the same operator basis elements."""
import itertools

import pytest

from instances import make_instance
from oracle import dm as DM
from oracle import qaoa as Q
from paper_2010_14962_amd import plan_instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-12, "fp32": 1e-6}


def _stream():
    return torch.cuda.current_stream().cuda_stream


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n,p,m,seed", [(6, 1, 1, 0), (6, 2, 2, 1), (8, 1, 2, 2)])
def test_dm_slices_against_markov_shi_oracle(precision, n, p, m, seed):
    print("case dm", n, p, m, precision, flush=True)
    inst = make_instance(n, p, 2, seed)
    plan = plan_instance(inst, k=m, precision=precision, density_matrix=True)
    cut = plan.cut()                       # 2m binary variables: ket ids, then bra copies
    V = n * p
    pairs = cut[:m]
    assert cut[m:] == [c + V for c in pairs]
    plan.bind_torch(4 ** m)
    tot = [pp.value() for pp in plan.contract(0, 4 ** m, _stream())]
    refs = []
    for b in range(2):
        ref = DM.dm_probability(n, inst.edges, p, inst.gamma, inst.beta, inst.bitstrings[b]).real
        sv = abs(Q.statevector_amplitude(n, inst.edges, p, inst.gamma, inst.beta, inst.bitstrings[b])) ** 2
        assert abs(ref - sv) <= 1e-12 * sv
        assert abs(tot[b].real - ref) <= TOL[precision] * ref, (b, tot[b], ref)
        assert abs(tot[b].imag) <= TOL[precision] * ref
        refs.append(ref)
    # single slices: slice bit j (j < m) is the ket value of pair j, bit m + j
    # its bra value; the oracle fixes the wire entering layer l of qubit q to
    # |a><b|, basis index 2a + b
    cpairs = [(v % n, v // n) for v in pairs]
    plan.set_graphs(False)
    wants = []
    for s in range(4 ** m):
        sig = [2 * ((s >> j) & 1) + ((s >> (m + j)) & 1) for j in range(m)]
        wants.append(DM.dm_slice(n, inst.edges, p, inst.gamma, inst.beta, inst.bitstrings[0], cpairs, sig))
    scale = max(abs(w) for w in wants)     # per-slice errors relative to the largest slice
    for s in range(4 ** m):
        got = plan.contract(s, s + 1, _stream())[0].value()
        assert abs(got - wants[s]) <= TOL[precision] * scale, (s, got, wants[s])
