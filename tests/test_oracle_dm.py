"""Pins of the density-matrix (Markov-Shi) oracle, oracle/dm.py, against facts
that do not come from it: the probability |<x|U|0^n>|^2 from the independent
statevector, the slice identity over 4-valued cut edges (Eq. (2), 4^m
subgraphs, Sec. III A), and the factorisation of a density-matrix slice into
a ket slice times the conjugate of a ket slice (the basis element |a><b|
fixes the ket wire to a and the bra wire to b)."""
import numpy as np
import pytest

from instances import make_instance
from oracle import dm as DM
from oracle import qaoa as Q


@pytest.mark.parametrize("n,p,seed", [(4, 1, 0), (6, 1, 1), (4, 2, 2), (6, 2, 3)])
def test_dm_probability_matches_statevector(n, p, seed):
    inst = make_instance(n, p, 3, seed)
    psi = Q.statevector(n, inst.edges, p, inst.gamma, inst.beta)
    for b in range(3):
        x = inst.bitstrings[b]
        ref = abs(psi[sum(int(v) << i for i, v in enumerate(x))]) ** 2
        got = DM.dm_probability(n, inst.edges, p, inst.gamma, inst.beta, x)
        assert abs(got.imag) <= 1e-14
        assert abs(got.real - ref) <= 1e-12 * max(ref, 1e-3)


def test_dm_probabilities_sum_to_one():
    inst = make_instance(4, 1, 1, 4)
    tot = 0.0
    for bits in range(16):
        x = [(bits >> i) & 1 for i in range(4)]
        tot += DM.dm_probability(4, inst.edges, 1, inst.gamma, inst.beta, x).real
    assert abs(tot - 1.0) <= 1e-12


@pytest.mark.parametrize("cut", [[(0, 0)], [(1, 0), (3, 0)], [(2, 1), (0, 0)]])
def test_dm_slice_identity_and_ket_bra_factorisation(cut):
    n, p = 4, 2
    inst = make_instance(n, p, 1, 5)
    x = inst.bitstrings[0]
    whole = DM.dm_probability(n, inst.edges, p, inst.gamma, inst.beta, x)
    sliced = DM.dm_sliced_sum(n, inst.edges, p, inst.gamma, inst.beta, x, cut)
    assert abs(sliced - whole) <= 1e-12 * abs(whole)
    # sigma = |a><b| on the wire of merged variable v(q, l): ket slice with
    # v = a times the conjugate of the ket slice with v = b
    kvars = [Q.variable_id(n, q, l) for q, l in cut]
    order = sorted(range(len(cut)), key=lambda j: kvars[j])
    kcut = [kvars[j] for j in order]
    for sig in [(0,) * len(cut), (1,) * len(cut), (2,) + (3,) * (len(cut) - 1)]:
        a = [s >> 1 for s in sig]
        bb = [s & 1 for s in sig]
        sa = sum(a[j] << i for i, j in enumerate(order))
        sb = sum(bb[j] << i for i, j in enumerate(order))
        ka = Q.slice_partial(n, inst.edges, p, inst.gamma, inst.beta, x, kcut, sa)
        kb = Q.slice_partial(n, inst.edges, p, inst.gamma, inst.beta, x, kcut, sb)
        got = DM.dm_slice(n, inst.edges, p, inst.gamma, inst.beta, x, cut, sig)
        ref = ka * np.conj(kb)
        assert abs(got - ref) <= 1e-12 * max(abs(whole), 1e-6), (sig, got, ref)
