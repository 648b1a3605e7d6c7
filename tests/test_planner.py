"""CPU tests of the host planner behind the C ABI: bit-exact agreement of the
min-fill order, the cut search and every index map with independent
re-derivations, and amplitudes of the exported schedule against the oracle."""
import os
import re

import numpy as np
import pytest

from instances import make_instance, workload_instance
from oracle import qaoa as Q
from oracle.search import ga_cut_search, ga_min_k
from paper_2010_14962_amd import qtn
from paper_2010_14962_amd.qtn import plan_instance, QtnError

import schedule_interp as SI

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "qtn.h")) as f:
        text = f.read()
    declared = set(re.findall(r"^\s*(?:int|void|const char \*)\s*(qtn_\w+)\s*\(", text, re.M))
    assert {"qtn_plan", "qtn_contract", "qtn_plan_bind_workspace"} <= declared
    L = qtn.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(qtn.EXPORTS)


@pytest.mark.parametrize("n,p,seed,k", [(16, 1, 0, 0), (16, 1, 1, 3), (20, 2, 2, 4),
                                        (40, 2, 3, 6), (60, 1, 4, 5)])
def test_min_fill_order_bit_exact(n, p, seed, k):
    inst = make_instance(n, p, 1, seed)
    rng = np.random.default_rng(seed)
    cut = sorted(int(c) for c in rng.choice(n * p, size=k, replace=False))
    P = plan_instance(inst, cut_vars=cut)
    adj = Q.interaction_graph(n, inst.edges, p)
    order, _ = Q.min_fill_order(adj, removed=cut)
    assert P.cut() == cut
    assert P.order() == order


@pytest.mark.parametrize("n,p,seed,M", [(16, 1, 5, 2), (20, 2, 6, 5), (40, 2, 7, 8)])
def test_cut_search_matches_reference_algorithm(n, p, seed, M):
    inst = make_instance(n, p, 1, seed)
    adj = Q.interaction_graph(n, inst.edges, p)
    ref_cut, (w, work) = ga_cut_search(adj, M, N=11, T=4, seed=1234 + seed)
    P = plan_instance(inst, k=M, seed=1234 + seed)
    assert P.cut() == ref_cut
    assert P.info()["work"] == work


def test_min_k_search_matches_reference():
    inst = make_instance(24, 2, 1, 8)
    adj = Q.interaction_graph(24, inst.edges, 2)
    w0 = Q.elimination_cost(adj, Q.min_fill_order(adj)[0])[0]
    cap = w0 - 3
    ref = ga_min_k(adj, cap, 10, seed=5)
    P = plan_instance(inst, k=-1, max_rank=cap, k_max=10, seed=5)
    assert P.cut() == ref[0]
    assert P.info()["width"] <= cap


def _check_maps(P):
    steps, tens = P.export()
    derived = SI.derived_masks(P, steps, tens)
    for t, rec in enumerate(steps):
        nin, nk, rC = int(rec[1]), int(rec[2]), int(rec[3])
        for i in range(nin):
            m = int(rec[13 + i]) & 0xFFFFFFFF
            assert m == derived[t][i], (t, i)
            tab = P.index_table(t, i)
            cm = m & ((1 << rC) - 1)
            km = m >> rC
            c = np.arange(256, dtype=np.int64)
            assert np.array_equal(tab[:256], SI.pext_vec(c, cm & 255))
            u = np.arange(16, dtype=np.int64)
            assert np.array_equal(tab[256:272], SI.pext_vec(u << 8, cm))
            assert tab[272] == cm >> 12 and tab[273] == SI.popcount(cm & 4095)
            kap = np.arange(1 << nk, dtype=np.int64)
            assert np.array_equal(tab[274:], SI.pext_vec(kap, km) << SI.popcount(cm))
            # every input variable list is a subsequence of the step's index list
            tr = tens[rec[5 + i]]
            assert SI.popcount(m) == tr[0]
    return steps, tens


@pytest.mark.parametrize("fuse", [True, False])
def test_index_maps_bit_exact(fuse):
    inst = make_instance(20, 2, 2, 9)
    P = plan_instance(inst, k=3, seed=2, fuse_chains=fuse)
    _check_maps(P)


def test_slice_bit_assignment_bit_exact():
    """Leaf variants are chosen by pext(slice, selmask); selmask holds the
    slice bits b of the cut variables cut[b] that the leaf touches."""
    inst = make_instance(16, 1, 1, 10)
    P = plan_instance(inst, cut_vars=[1, 6, 11])
    cut = P.cut()
    steps, tens = P.export()
    adj_f, _ = Q.qaoa_factors(16, inst.edges, 1, inst.gamma, inst.beta, inst.bitstrings[0])
    order = P.order()
    pos = {v: i for i, v in enumerate(order)}
    seen = 0
    for t in range(tens.shape[0]):
        if tens[t, 1] != 0:
            continue
        sel = int(tens[t, 3]) & 0xFFFFFFFF
        vars_ = [int(v) for v in tens[t, 4:4 + tens[t, 0]]]
        # cut variables adjacent (through one factor) to the leaf's first variable group
        bits = [b for b in range(len(cut)) if (sel >> b) & 1]
        for b in bits:
            c = cut[b]
            assert any(c in vs and any(v in vs for v in vars_) or (c in vs and not vars_)
                       for vs, _ in adj_f)
        seen |= sel
        assert vars_ == sorted(vars_, key=lambda v: pos[v])
    assert seen == (1 << len(cut)) - 1


@pytest.mark.parametrize("n,p,seed,k,fuse", [(16, 1, 0, 2, True), (16, 1, 0, 2, False),
                                             (12, 2, 1, 3, True), (10, 2, 2, 0, True),
                                             (8, 2, 3, 5, True)])
def test_schedule_amplitude_matches_oracle(n, p, seed, k, fuse):
    inst = make_instance(n, p, 2, seed)
    P = plan_instance(inst, k=k, seed=seed, fuse_chains=fuse)
    cut = P.cut()
    _check_maps(P)
    got = SI.run(P, range(1 << len(cut)))
    for b in range(2):
        x = inst.bitstrings[b]
        ref_parts = [Q.slice_partial(n, inst.edges, p, inst.gamma, inst.beta, x, cut, s)
                     for s in range(1 << len(cut))]
        for a, r in zip(got[b], ref_parts):
            assert abs(a - r) <= 1e-13 * 2.0 ** (-n / 2)
        sv = Q.statevector_amplitude(n, inst.edges, p, inst.gamma, inst.beta, x)
        assert abs(sum(got[b]) - sv) <= 1e-12 * 2.0 ** (-n / 2)


def _absorbed_inputs(P):
    """Inputs of fused steps that are stored intermediates without the first
    summed variable: tensors of a following bucket taken into the step."""
    steps, tens = P.export()
    hits = []
    for t in range(len(steps)):
        if steps[t, 2] < 2:
            continue
        kap = P.kappa(t)
        for i in steps[t, 5:5 + steps[t, 1]]:
            vs = [int(v) for v in tens[i, 4:4 + tens[i, 0]]]
            if tens[i, 1] == 1 and kap[0] not in vs:
                assert all(v in kap or v in _step_vars(P, steps, tens, t) for v in vs)
                hits.append((t, int(i)))
    return hits


def _step_vars(P, steps, tens, t):
    out = int(steps[t, 0])
    return [int(v) for v in tens[out, 4:4 + tens[out, 0]]]


def test_chain_fusion_absorbs_tensors_inside_the_index_space():
    # a following bucket whose other tensors lie inside the step's index
    # space is summed in the same step; the sum over the whole schedule is
    # still the amplitude (Eq. (1) per bucket, Sec. II B)
    inst = make_instance(10, 2, 2, 0)
    P = plan_instance(inst, k=0, seed=0)
    assert len(_absorbed_inputs(P)) >= 1
    got = SI.run(P, [0])
    for b in range(2):
        sv = Q.statevector_amplitude(10, inst.edges, 2, inst.gamma, inst.beta, inst.bitstrings[b])
        assert abs(got[b][0] - sv) <= 1e-12 * 2.0 ** (-5)
    # n=80 p=2 k=16: the last expansion of the order (to a rank-19 tensor that
    # only the next bucket reads) is not stored any more
    inst = workload_instance("qaoa_n80_p2_k16")
    from instances import search_params
    P = plan_instance(inst, k=16, max_rank=inst.meta["max_rank"], precision="fp32",
                      **search_params("qaoa_n80_p2_k16"))
    info = P.info()
    assert _absorbed_inputs(P)
    assert info["width"] < info["mf_width"], info


def test_workload_plans_meet_caps():
    for name in ["qaoa_n16_p1_k2", "qaoa_n40_p2_b32_k8", "qaoa_n120_p1_b8"]:
        inst = workload_instance(name)
        w = inst.meta
        P = plan_instance(inst, k=w["k"] if w["k"] is not None else -1,
                          max_rank=w["max_rank"] or 0, precision=w["precision"])
        info = P.info()
        if w["k"] is not None:
            assert info["k"] == w["k"]
        if w["max_rank"]:
            assert info["width"] <= w["max_rank"]
        assert P.workspace_bytes(1) > 0


def test_errors_are_reported():
    inst = make_instance(8, 1, 1, 0)
    with pytest.raises(QtnError) as e:
        qtn.qtn_plan(8, [(0, 0)] + list(inst.edges[1:]), 1, inst.gamma, inst.beta, inst.bitstrings)
    assert e.value.code == qtn.QTN_EINVAL
    with pytest.raises(QtnError):
        qtn.qtn_plan(8, inst.edges + [inst.edges[0]], 1, inst.gamma, inst.beta, inst.bitstrings)
    bad = inst.bitstrings.copy()
    bad[0, 0] = 2
    with pytest.raises(QtnError):
        qtn.qtn_plan(8, inst.edges, 1, inst.gamma, inst.beta, bad)
    with pytest.raises(QtnError):
        qtn.qtn_plan(8, inst.edges, 1, [float("nan")], inst.beta, inst.bitstrings)
    with pytest.raises(QtnError):
        plan_instance(inst, cut_vars=[99])
    with pytest.raises(QtnError) as e:
        plan_instance(inst, k=2, precision="3xbf16")
    assert e.value.code == qtn.QTN_EINVAL and "dense" in str(e.value)
    with pytest.raises(QtnError) as e:
        plan_instance(inst, k=-1, max_rank=0, k_max=0, cut_vars=None) and None
        plan_instance(inst, k=0, max_rank=1)
    assert e.value.code == qtn.QTN_ERANK
    P = plan_instance(inst, k=2)
    with pytest.raises(QtnError) as e:
        P.contract(3, 2)
    assert e.value.code == qtn.QTN_ERANGE
    with pytest.raises(QtnError) as e:
        P.contract(0, 5)
    assert e.value.code == qtn.QTN_ERANGE
    with pytest.raises(QtnError) as e:
        P.contract(0, 4)
    assert e.value.code == qtn.QTN_ENOMEM
    assert P.contract(2, 2)[0].value() == 0j


def test_partial_combine_is_error_free():
    a = qtn.QtnPartial(1e16, 1.0, 0.0, 0.0)
    b = qtn.QtnPartial(1.0, -1e16, 0.0, 0.0)
    c = qtn.qtn_partial_combine(a, b)
    assert c.re == 1e16 + 1.0 and c.re_comp == 1.0 - ((1e16 + 1.0) - 1e16)
    assert (c.re + c.re_comp) - 1e16 == 0.0 or c.re_comp == 1.0


@pytest.mark.parametrize("name,k,mode", [("qaoa_n120_p1_b8", -1, "wide"), ("qaoa_n120_p1_b8", 4, "wide"),
                                         ("qaoa_n120_p1_b8", 4, "slice"),
                                         ("qaoa_n40_p2_b32_k8", 8, "wide"),
                                         ("qaoa_n80_p2_k16", 16, "wide"), ("qaoa_n80_p2_k16", 16, "slice")])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_workspace_layout_self_check(name, k, mode, precision):
    """Layouts for every wave size keep simultaneously live tensors apart
    (the library verifies this itself and errors otherwise)."""
    inst = workload_instance(name)
    P = plan_instance(inst, k=k, max_rank=26, precision=precision, exec_mode=mode)
    for S in (1, 3, 64, 1 << min(P.info()["k"], 10)):
        assert P.workspace_bytes(S) > 0


def test_rescaling_only_with_64bit_tensors():
    """The mixed form runs the rescaling kernels only when some intermediate
    is stored in the 64-bit form outside LDS; with every stored tensor
    complex128 it reduces to the FP64 kernels.  FP64 plans never rescale."""
    big = workload_instance("qaoa_n120_p1_b8")
    P = plan_instance(big, k=-1, max_rank=26, precision="fp32")
    steps, tens = P.export()
    assert any(t[1] == 1 and not (t[2] & 4) for t in tens)
    assert P.info()["rescaled"] & 1
    assert plan_instance(big, k=-1, max_rank=26, precision="fp64").info()["rescaled"] == 0
    # width 8: every intermediate of a slice lives in LDS (complex128 there)
    small = workload_instance("qaoa_n120_p1_b8_k16")
    Ps = plan_instance(small, k=16, max_rank=26, precision="fp32")
    assert Ps.info()["rescaled"] == 0
