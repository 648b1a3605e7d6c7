"""qtn_contract_noalloc (the entry point for callers that cannot allocate)
against qtn_contract on the same plans and slices per wave: two calls in a
row on one plan, the second on a smaller slice range, then a smaller plan,
each compared bit for bit (the same kernels in the same order).  The file
name puts it after every other GPU test."""
import numpy as np
import pytest

from instances import make_instance, workload_instance
from paper_2010_14962_amd import plan_instance, qtn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _noalloc(plan, lo, hi, S):
    B = plan.n_bitstrings
    out = torch.full((B, 4), float("nan"), dtype=torch.float64, device="cuda")
    plan.contract_noalloc(lo, hi, S, out.data_ptr(), _stream())
    torch.cuda.synchronize()
    return [tuple(r) for r in out.cpu().numpy().tolist()]


def _bound(plan, lo, hi):
    return [(p.re, p.im, p.re_comp, p.im_comp) for p in plan.contract(lo, hi, _stream())]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_bound_workspace(precision):
    print("case noalloc", precision, flush=True)
    big = plan_instance(make_instance(30, 2, 4, 0), k=4, precision=precision)
    S = 16
    ref_full = None
    # the bound-workspace reference (its own memory, graph replay)
    ref = plan_instance(make_instance(30, 2, 4, 0), cut_vars=big.cut(), precision=precision)
    ref.bind_torch(S)
    ref_full = _bound(ref, 0, 16)
    ref_part = _bound(ref, 3, 13)
    got_full = _noalloc(big, 0, 16, S)
    assert got_full == ref_full
    got_part = _noalloc(big, 3, 13, S)          # second call: a smaller slice range
    assert got_part == ref_part
    # a smaller plan on the same scratch
    small_inst = make_instance(16, 1, 1, 3)
    small = plan_instance(small_inst, k=2, precision=precision)
    sref = plan_instance(small_inst, cut_vars=small.cut(), precision=precision)
    sref.bind_torch(4)
    assert _noalloc(small, 0, 4, 4) == _bound(sref, 0, 4)
    # empty range: exact zeros
    assert _noalloc(small, 2, 2, 4) == [(0.0, 0.0, 0.0, 0.0)]


def test_noalloc_rejects_oversize_plan():
    inst = workload_instance("qaoa_n120_p1_b8", seed=0)
    plan = plan_instance(inst, k=0, precision="fp32")
    out = torch.zeros((8, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(qtn.QtnError) as e:
        plan.contract_noalloc(0, 1, 1, out.data_ptr(), _stream())
    assert e.value.code == qtn.QTN_ENOMEM and "bytes of scratch" in str(e.value)
