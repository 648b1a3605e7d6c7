"""Several circuits of uneven size in one persistent launch
(qtn_batch_contract): every plan's partials equal its own contraction bit for
bit, and the summed slices equal the oracle amplitude (Eq. (2))."""
import pytest

from instances import make_instance
from oracle import qaoa as Q
from paper_2010_14962_amd import batch_contract, plan_instance, qtn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SPECS = [(16, 1, 2, 2, 0), (24, 2, 1, 3, 1), (30, 1, 3, 4, 2), (20, 2, 2, 0, 3)]   # n, p, B, k, seed


def _key(parts):
    return [(p.re, p.im, p.re_comp, p.im_comp) for p in parts]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_uneven_circuits_in_one_launch(precision):
    print("case batch", precision, flush=True)
    stream = torch.cuda.current_stream().cuda_stream
    insts = [make_instance(n, p, B, seed) for n, p, B, k, seed in SPECS]
    plans, refs = [], []
    for inst, (n, p, B, k, seed) in zip(insts, SPECS):
        plan = plan_instance(inst, k=k, precision=precision, exec_mode="slice")
        plan.bind_torch(1 << k)
        plans.append(plan)
        refs.append(_key(plan.contract(0, 1 << k, stream)))
    got = batch_contract(plans, [(0, 1 << s[3]) for s in SPECS], stream)
    for i, g in enumerate(got):
        assert _key(g) == refs[i], i
    # amplitudes against the oracle
    for inst, plan, g in zip(insts, plans, got):
        for b in range(inst.n_bitstrings):
            ref = Q.ve_amplitude(inst.n, inst.edges, inst.p, inst.gamma, inst.beta, inst.bitstrings[b])
            assert abs(g[b].value() - ref) <= (1e-12 if precision == "fp64" else 1e-6) * abs(ref)
    # partial ranges, one empty, in a second call on the same plans
    ranges = [(1, 3), (0, 0), (5, 16), (0, 1)]
    got2 = batch_contract(plans, ranges, stream)
    for i, (plan, (lo, hi)) in enumerate(zip(plans, ranges)):
        want = _key(plan.contract(lo, hi, stream)) if hi > lo else [(0.0, 0.0, 0.0, 0.0)] * plan.n_bitstrings
        assert _key(got2[i]) == want, i


def test_batch_rejects_plans_not_in_slice_mode():
    inst = make_instance(16, 1, 1, 0)
    plan = plan_instance(inst, k=2, precision="fp64", exec_mode="wide")
    plan.bind_torch(4)
    with pytest.raises(qtn.QtnError) as e:
        batch_contract([plan], [(0, 4)])
    assert e.value.code == qtn.QTN_ESTATE
