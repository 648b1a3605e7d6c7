"""Range-partitioned contraction: fixed-order combination, re-issue of a lost
range and resume from the JSONL checkpoint (Sec. III A: independent slices
whose values the master sums; Sec. V: missing slices are recomputed).

The host-only tests need no GPU: a checkpoint that already holds every range
is combined without any device work."""
import numpy as np
import pytest

from instances import make_instance, workload_instance
from paper_2010_14962_amd import plan_instance, qtn


def _two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def _combine(a, b):
    """TwoSum on each component, written from its definition (Knuth)."""
    sr, er = _two_sum(a[0], b[0])
    si, ei = _two_sum(a[1], b[1])
    return (sr, si, a[2] + b[2] + er, a[3] + b[3] + ei)


def _header(plan, R, B, k):
    return ('{"qtn_checkpoint": 1, "plan": "%016x", "range_slices": %d, "bitstrings": %d, "k": %d}'
            % (plan.fingerprint(), R, B, k))


def _line(lo, hi, parts):
    vals = ", ".join('"%s"' % float(v).hex() for p in parts for v in p)
    return '{"lo": %d, "hi": %d, "p": [%s]}' % (lo, hi, vals)


def test_checkpoint_resume_combines_in_range_order(tmp_path):
    inst = make_instance(16, 1, 2, 5)
    plan = qtn.qtn_plan(16, inst.edges, 1, inst.gamma, inst.beta, inst.bitstrings, k=3)
    R, B = 3, 2                       # ranges [0,3) [3,6) [6,8)
    rng = np.random.default_rng(0)
    parts = {lo: [tuple(rng.normal(size=4) * 10.0 ** rng.integers(-20, 0, size=4)) for _ in range(B)]
             for lo in (0, 3, 6)}
    ck = tmp_path / "ck.jsonl"
    lines = [_header(plan, R, B, 3)]
    for lo in (6, 0, 3):               # written out of order
        lines.append(_line(lo, min(8, lo + R), parts[lo]))
    lines.append('{"lo": 0, "hi"')     # a torn last line
    ck.write_text("\n".join(lines) + "\n")
    out, st = plan.contract_ranges(R, checkpoint=str(ck))
    assert st == {"ranges": 3, "contracted": 0, "resumed": 3, "retried": 0}
    for b in range(B):
        acc = parts[0][b]
        for lo in (3, 6):
            acc = _combine(acc, parts[lo][b])
        got = (out[b].re, out[b].im, out[b].re_comp, out[b].im_comp)
        assert got == acc, (b, got, acc)
    # the torn line is gone, the rest kept
    kept = ck.read_text().splitlines()
    assert len(kept) == 4 and kept[0] == lines[0]


def test_checkpoint_of_another_plan_is_rejected(tmp_path):
    inst = make_instance(16, 1, 1, 6)
    plan = qtn.qtn_plan(16, inst.edges, 1, inst.gamma, inst.beta, inst.bitstrings, k=2)
    other = qtn.qtn_plan(16, inst.edges, 1, [0.1], inst.beta, inst.bitstrings, k=2)
    assert plan.fingerprint() != other.fingerprint()
    ck = tmp_path / "ck.jsonl"
    ck.write_text(_header(other, 2, 1, 2) + "\n")
    with pytest.raises(qtn.QtnError) as e:
        plan.contract_ranges(2, checkpoint=str(ck))
    assert e.value.code == qtn.QTN_EINVAL
    ck.write_text(_header(plan, 4, 1, 2) + "\n")      # another range size
    with pytest.raises(qtn.QtnError):
        plan.contract_ranges(2, checkpoint=str(ck))


def _key(out):
    return [(p.re, p.im, p.re_comp, p.im_comp) for p in out]


@pytest.mark.gpu
def test_lost_range_reissued_bitwise():
    """One range fails once (forced from the host); re-issued after the pass,
    the combined partials equal the undisturbed run bit for bit, and equal the
    ordered combination of per-range qtn_contract calls."""
    torch = pytest.importorskip("torch")
    inst = workload_instance("qaoa_n40_p2_b32_k8", seed=1)
    plan = plan_instance(inst, k=8, precision="fp32")
    plan.bind_torch(64)
    stream = torch.cuda.current_stream().cuda_stream
    ref, st0 = plan.contract_ranges(64, stream=stream)
    assert st0 == {"ranges": 4, "contracted": 4, "resumed": 0, "retried": 0}
    manual = plan.contract(0, 64, stream)
    for lo in (64, 128, 192):
        nxt = plan.contract(lo, lo + 64, stream)
        manual = [qtn.qtn_partial_combine(a, b) for a, b in zip(manual, nxt)]
    assert _key(manual) == _key(ref)
    plan.inject_faults(128, 1)
    got, st = plan.contract_ranges(64, max_retries=1, stream=stream)
    assert st == {"ranges": 4, "contracted": 4, "resumed": 0, "retried": 1}
    assert _key(got) == _key(ref)
    plan.inject_faults(64, 1)
    with pytest.raises(qtn.QtnError) as e:
        plan.contract_ranges(64, max_retries=0, stream=stream)
    assert e.value.code == qtn.QTN_EHIP


@pytest.mark.gpu
def test_checkpoint_resume_bitwise(tmp_path):
    """A run that loses one range for good leaves the other ranges in the
    checkpoint; the resumed run contracts only the missing range and gives
    the undisturbed result bit for bit."""
    torch = pytest.importorskip("torch")
    inst = workload_instance("qaoa_n40_p2_b32_k8", seed=1)
    plan = plan_instance(inst, k=8, precision="fp32")
    plan.bind_torch(64)
    stream = torch.cuda.current_stream().cuda_stream
    ref, _ = plan.contract_ranges(64, stream=stream)
    ck = tmp_path / "ck.jsonl"
    plan.inject_faults(128, 5)
    with pytest.raises(qtn.QtnError):
        plan.contract_ranges(64, max_retries=1, checkpoint=str(ck), stream=stream)
    assert len(ck.read_text().splitlines()) == 1 + 3
    plan.inject_faults(128, 0)
    got, st = plan.contract_ranges(64, checkpoint=str(ck), stream=stream)
    assert st == {"ranges": 4, "contracted": 1, "resumed": 3, "retried": 0}
    assert _key(got) == _key(ref)
    again, st2 = plan.contract_ranges(64, checkpoint=str(ck), stream=stream)
    assert st2["contracted"] == 0 and _key(again) == _key(ref)
