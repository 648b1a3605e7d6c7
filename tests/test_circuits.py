"""General circuits with non-diagonal two-qubit gates (qtn_plan_circuit):
the planner's network on the CPU through the exported schedule, and on the
GPU the contraction against the statevector of the circuit oracle."""
import numpy as np
import pytest

from instances.circuits import random_circuit
from oracle import circuits as C
from paper_2010_14962_amd import qtn

import schedule_interp as SI


@pytest.mark.parametrize("n,depth,seed,cz", [(6, 4, 0, False), (8, 6, 1, False), (7, 5, 2, True)])
def test_circuit_schedule_matches_statevector(n, depth, seed, cz):
    """The exported schedule of a circuit plan, executed by the test-only
    numpy interpreter, gives the statevector amplitudes (every index map and
    leaf value of the planner's circuit network checked)."""
    c = random_circuit(n, depth, 2, seed, cz_gates=cz)
    plan = qtn.qtn_plan_circuit(n, c.gates, c.bitstrings, k=2)
    k = plan.info()["k"]
    vals = SI.run(plan, range(1 << k))
    psi = C.statevector(n, c.gates)
    for b in range(2):
        ref = psi[sum(int(v) << i for i, v in enumerate(c.bitstrings[b]))]
        got = sum(vals[b])
        assert abs(got - ref) <= 1e-12 * max(abs(ref), 1e-3), (b, got, ref)


def test_circuit_input_validation():
    c = random_circuit(4, 2, 1, 0)
    with pytest.raises(qtn.QtnError):
        qtn.qtn_plan_circuit(4, [((0, 0), np.eye(4))], c.bitstrings)
    with pytest.raises(qtn.QtnError):
        qtn.qtn_plan_circuit(4, [((5,), np.eye(2))], c.bitstrings)
    with pytest.raises(qtn.QtnError):
        qtn.qtn_plan_circuit(4, c.gates, c.bitstrings, precision="3xbf16")


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n,depth,seed,k", [(12, 8, 0, 0), (16, 10, 1, 3), (20, 12, 2, 4)])
def test_random_circuits_on_gpu(precision, n, depth, seed, k):
    torch = pytest.importorskip("torch")
    print("case circuit", n, depth, k, precision, flush=True)
    stream = torch.cuda.current_stream().cuda_stream
    c = random_circuit(n, depth, 4, seed)
    plan = qtn.qtn_plan_circuit(n, c.gates, c.bitstrings, k=k, precision=precision)
    plan.bind_torch(1 << k)
    amps = [p.value() for p in plan.contract(0, 1 << k, stream)]
    psi = C.statevector(n, c.gates)
    tol = 1e-12 if precision == "fp64" else 1e-6
    for b in range(4):
        ref = psi[sum(int(v) << i for i, v in enumerate(c.bitstrings[b]))]
        den = abs(ref) if abs(ref) >= 1e-6 * 2.0 ** (-n / 2) else 2.0 ** (-n / 2)
        assert abs(amps[b] - ref) <= tol * den, (b, amps[b], ref)
