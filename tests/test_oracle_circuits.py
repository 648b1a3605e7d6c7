"""Pins of the general-circuit oracle (oracle/circuits.py): its two routes,
statevector and literal tensor network, agree; the statevector stays
normalised and matches hand-derived states; slicing wire variables sums to
the uncut contraction (Eq. (2)); and on a QAOA circuit written as gates it
reproduces the QAOA oracle's amplitude."""
import math

import numpy as np
import pytest

from instances import make_instance
from instances.circuits import cz, fsim, random_circuit
from oracle import circuits as C
from oracle import qaoa as Q

H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)


def test_statevector_hand_derived():
    # Bell state from H on qubit 0 then CNOT(0 -> 1): (|00> + |11>)/sqrt 2
    psi = C.statevector(2, [((0,), H), ((0, 1), CNOT)])
    assert np.allclose(psi, [1 / math.sqrt(2), 0, 0, 1 / math.sqrt(2)])
    # X on qubit 2 of 3: index 4
    psi = C.statevector(3, [((2,), X)])
    assert psi[4] == 1.0 and abs(np.vdot(psi, psi) - 1) < 1e-15
    # CNOT with qubit 1 as control: |q0=0, q1=1> -> |q0=1, q1=1>
    psi = C.statevector(2, [((1,), X), ((1, 0), CNOT)])
    assert psi[3] == 1.0


@pytest.mark.parametrize("n,depth,seed", [(4, 3, 0), (6, 4, 1), (8, 5, 2), (7, 6, 3)])
def test_network_matches_statevector(n, depth, seed):
    c = random_circuit(n, depth, 3, seed)
    psi = C.statevector(n, c.gates)
    assert abs(np.vdot(psi, psi) - 1.0) < 1e-12
    for b in range(3):
        x = c.bitstrings[b]
        ref = psi[sum(int(v) << i for i, v in enumerate(x))]
        got = C.amplitude_network(n, c.gates, x)
        assert abs(got - ref) <= 1e-12 * max(abs(ref), 1e-3)


def test_slicing_wire_variables():
    c = random_circuit(5, 4, 1, 4)
    x = c.bitstrings[0]
    whole = C.amplitude_network(5, c.gates, x)
    _, segs = C.network(5, c.gates, x)
    for cut in ([segs[0][1]], [segs[2][2], segs[3][1]], [segs[1][-1], segs[4][0], segs[2][1]]):
        assert abs(C.sliced_network(5, c.gates, x, cut) - whole) <= 1e-12 * max(abs(whole), 1e-3)


def test_qaoa_as_gates_matches_qaoa_oracle():
    inst = make_instance(6, 2, 2, 5)
    gates = [((q,), H) for q in range(6)]
    for l in range(2):
        g = inst.gamma[l]
        zz = np.diag([complex(math.cos(g * z), -math.sin(g * z)) for z in (1, -1, -1, 1)])
        gates += [((i, j), zz) for (i, j) in inst.edges]
        b = inst.beta[l]
        rx = np.array([[math.cos(b), -1j * math.sin(b)], [-1j * math.sin(b), math.cos(b)]])
        gates += [((q,), rx) for q in range(6)]
    for k in range(2):
        x = inst.bitstrings[k]
        ref = Q.statevector_amplitude(6, inst.edges, 2, inst.gamma, inst.beta, x)
        assert abs(C.amplitude_network(6, gates, x) - ref) <= 1e-12 * max(abs(ref), 1e-3)


def test_gate_definitions():
    U = fsim(0.3, 1.1)
    assert np.allclose(U.conj().T @ U, np.eye(4))
    assert np.allclose(cz(), np.diag([1, 1, 1, -1]))
    assert np.allclose(fsim(0.0, 0.0), np.eye(4))
