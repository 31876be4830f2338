"""Pins of the oracle's CAMPS (oracle/camps.py) against what the mathematics
fixes: the symplectic group of two qubits and its classes under local
Cliffords, the candidate unitaries' Pauli maps, the CS network, exactness
(P_acc, infidelity and rejection equal the state vector's on sampled
shots), a Clifford circuit keeping the residual a product state, and the
frame absorbing Clifford entanglement that a plain MPS has to carry.
"""
import numpy as np
import pytest

from oracle import camps
from oracle import mps as omps
from oracle import sampler as osamp
from oracle import statevector as sv
from oracle.gates import G1
from oracle.ir import parse
from workloads.circuits import config_circuit


def test_symplectic_classes():
    grp = camps.symplectic_group()
    assert len(grp) == 720                                 # |Sp(4, 2)|
    reps = camps.candidate_classes()
    assert len(reps) == 19 and reps == sorted(reps)        # 20 classes minus the local one
    cx = np.array([[1, 0, 0, 0], [0, 1, 0, 1], [1, 0, 1, 0], [0, 0, 0, 1]])
    assert camps._sym_ok(cx)
    # every class has 36 members; the CNOT's class is a candidate
    locs = []
    for a in camps._sl2():
        for b in camps._sl2():
            L = np.zeros((4, 4), dtype=np.int64)
            L[:2, :2], L[2:, 2:] = a, b
            locs.append(L)
    assert len(locs) == 36
    assert min(camps._code((L @ cx) % 2) for L in locs) in reps


@pytest.mark.parametrize("i", range(19))
def test_candidate_unitaries_realise_their_pauli_maps(i):
    code = camps.candidate_classes()[i]
    S = camps._from_code(code)
    D = camps.clifford_of(code)
    assert np.allclose(D.conj().T @ D, np.eye(4), atol=1e-12)
    basis = [np.kron(camps.X, np.eye(2)), np.kron(camps.Z, np.eye(2)),
             np.kron(np.eye(2), camps.X), np.kron(np.eye(2), camps.Z)]
    for c, P in enumerate(basis):
        assert np.allclose(D @ P @ D.conj().T, camps.pauli_q(S[:, c]), atol=1e-12)


def test_cs_network():
    circ = parse("QUBITS 2\nCS 0 1\n")
    ops = camps._expand(circ)
    U = np.eye(4, dtype=complex)
    for op in ops:
        if op[0] == "g1":
            g = np.kron(G1[op[1]], np.eye(2)) if op[2] == 0 else np.kron(np.eye(2), G1[op[1]])
        else:
            g = camps.CX4
        U = g @ U
    assert np.allclose(U, np.diag([1, 1, 1, 1j]), atol=1e-12)


@pytest.mark.parametrize("name", ["tiny", "tiny_ghz"])
def test_camps_equals_state_vector(name):
    circ = parse(config_circuit(name).text)
    off, ch, pa = osamp.sample_csr(circ, 0x5EED0061, 0, 8, weights=[0, 1, 2, 3] * 2)
    for f in osamp.csr_to_dicts(off, ch, pa):
        a = camps.run_shot(circ, f)
        b = sv.run_shot(circ, f)
        assert a.rejected_at == b.rejected_at
        assert abs(a.p_acc - b.p_acc) < 1e-10
        if b.p_acc > 0:
            assert abs(a.infid - b.infid) < 1e-10


def test_accepted_faulty_shot_equals_state_vector():
    # a shot that survives with a non-trivial branch probability
    circ = parse(config_circuit("tiny_ghz").text)
    off, ch, pa = osamp.sample_csr(circ, 7, 0, 12, weights=[1, 2, 3] * 4)
    shots = osamp.csr_to_dicts(off, ch, pa)
    hit = 0
    for f in shots:
        b = sv.run_shot(circ, f)
        if b.p_acc > 0:
            a = camps.run_shot(circ, f)
            assert abs(a.p_acc - b.p_acc) < 1e-10 and abs(a.infid - b.infid) < 1e-10
            hit += 1
    assert hit >= 1


def test_clifford_circuit_keeps_a_product_residual():
    circ = parse(config_circuit("tiny", target="S").text)
    off, ch, pa = osamp.sample_csr(circ, 9, 0, 6, weights=[0, 1, 2] * 2)
    for f in osamp.csr_to_dicts(off, ch, pa):
        assert camps.run_shot(circ, f).chi_peak == 1


def test_frame_absorbs_clifford_entanglement():
    text = "QUBITS 3\nSEED 0\nH 0\nCX 0 1\nCX 1 2\nT 0\nT 2\n"
    circ = parse(text)
    a = camps.run_shot(circ, {})
    b = omps.run_shot(circ, {})
    assert b.chi_peak == 2 and a.chi_peak == 1
    # and the noiseless cultivation-like circuit needs a smaller residual
    for name in ("tiny", "tiny_ghz"):
        c = parse(config_circuit(name).text)
        assert camps.run_shot(c, {}).chi_peak < omps.run_shot(c, {}).chi_peak
