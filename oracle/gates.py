"""Gate matrices written out from their textbook definitions (complex128).

|T> = T|+> = (|0> + e^{i pi/4}|1>)/sqrt(2) is the magic state of the
Introduction; |S> = S|+> is the Clifford proxy of Section 2.
"""
import numpy as np

_r = 1.0 / np.sqrt(2.0)
_w = np.exp(1j * np.pi / 4)

G1 = {
    "H": np.array([[_r, _r], [_r, -_r]], dtype=np.complex128),
    "S": np.array([[1, 0], [0, 1j]], dtype=np.complex128),
    "SDG": np.array([[1, 0], [0, -1j]], dtype=np.complex128),
    "T": np.array([[1, 0], [0, _w]], dtype=np.complex128),
    "TDG": np.array([[1, 0], [0, np.conj(_w)]], dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
    "I": np.eye(2, dtype=np.complex128),
}

# two-qubit gates as 4x4 in the basis |a b> (a = first operand, most
# significant): CX(a -> b), CZ(a, b)
G2 = {
    "CX": np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]],
                   dtype=np.complex128),
    "CZ": np.diag([1, 1, 1, -1]).astype(np.complex128),
    "SWAP": np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]],
                     dtype=np.complex128),
    "CS": np.diag([1, 1, 1, 1j]).astype(np.complex128),
    "CSDG": np.diag([1, 1, 1, -1j]).astype(np.complex128),
}

# CCZ = diag(1, ..., 1, -1) as a Clifford+T sequence (the textbook Toffoli
# circuit with the target's Hadamards removed); the state vector applies CCZ
# from its definition, the MPS from this sequence.
def ccz_sequence(a, b, c):
    return [("CX", b, c), ("TDG", c), ("CX", a, c), ("T", c), ("CX", b, c), ("TDG", c),
            ("CX", a, c), ("T", b), ("T", c), ("CX", a, b), ("T", a), ("TDG", b),
            ("CX", a, b)]


def fault_paulis(code: int, qubits):
    """(qubit, 2x2 Pauli) pairs of a fault code: bits 2j, 2j+1 are the x, z
    bits of the channel's j-th qubit."""
    out = []
    for j, q in enumerate(qubits):
        x, z = code >> (2 * j) & 1, code >> (2 * j + 1) & 1
        if x or z:
            out.append((q, pauli_from_bits(x, z)))
    return out


def pauli_from_bits(x: int, z: int) -> np.ndarray:
    """Single-qubit Pauli with symplectic bits (x, z): X, Z or Y (x=z=1)."""
    if x and z:
        return G1["Y"]
    if x:
        return G1["X"]
    if z:
        return G1["Z"]
    return G1["I"]


def target_state(target: str) -> np.ndarray:
    plus = np.array([_r, _r], dtype=np.complex128)
    return (G1["T"] if target == "T" else G1["S"]) @ plus
