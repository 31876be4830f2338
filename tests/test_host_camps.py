"""CPU: the library's CAMPS candidates (msc_camps_candidates) equal the
oracle's: the same 19 class representatives, the same unitaries and Pauli
maps that each unitary realises."""
import numpy as np

import paper_2609_19116_amd as msc
from oracle import camps


def _pauli(bits):
    b = [np.kron(camps.X, np.eye(2)), np.kron(camps.Z, np.eye(2)),
         np.kron(np.eye(2), camps.X), np.kron(np.eye(2), camps.Z)]
    out = np.eye(4, dtype=complex)
    for f in range(4):
        if (bits >> f) & 1:
            out = out @ b[f]
    return out


def test_candidates_equal_oracle():
    U, T = msc.camps_candidates()
    codes = camps.candidate_classes()
    assert U.shape == (19, 4, 4) and T.shape == (19, 16) and len(codes) == 19
    for c, code in enumerate(codes):
        D = camps.clifford_of(code)
        assert np.allclose(U[c], D, atol=1e-12)
        for loc in range(16):
            t = int(T[c][loc])
            img = _pauli(t & 15) * (1j ** (t >> 4))
            assert np.allclose(D @ _pauli(loc) @ D.conj().T, img, atol=1e-12)
