"""Clifford-augmented MPS (CAMPS) simulation of one shot, oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written from the
section "Clifford augmented MPS": the state is C|m> with C a Clifford frame
and |m> the magic residual; Clifford operations go into the frame; a
non-Clifford gate or a projector is a sum of Pauli strings, which are
propagated through the frame and applied to the residual; a greedy
disentangler then sweeps nearest-neighbour bonds for entanglement-lowering
two-qubit Cliffords and moves them into the frame.

Dense form for small circuits, so that every step is its definition: the
frame is a 2^n x 2^n unitary and the residual a 2^n vector, tensor factor i
being MPS site i (qubit q sits on site site_of[q] of the circuit's order).

* Clifford gate G (H S SDG X Y Z CX CZ, and SWAP-free: the layout is fixed):
  C <- G C.  Pauli fault F: C <- F C.  Reset after a measurement with
  outcome e: C <- X_q^e C.
* T^(+-1) on q: R = C^dag Z_q C, |m> <- (cos(pi/8) I -+ i sin(pi/8) R)|m>
  (T = e^(i pi/8) exp(-i pi/8 Z); global phases dropped).  CS, CS^dag and
  CCZ are first written over T, T^dag and CX (textbook networks).
* measurement of q with expected outcome e: R as above,
  p = (1 + (-1)^e <m|R|m>)/2, rejected if p < tau_rej, else
  |m> <- (I + (-1)^e R)|m> / (2 sqrt p) and P_acc *= p.
* after every rotation or projection that changed |m> and whose string R
  acts on two sites or more, one greedy sweep over the bonds
  k = max(lo - 1, 0) .. min(hi, n - 2), lo and hi the first and last site
  where R acts: for every candidate D below, the purity
  tr(rho^2) of D_(k,k+1)|m> across bond k; the best candidate, if it beats
  the current purity by more than a relative 1e-9 (the earlier candidate
  wins among equals), is applied: |m> <- D|m>, C <- C D^dag.
* the seed's Bloch vector <m|C^dag sigma C|m> gives f.

Candidates.  Two-qubit Cliffords modulo Paulis are the symplectic matrices
S over GF(2) acting on (x1, z1, x2, z2) (720 of them).  D|m> has the same
entanglement across the bond for every member of a class
{(L1 + L2) S : L1, L2 in SL(2, 2)} (local Cliffords after D), 20 classes.
A class is represented by its member with the smallest code
sum_{r,c} S[r][c] 2^(4r+c); the classes are ordered by that code and the
one of the identity is left out (19 candidates).  D for S: the Clifford
with D P D^dag = Q(S v_P) for P = X1, Z1, X2, Z2, where
Q(v) = i^(x1 z1 + x2 z2) X^x1 Z^z1 (x) X^x2 Z^z2 (Hermitian); fixed up to a
phase by D|00> = normalised (I + Q_Z1)(I + Q_Z2)|w> (|w> the first of |00>,
|01>, |10>, |11> giving a nonzero vector, rotated so that its first nonzero
amplitude is real positive) and D|ab> = Q_X1^a Q_X2^b D|00>, with qubit 1
the left site (high bit).

Bond dimension: the Schmidt rank of |m> at each bond (sigma > 1e-12
sigma_0), recorded after each operator's application and after each
disentangler step; chi_peak is their maximum.
"""
from __future__ import annotations

import math

import numpy as np

from .gates import G1, ccz_sequence, fault_paulis, target_state

I2 = np.eye(2, dtype=complex)
X = np.array([[0, 1], [1, 0]], dtype=complex)
Z = np.array([[1, 0], [0, -1]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
CX4 = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)
CZ4 = np.diag([1, 1, 1, -1]).astype(complex)


# ------------------------------------------------------------ candidates
def _sym_ok(S):
    # S^T Omega S = Omega, Omega pairing (x1, z1) and (x2, z2)
    Om = np.array([[0, 1, 0, 0], [1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.int64)
    return np.array_equal((S.T @ Om @ S) % 2, Om)


def _code(S) -> int:
    return int(sum(int(S[r, c]) << (4 * r + c) for r in range(4) for c in range(4)))


def _from_code(code: int):
    return np.array([[(code >> (4 * r + c)) & 1 for c in range(4)] for r in range(4)],
                    dtype=np.int64)


def symplectic_group():
    return [_from_code(k) for k in range(1 << 16) if _sym_ok(_from_code(k))]


def _sl2():
    out = []
    for k in range(16):
        m = np.array([[(k >> 0) & 1, (k >> 1) & 1], [(k >> 2) & 1, (k >> 3) & 1]], dtype=np.int64)
        if (m[0, 0] * m[1, 1] - m[0, 1] * m[1, 0]) % 2 == 1:
            out.append(m)
    return out


def candidate_classes():
    """Codes of the 19 candidate class representatives, in order."""
    locs = []
    for a in _sl2():
        for b in _sl2():
            L = np.zeros((4, 4), dtype=np.int64)
            L[:2, :2] = a
            L[2:, 2:] = b
            locs.append(L)
    reps = set()
    for S in symplectic_group():
        reps.add(min(_code((L @ S) % 2) for L in locs))
    ident_rep = min(_code(L) for L in locs)
    return sorted(r for r in reps if r != ident_rep)


def pauli_q(v) -> np.ndarray:
    """Q(v) = i^(x1 z1 + x2 z2) X^x1 Z^z1 (x) X^x2 Z^z2."""
    x1, z1, x2, z2 = (int(t) for t in v)
    a = np.linalg.matrix_power(X, x1) @ np.linalg.matrix_power(Z, z1)
    b = np.linalg.matrix_power(X, x2) @ np.linalg.matrix_power(Z, z2)
    return (1j ** (x1 * z1 + x2 * z2)) * np.kron(a, b)


def clifford_of(code: int) -> np.ndarray:
    S = _from_code(code)
    Q = [pauli_q(S[:, c]) for c in range(4)]      # images of X1, Z1, X2, Z2
    proj = (np.eye(4) + Q[1]) @ (np.eye(4) + Q[3])
    v00 = None
    for w in range(4):
        v = proj[:, w]
        if np.linalg.norm(v) > 1e-9:
            v00 = v / np.linalg.norm(v)
            break
    j = int(np.flatnonzero(np.abs(v00) > 1e-9)[0])
    v00 = v00 * (abs(v00[j]) / v00[j])
    D = np.zeros((4, 4), dtype=complex)
    for a in (0, 1):
        for b in (0, 1):
            v = v00
            if a:
                v = Q[0] @ v
            if b:
                v = Q[2] @ v
            D[:, 2 * a + b] = v
    return D


# ------------------------------------------------------------ dense helpers
def _apply(op: np.ndarray, mat: np.ndarray, sites, n: int) -> np.ndarray:
    """op (2^k x 2^k on the given sites, first site most significant)
    applied from the left to every column of mat (2^n x cols)."""
    k = len(sites)
    cols = mat.shape[1]
    t = mat.reshape([2] * n + [cols])
    rest = [i for i in range(n) if i not in sites]
    t = np.transpose(t, list(sites) + rest + [n])
    t = t.reshape(2 ** k, -1)
    t = (op @ t).reshape([2] * k + [2] * (n - k) + [cols])
    inv = np.argsort(list(sites) + rest + [n])
    return np.transpose(t, inv).reshape(2 ** n, cols)


def _single(P: np.ndarray, site: int, n: int) -> np.ndarray:
    return _apply(P, np.eye(2 ** n, dtype=complex), [site], n)


def _support(R: np.ndarray, n: int):
    """Sites where the Pauli string R (up to a phase) acts nontrivially."""
    out = []
    for j in range(n):
        xj, zj = _single(X, j, n), _single(Z, j, n)
        if not (np.allclose(R @ xj, xj @ R) and np.allclose(R @ zj, zj @ R)):
            out.append(j)
    return out


def _ranks(m: np.ndarray, n: int, tau: float = 1e-12):
    out = []
    for k in range(n - 1):
        s = np.linalg.svd(m.reshape(2 ** (k + 1), -1), compute_uv=False)
        out.append(int((s > tau * s[0]).sum()) if s[0] > 0 else 0)
    return out


def _purity(m: np.ndarray, k: int) -> float:
    M = m.reshape(2 ** (k + 1), -1)
    rho = M @ M.conj().T
    return float(np.sum(np.abs(rho) ** 2))


class ShotResult:
    def __init__(self, p_acc, infid, rejected_at, chi_peak):
        self.p_acc, self.infid, self.rejected_at, self.chi_peak = p_acc, infid, rejected_at, chi_peak


def _expand(circ):
    """Ops with CS, CS^dag and CCZ written over T, T^dag and CX."""
    out = []
    for op in circ.ops:
        if op[0] == "g2" and op[1] in ("CS", "CSDG"):
            a, b = op[2], op[3]
            t, td = ("T", "TDG") if op[1] == "CS" else ("TDG", "T")
            out += [("g1", t, a), ("g1", t, b), ("g2", "CX", a, b), ("g1", td, b),
                    ("g2", "CX", a, b)]
        elif op[0] == "g3":
            for g in ccz_sequence(op[2], op[3], op[4]):
                out.append(("g1", g[0], g[1]) if len(g) == 2 else ("g2", g[0], g[1], g[2]))
        else:
            out.append(op)
    return out


def run_shot(circ, faults: dict, expected=None, tau_rej: float = 1e-6) -> ShotResult:
    n = circ.n
    if n > 10:
        raise ValueError("dense CAMPS oracle limited to small circuits")
    site = [0] * n
    for s, q in enumerate(circ.order):
        site[q] = s
    N = 2 ** n
    C = np.eye(N, dtype=complex)
    m = np.zeros(N, dtype=complex)
    m[0] = 1.0
    cands = [clifford_of(c) for c in candidate_classes()]
    p_acc = 1.0
    chi_peak = 1
    last_e = [0] * n
    c8, s8 = math.cos(math.pi / 8), math.sin(math.pi / 8)

    def rot_or_proj(R, a, b):
        """|m> <- (a I + b R)|m>, then one disentangling sweep."""
        nonlocal m, C, chi_peak
        m = a * m + b * (R @ m)
        chi_peak = max(chi_peak, max(_ranks(m, n)) if n > 1 else 1)
        sup = _support(R, n)
        if len(sup) < 2:
            return                     # a one-site operator changes no bond
        for k in range(max(sup[0] - 1, 0), min(sup[-1], n - 2) + 1):
            best = _purity(m, k)
            choice = None
            for D in cands:
                pk = _purity(_apply(D, m[:, None], [k, k + 1], n)[:, 0], k)
                if pk > best * (1.0 + 1e-9):
                    best, choice = pk, D
            if choice is not None:
                m = _apply(choice, m[:, None], [k, k + 1], n)[:, 0]
                # C <- C D^dag, D^dag acting on the residual's sites k, k+1
                C = C @ _apply(choice.conj().T, np.eye(N, dtype=complex), [k, k + 1], n)
                s = np.linalg.svd(m.reshape(2 ** (k + 1), -1), compute_uv=False)
                chi_peak = max(chi_peak, int((s > 1e-12 * s[0]).sum()))

    for op in _expand(circ):
        kind = op[0]
        if kind == "g1":
            g, q = op[1], op[2]
            if g in ("T", "TDG"):
                R = C.conj().T @ _apply(Z, C, [site[q]], n)
                rot_or_proj(R, c8, (-1j if g == "T" else 1j) * s8)
            else:
                C = _apply(G1[g], C, [site[q]], n)
        elif kind == "g2":
            a, b = op[2], op[3]
            U = CX4 if op[1] == "CX" else CZ4
            C = _apply(U, C, [site[a], site[b]], n)
        elif kind == "ch":
            for q, P in fault_paulis(faults.get(op[2], 0), op[3]):
                C = _apply(P, C, [site[q]], n)
        elif kind == "m":
            q, mi = op[1], op[2]
            e = 0 if expected is None else int(expected[mi])
            R = C.conj().T @ _apply(Z, C, [site[q]], n)
            sgn = 1.0 if e == 0 else -1.0
            ev = float(np.real(np.vdot(m, R @ m)))
            pe = 0.5 * (1.0 + sgn * ev)
            if pe < tau_rej or pe <= 0.0:
                return ShotResult(0.0, 0.0, mi, chi_peak)
            p_acc *= pe
            if abs(pe - 1.0) > 1e-12:
                rot_or_proj(R, 0.5 / math.sqrt(pe), sgn * 0.5 / math.sqrt(pe))
            last_e[q] = e
        elif kind == "r":
            q = op[1]
            if last_e[q]:
                C = _apply(X, C, [site[q]], n)
                last_e[q] = 0
    s = site[circ.seed]
    bloch = []
    for P in (X, Y, Z):
        R = C.conj().T @ _apply(P, C, [s], n)
        bloch.append(float(np.real(np.vdot(m, R @ m))))
    t = target_state(circ.target)
    rt = [2 * np.real(np.conj(t[0]) * t[1]), 2 * np.imag(np.conj(t[0]) * t[1]),
          abs(t[0]) ** 2 - abs(t[1]) ** 2]
    f = 0.5 * (1.0 + sum(a * b for a, b in zip(bloch, rt)))
    return ShotResult(p_acc, max(0.0, 1.0 - f), -1, chi_peak)
