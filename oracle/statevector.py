"""Dense state-vector simulation of one noisy shot (complex128, N <= 20).

Definitions followed (Section 4 and Appendix "Post-selection and logical
error"):

* a shot is one fault configuration F: a Pauli inserted at each channel
  that fired;
* each measurement m is a detector post-selected on its noiseless outcome
  e_m (all 0 for the circuits here), so the kept branch is unique;
* P_acc(F) = prod_m p_m(F), the chain-rule product of the conditional
  probabilities of the expected outcomes, which equals the squared norm of
  the state with every measurement replaced by its projector;
* after the noiseless decoding the seed qubit's state rho is compared with
  the target: f = <t|rho|t>, and the shot is a logical failure iff
  1 - f > tau_f.

Online screening (Section 4.3): the shot stops at the first measurement
whose expected outcome has probability below tau_rej; P_acc is then 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .gates import G1, fault_paulis, target_state


@dataclass
class ShotResult:
    p_acc: float
    infid: float
    rejected_at: int                  # measurement index or -1
    meas_probs: list = field(default_factory=list)
    chi_peak: int = 0


def _apply1(psi: np.ndarray, u: np.ndarray, q: int, n: int) -> np.ndarray:
    v = psi.reshape(2 ** q, 2, 2 ** (n - q - 1))
    return np.einsum("ij,ajb->aib", u, v).reshape(-1)


def _cx(psi: np.ndarray, c: int, t: int, n: int) -> np.ndarray:
    v = psi.reshape((2,) * n).copy()
    idx = [slice(None)] * n
    idx[c] = 1
    sub = v[tuple(idx)]
    ax = t - (1 if t > c else 0)
    v[tuple(idx)] = np.flip(sub, axis=ax).copy()
    return v.reshape(-1)


def _phase(psi: np.ndarray, qs, ph: complex, n: int) -> np.ndarray:
    """Multiply the amplitudes with every qubit of qs equal to 1 by ph
    (CZ, CS, CS^dagger, CCZ are all of this form)."""
    v = psi.reshape((2,) * n).copy()
    idx = [slice(None)] * n
    for q in qs:
        idx[q] = 1
    v[tuple(idx)] *= ph
    return v.reshape(-1)


_PHASE = {"CZ": -1.0, "CS": 1j, "CSDG": -1j, "CCZ": -1.0}


def _apply_op(psi, op, n, faults):
    kind = op[0]
    if kind == "g1":
        return _apply1(psi, G1[op[1]], op[2], n)
    if kind == "g2":
        if op[1] == "CX":
            return _cx(psi, op[2], op[3], n)
        return _phase(psi, (op[2], op[3]), _PHASE[op[1]], n)
    if kind == "g3":
        return _phase(psi, (op[2], op[3], op[4]), _PHASE[op[1]], n)
    if kind == "ch":
        code = faults.get(op[2], 0)
        for q, P in fault_paulis(code, op[3]):
            psi = _apply1(psi, P, q, n)
        return psi
    raise ValueError(kind)


def _slice_prob(psi: np.ndarray, q: int, n: int, e: int) -> float:
    v = psi.reshape(2 ** q, 2, 2 ** (n - q - 1))
    return float(np.vdot(v[:, e, :], v[:, e, :]).real)


def run_shot(circ, faults: dict, expected=None, tau_rej: float = 1e-6,
             record: bool = False) -> ShotResult:
    """Simulate one shot.  ``faults`` maps channel index -> Pauli code
    (bits 2j, 2j+1 = x, z bits of the channel's j-th qubit).  ``expected`` maps measurement
    index -> expected outcome (default 0, the paper's acceptance rule)."""
    n = circ.n
    if n > 22:
        raise ValueError("state vector limited to small circuits")
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    p_acc = 1.0
    probs = []
    for op in circ.ops:
        kind = op[0]
        if kind in ("g1", "g2", "g3", "ch"):
            psi = _apply_op(psi, op, n, faults)
        elif kind == "m":
            q, mi = op[1], op[2]
            e = 0 if expected is None else int(expected[mi])
            pe = _slice_prob(psi, q, n, e)
            if record:
                probs.append(pe)
            if pe < tau_rej or pe <= 0.0:
                return ShotResult(0.0, 0.0, mi, probs)
            v = psi.reshape(2 ** q, 2, 2 ** (n - q - 1))
            v[:, 1 - e, :] = 0.0
            psi = (v / np.sqrt(pe)).reshape(-1)
            p_acc *= pe
        elif kind == "r":
            q = op[1]
            p1 = _slice_prob(psi, q, n, 1)
            p0 = _slice_prob(psi, q, n, 0)
            if min(p0, p1) > 1e-9:
                raise ValueError("reset of a qubit not in a Z eigenstate")
            if p1 > p0:
                psi = _apply1(psi, G1["X"], q, n)
    s = circ.seed
    v = psi.reshape(2 ** s, 2, 2 ** (n - s - 1))
    rho = np.einsum("aib,ajb->ij", v, v.conj())
    rho = rho / np.trace(rho).real
    t = target_state(circ.target)
    f = float(np.real(np.conj(t) @ rho @ t))
    return ShotResult(p_acc, max(0.0, 1.0 - f), -1, probs)


def final_state(circ, faults: dict) -> np.ndarray:
    """Unnormalised state with every measurement replaced by its projector
    onto 0 (used to pin P_acc = ||psi_F||^2 against the chain rule)."""
    n = circ.n
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    for op in circ.ops:
        kind = op[0]
        if kind in ("g1", "g2", "g3", "ch"):
            psi = _apply_op(psi, op, n, faults)
        elif kind == "m":
            q = op[1]
            v = psi.reshape(2 ** q, 2, 2 ** (n - q - 1)).copy()
            v[:, 1, :] = 0.0
            psi = v.reshape(-1)
        elif kind == "r":
            q = op[1]
            p1 = _slice_prob(psi, q, n, 1)
            p0 = _slice_prob(psi, q, n, 0)
            if p1 > p0:
                psi = _apply1(psi, G1["X"], q, n)
    return psi
