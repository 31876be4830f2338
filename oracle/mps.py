"""Plain FP64 matrix-product-state simulation of one noisy shot.

Follows Section 3.1: the state is a chain of rank-3 tensors A[k] with
shape (chi_{k-1}, 2, chi_k) in the linear order given by the circuit's
ORDER line; every bond dimension is the number of nonzero singular values
of the corresponding bipartition.  "Exact regime" (Section 5.1): after each
two-site update the SVD keeps every sigma_i > tau * sigma_0 (tau = 1e-12,
numerical zeros only) and there is no cap on chi.

Long-range two-qubit gates touch every bond in between (Section 3.1); here
they are applied by moving the first qubit next to the second with SWAP
updates, applying the gate, and moving it back.  The orthogonality centre
is moved with SVD splits and every measurement is taken with the centre on
the measured site, so p_e is the squared norm of one physical slice.

Shot semantics (P_acc chain rule, tau_rej early exit, fidelity with the
target after the noiseless decoding) are those of ``statevector``.
"""
from __future__ import annotations

import numpy as np

from .gates import G1, G2, ccz_sequence, fault_paulis, target_state
from .statevector import ShotResult


class MPS:
    def __init__(self, n: int, tau: float = 1e-12):
        self.n = n
        self.tau = tau
        self.A = []
        for _ in range(n):
            t = np.zeros((1, 2, 1), dtype=np.complex128)
            t[0, 0, 0] = 1.0
            self.A.append(t)
        self.center = 0
        self.chi_peak = 1
        self.discarded = 0.0
        self.n2q = 0

    def bonds(self):
        return [a.shape[2] for a in self.A[:-1]]

    # --- local operations -------------------------------------------------
    def apply1(self, u: np.ndarray, k: int) -> None:
        self.A[k] = np.einsum("ij,ajb->aib", u, self.A[k])

    def _split(self, theta: np.ndarray, k: int, to_right: bool) -> None:
        """SVD split of a two-site tensor (chi_l, 2, 2, chi_r) onto sites
        k, k+1, keeping singular values above tau * sigma_0."""
        cl, _, _, cr = theta.shape
        m = theta.reshape(cl * 2, 2 * cr)
        try:
            u, s, vh = np.linalg.svd(m, full_matrices=False)
        except np.linalg.LinAlgError:
            # LAPACK's divide-and-conquer driver (gesdd) can fail to converge
            # on exactly degenerate spectra; the QR-iteration driver (gesvd)
            # computes the same decomposition
            import scipy.linalg
            u, s, vh = scipy.linalg.svd(m, full_matrices=False, lapack_driver="gesvd")
        keep = int(np.sum(s > self.tau * s[0])) if s[0] > 0 else 1
        keep = max(keep, 1)
        self.discarded += float(np.sum(s[keep:] ** 2))
        u, s, vh = u[:, :keep], s[:keep], vh[:keep]
        if to_right:
            self.A[k] = u.reshape(cl, 2, keep)
            self.A[k + 1] = (s[:, None] * vh).reshape(keep, 2, cr)
            self.center = k + 1
        else:
            self.A[k] = (u * s[None, :]).reshape(cl, 2, keep)
            self.A[k + 1] = vh.reshape(keep, 2, cr)
            self.center = k
        self.chi_peak = max(self.chi_peak, keep)
        self.n2q += 1

    def move_center(self, target: int) -> None:
        while self.center < target:
            k = self.center
            th = np.einsum("aib,bjc->aijc", self.A[k], self.A[k + 1])
            self._split(th, k, True)
        while self.center > target:
            k = self.center - 1
            th = np.einsum("aib,bjc->aijc", self.A[k], self.A[k + 1])
            self._split(th, k, False)

    def apply2_adjacent(self, g: np.ndarray, k: int, to_right: bool = True) -> None:
        """Apply a 4x4 gate to sites (k, k+1); g's first operand is site k."""
        if self.center < k:
            self.move_center(k)
        elif self.center > k + 1:
            self.move_center(k + 1)
        th = np.einsum("aib,bjc->aijc", self.A[k], self.A[k + 1])
        g4 = g.reshape(2, 2, 2, 2)
        th = np.einsum("ijkl,aklc->aijc", g4, th)
        self._split(th, k, to_right)

    def prob(self, k: int, e: int) -> float:
        self.move_center(k)
        sl = self.A[k][:, e, :]
        return float(np.vdot(sl, sl).real)

    def project(self, k: int, e: int, pe: float) -> None:
        t = self.A[k].copy()
        t[:, 1 - e, :] = 0.0
        self.A[k] = t / np.sqrt(pe)

    def rho1(self, k: int) -> np.ndarray:
        self.move_center(k)
        a = self.A[k]
        rho = np.einsum("aib,ajb->ij", a, a.conj())
        return rho / np.trace(rho).real


def run_shot(circ, faults: dict, expected=None, tau_rej: float = 1e-6,
             tau: float = 1e-12, record: bool = False) -> ShotResult:
    """Simulate one shot on an FP64 MPS (same contract as the state vector)."""
    n = circ.n
    site = [0] * n
    for s, q in enumerate(circ.order):
        site[q] = s
    qubit_at = list(circ.order)
    mps = MPS(n, tau)
    p_acc = 1.0
    probs = []

    def swap_sites(k):
        mps.apply2_adjacent(G2["SWAP"], k, to_right=True)
        qa, qb = qubit_at[k], qubit_at[k + 1]
        qubit_at[k], qubit_at[k + 1] = qb, qa
        site[qa], site[qb] = k + 1, k

    def swap_sites_left(k):
        mps.apply2_adjacent(G2["SWAP"], k, to_right=False)
        qa, qb = qubit_at[k], qubit_at[k + 1]
        qubit_at[k], qubit_at[k + 1] = qb, qa
        site[qa], site[qb] = k + 1, k

    def gate2(name, a, b):
        g = G2[name]
        home = site[a]
        # bring qubit a next to qubit b
        moves = []
        while abs(site[a] - site[b]) > 1:
            if site[a] < site[b]:
                k = site[a]
                swap_sites(k)
                moves.append(("r", k))
            else:
                k = site[a] - 1
                swap_sites_left(k)
                moves.append(("l", k))
        k = min(site[a], site[b])
        if site[a] < site[b]:
            mps.apply2_adjacent(g, k)
        else:
            sw = G2["SWAP"]
            mps.apply2_adjacent(sw @ g @ sw, k)
        for d, k in reversed(moves):
            if d == "r":
                swap_sites_left(k)
            else:
                swap_sites(k)
        assert site[a] == home

    for op in circ.ops:
        kind = op[0]
        if kind == "g1":
            mps.apply1(G1[op[1]], site[op[2]])
        elif kind == "g2":
            gate2(op[1], op[2], op[3])
        elif kind == "g3":
            for g in ccz_sequence(op[2], op[3], op[4]):
                if g[0] == "CX":
                    gate2("CX", g[1], g[2])
                else:
                    mps.apply1(G1[g[0]], site[g[1]])
        elif kind == "ch":
            for q, P in fault_paulis(faults.get(op[2], 0), op[3]):
                mps.apply1(P, site[q])
        elif kind == "m":
            q, mi = op[1], op[2]
            e = 0 if expected is None else int(expected[mi])
            k = site[q]
            pe = mps.prob(k, e)
            if record:
                probs.append(pe)
            if pe < tau_rej or pe <= 0.0:
                r = ShotResult(0.0, 0.0, mi, probs)
                r.chi_peak = mps.chi_peak
                return r
            mps.project(k, e, pe)
            p_acc *= pe
        elif kind == "r":
            k = site[op[1]]
            mps.move_center(k)
            p1 = float(np.vdot(mps.A[k][:, 1, :], mps.A[k][:, 1, :]).real)
            p0 = float(np.vdot(mps.A[k][:, 0, :], mps.A[k][:, 0, :]).real)
            if min(p0, p1) > 1e-9:
                raise ValueError("reset of a qubit not in a Z eigenstate")
            if p1 > p0:
                mps.apply1(G1["X"], k)
    rho = mps.rho1(site[circ.seed])
    t = target_state(circ.target)
    f = float(np.real(np.conj(t) @ rho @ t))
    r = ShotResult(p_acc, max(0.0, 1.0 - f), -1, probs)
    r.chi_peak = mps.chi_peak
    run_shot.last = mps
    return r
