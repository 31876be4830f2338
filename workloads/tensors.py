"""Seeded random two-site inputs for the fixed-shape contraction benchmark.

A and B are normalised complex tensors of shape (chi, 2, chi) stored as
planar FP32 ([2 (re, im)][rows][cols]) with A's rows (a, i) and columns c,
and B's rows c and columns (j, b); the gate is a Haar-random 4x4 unitary
(QR of a complex Gaussian matrix with the phases of R's diagonal divided
out) or a named Clifford.
"""
from __future__ import annotations

import numpy as np

CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)


def haar_unitary(rng: np.random.Generator, d: int = 4) -> np.ndarray:
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def random_twosite(chi: int, batch: int, seed: int, gate: str = "haar"):
    """Returns (A, B, G, Ac, Bc): planar float32 arrays of shapes
    [batch, 2, 2chi, chi] and [batch, 2, chi, 2chi], the gate as 32 float32
    (re, im) values row-major, and the complex128 copies of A and B."""
    rng = np.random.default_rng(seed)
    Ac = (rng.standard_normal((batch, 2 * chi, chi)) +
          1j * rng.standard_normal((batch, 2 * chi, chi)))
    Bc = (rng.standard_normal((batch, chi, 2 * chi)) +
          1j * rng.standard_normal((batch, chi, 2 * chi)))
    Ac /= np.linalg.norm(Ac.reshape(batch, -1), axis=1)[:, None, None]
    Bc /= np.linalg.norm(Bc.reshape(batch, -1), axis=1)[:, None, None]
    # round to FP32 so every consumer sees the same inputs
    A = np.stack([Ac.real, Ac.imag], axis=1).astype(np.float32)
    B = np.stack([Bc.real, Bc.imag], axis=1).astype(np.float32)
    Ac = A[:, 0].astype(np.float64) + 1j * A[:, 1].astype(np.float64)
    Bc = B[:, 0].astype(np.float64) + 1j * B[:, 1].astype(np.float64)
    Gc = haar_unitary(rng) if gate == "haar" else CNOT
    G = np.stack([Gc.real, Gc.imag], axis=-1).astype(np.float32).reshape(-1)
    return A, B, G, Ac, Bc, Gc
