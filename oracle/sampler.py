"""Subset-sampling fault draws (Section 4 and Section 4.1), oracle twin.

A shot is a fault configuration: a weight w (either given per shot, or
drawn from Bin(M, p) as in Section 4.1), a uniform w-subset of the M
channels (valid because all channels share p), and for each chosen channel
a uniform non-identity Pauli: 3 choices for a 1-qubit depolarising channel,
15 for a 2-qubit one, 63 for a 3-qubit one, X only for an X-flip channel
(Section 4 and Appendix "Noise model").

Random numbers come from published generators written here from their
definitions, keyed by (seed, shot index) so any shot can be regenerated:

* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) for the 64-bit stream; the
  per-shot state is mix(seed ^ mix(shot)) with mix the SplitMix64 output
  function;
* Lemire's nearly-divisionless bounded integers (ACM TOMACS 2019);
* Floyd's algorithm for a uniform w-subset (Bentley & Floyd, CACM 1987);
* the Bin(M, p) weight by inversion of an FP64 cumulative table built with
  the ratio recurrence Bin_{w+1} = Bin_w (M-w)/(w+1) p/(1-p) starting from
  (1-p)^M by repeated squaring, compared against u = (x >> 11) 2^-53.
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


class SplitMix64:
    def __init__(self, seed: int, shot: int):
        self.s = mix64((seed & MASK) ^ mix64(shot & MASK))

    def next(self) -> int:
        self.s = (self.s + GOLDEN) & MASK
        return mix64(self.s)

    def bounded(self, n: int) -> int:
        """Uniform integer in [0, n) (Lemire)."""
        x = self.next()
        m = x * n
        lo = m & MASK
        if lo < n:
            t = ((1 << 64) - n) % n
            while lo < t:
                x = self.next()
                m = x * n
                lo = m & MASK
        return m >> 64

    def uniform01(self) -> float:
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)


def _pow_int(x: float, k: int) -> float:
    r = 1.0
    b = x
    while k:
        if k & 1:
            r *= b
        b *= b
        k >>= 1
    return r


def binomial_cdf_table(M: int, p: float) -> list:
    """FP64 cumulative Bin(M, p) table by the ratio recurrence."""
    q = 1.0 - p
    b = _pow_int(q, M)
    ratio = p / q if q > 0 else float("inf")
    cdf = []
    acc = 0.0
    for w in range(M + 1):
        acc += b
        cdf.append(acc)
        if w < M:
            b = b * (M - w) / (w + 1) * ratio
        if b == 0.0 and w > M * p:
            break
    return cdf


def draw_weight(rng: SplitMix64, cdf: list) -> int:
    u = rng.uniform01()
    for w, c in enumerate(cdf):
        if u < c:
            return w
    return len(cdf) - 1


def floyd_subset(rng: SplitMix64, M: int, w: int) -> list:
    s = set()
    for j in range(M - w, M):
        t = rng.bounded(j + 1)
        s.add(j if t in s else t)
    return sorted(s)


def sample_shot(circ, seed: int, shot: int, weight=None, cdf=None) -> dict:
    """One shot's faults as {channel: Pauli code, bits 2j, 2j+1 = x, z of qubit j}."""
    rng = SplitMix64(seed, shot)
    M = circ.n_channels
    w = weight if weight is not None else draw_weight(rng, cdf)
    w = min(w, M)
    chans = floyd_subset(rng, M, w)
    out = {}
    for c in chans:
        kind = circ.channel_kind[c]
        if kind == "XERR":
            out[c] = 1
        elif kind == "DEP1":
            out[c] = 1 + rng.bounded(3)
        elif kind == "DEP2":
            out[c] = 1 + rng.bounded(15)
        else:
            out[c] = 1 + rng.bounded(63)
    return out


def sample_csr(circ, seed: int, first_shot: int, n_shots: int,
               weights=None, p: float = 0.0):
    """CSR arrays (shot_off int64[n+1], chan int32[nnz], pauli uint8[nnz])."""
    cdf = None if weights is not None else binomial_cdf_table(circ.n_channels, p)
    off = [0]
    ch = []
    pa = []
    for i in range(n_shots):
        w = None if weights is None else int(weights[i])
        f = sample_shot(circ, seed, first_shot + i, w, cdf)
        for c in sorted(f):
            ch.append(c)
            pa.append(f[c])
        off.append(len(ch))
    return (np.array(off, dtype=np.int64), np.array(ch, dtype=np.int32),
            np.array(pa, dtype=np.uint8))


def csr_to_dicts(off, ch, pa) -> list:
    return [{int(c): int(p) for c, p in zip(ch[off[i]:off[i + 1]], pa[off[i]:off[i + 1]])}
            for i in range(len(off) - 1)]
