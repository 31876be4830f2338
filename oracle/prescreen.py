"""Offline screening by stabiliser propagation (Section 4.2), oracle form.

The non-Clifford gates of these circuits are diagonal, so a Pauli with only
I or Z on their support commutes through them.  Starting from |0>^n the
oracle tracks a set of independent stabiliser generators of the noiseless
state through the circuit:

* a Clifford gate conjugates every generator;
* a diagonal non-Clifford gate (T, T^dagger, CS, CS^dagger, CCZ) keeps the
  largest subgroup without X/Y on its support (GF(2) elimination, one qubit
  of the support at a time: one generator with X on q becomes the pivot, is
  multiplied into every other generator with X on q, and is dropped);
* a Z measurement is *decided* if Z_q lies in the tracked group; otherwise
  it is undecided and, since only its expected outcome is ever accepted,
  +Z_q joins the group after the standard measurement update.

Pauli noise only changes generator signs (Section 4.2).  Each generator
therefore carries a GF(2) vector over "basis faults" (channel c, component
X_a, Z_a, X_b, Z_b, X_c, Z_c): bit b is set iff basis fault b anticommutes with the
generator at the time it is injected.  Products of generators XOR these
vectors.  A decided measurement's flip vector is the XOR over the
generators whose product is Z_q; a shot is discarded iff, for some decided
measurement, the parity of (its flip vector AND the shot's basis faults) is
odd.  The rule has no false discards: a discarded shot has P_acc = 0.
"""
from __future__ import annotations

# basis faults per channel: X and Z on each of up to three qubits
NCOMP = 6


class Tableau:
    def __init__(self, n: int):
        self.n = n
        # generators: [x(int bitmask), z(int bitmask), flip(int bitmask)]
        self.g = [[0, 1 << q, 0] for q in range(n)]

    # --- Clifford conjugation (signs are noiseless constants, ignored) ------
    def h(self, q):
        for g in self.g:
            xb, zb = g[0] >> q & 1, g[1] >> q & 1
            if xb != zb:
                g[0] ^= 1 << q
                g[1] ^= 1 << q

    def s(self, q):
        for g in self.g:
            if g[0] >> q & 1:
                g[1] ^= 1 << q

    def cx(self, c, t):
        for g in self.g:
            if g[0] >> c & 1:
                g[0] ^= 1 << t
            if g[1] >> t & 1:
                g[1] ^= 1 << c

    def cz(self, a, b):
        for g in self.g:
            if g[0] >> b & 1:
                g[1] ^= 1 << a
            if g[0] >> a & 1:
                g[1] ^= 1 << b

    def drop_x(self, q):
        """Keep the maximal subgroup with no X/Y on qubit q."""
        hits = [i for i, g in enumerate(self.g) if g[0] >> q & 1]
        if not hits:
            return
        p = hits[0]
        gp = self.g[p]
        for i in hits[1:]:
            g = self.g[i]
            g[0] ^= gp[0]
            g[1] ^= gp[1]
            g[2] ^= gp[2]
        del self.g[p]

    def inject(self, q, xb, zb, bit):
        """Basis fault (Pauli on q with bits xb, zb) flips anticommuting
        generators."""
        for g in self.g:
            anti = (xb and (g[1] >> q & 1)) ^ (zb and (g[0] >> q & 1))
            if anti:
                g[2] ^= bit

    def express(self, x, z):
        """Return the flip vector of the product of generators equal to the
        Pauli (x, z) (up to sign), or None if it is not in the group."""
        rows = [(g[0], g[1], g[2]) for g in self.g]
        tx, tz, tf = x, z, 0
        # Gaussian elimination over the symplectic bits
        basis = []          # (pivot_bit, x, z, f)
        for gx, gz, gf in rows:
            v = (gx << self.n) | gz
            for pb, bv, bf in basis:
                if v >> pb & 1:
                    v ^= bv
                    gf ^= bf
            if v:
                pb = v.bit_length() - 1
                # keep basis reduced on the new pivot
                nb = []
                for opb, obv, obf in basis:
                    if obv >> pb & 1:
                        obv ^= v
                        obf ^= gf
                    nb.append((opb, obv, obf))
                basis = nb + [(pb, v, gf)]
        t = (tx << self.n) | tz
        for pb, bv, bf in basis:
            if t >> pb & 1:
                t ^= bv
                tf ^= bf
        return tf if t == 0 else None

    def measure_undecided(self, q):
        hits = [i for i, g in enumerate(self.g) if g[0] >> q & 1]
        nondet = bool(hits)
        if hits:
            p = hits[0]
            gp = self.g[p]
            for i in hits[1:]:
                g = self.g[i]
                g[0] ^= gp[0]
                g[1] ^= gp[1]
                g[2] ^= gp[2]
            del self.g[p]
        self.g.append([0, 1 << q, 0])
        return nondet


def analyse(circ):
    """Run the tracked-group propagation once.

    Returns (decided, flips): ``decided[m]`` is True for decided
    measurements and ``flips[m]`` their basis-fault flip vector (Python int,
    bit NCOMP*c + k for channel c and component k in X_a, Z_a, X_b, Z_b,
    X_c, Z_c)."""
    tab = Tableau(circ.n)
    decided = [False] * circ.n_meas
    flips = [0] * circ.n_meas
    for op in circ.ops:
        kind = op[0]
        if kind == "g1":
            name, q = op[1], op[2]
            if name == "H":
                tab.h(q)
            elif name in ("S", "SDG"):
                tab.s(q)
            elif name in ("T", "TDG"):
                tab.drop_x(q)
            # X, Y, Z only change signs: noiseless constants
        elif kind == "g2":
            if op[1] == "CX":
                tab.cx(op[2], op[3])
            elif op[1] == "CZ":
                tab.cz(op[2], op[3])
            else:                               # CS, CS^dagger: diagonal
                tab.drop_x(op[2])
                tab.drop_x(op[3])
        elif kind == "g3":                      # CCZ: diagonal
            for q in op[2:5]:
                tab.drop_x(q)
        elif kind == "ch":
            c, qs = op[2], op[3]
            base = NCOMP * c
            for j, q in enumerate(qs):
                tab.inject(q, 1, 0, 1 << (base + 2 * j))
                tab.inject(q, 0, 1, 1 << (base + 2 * j + 1))
        elif kind == "m":
            q, mi = op[1], op[2]
            f = tab.express(0, 1 << q)
            if f is not None:
                decided[mi] = True
                flips[mi] = f
            else:
                tab.measure_undecided(q)
        # reset after a measurement: the qubit already carries +-Z_q
    return decided, flips


def fault_vector(faults: dict) -> int:
    """Basis-fault bitmask of a shot {channel: 6-bit Pauli code}."""
    v = 0
    for c, code in faults.items():
        for k in range(NCOMP):
            if code >> k & 1:
                v |= 1 << (NCOMP * c + k)
    return v


def discard(decided, flips, faults: dict) -> bool:
    v = fault_vector(faults)
    for d, f in zip(decided, flips):
        if d and bin(f & v).count("1") & 1:
            return True
    return False


def signature_table(circ, decided, flips):
    """The oracle's own per-basis-fault signatures, derived from its flip
    vectors: sig[NCOMP c + k] has bit d set iff basis fault (c, k) flips the
    d-th decided measurement.  Returned as a uint64 array [NCOMP M, W]."""
    import numpy as np
    dlist = [m for m, d in enumerate(decided) if d]
    W = max(1, (len(dlist) + 63) // 64)
    sig = np.zeros((NCOMP * circ.n_channels, W), dtype=np.uint64)
    for d, m in enumerate(dlist):
        f = flips[m]
        while f:
            b = (f & -f).bit_length() - 1
            f &= f - 1
            sig[b, d >> 6] |= np.uint64(1) << np.uint64(d & 63)
    return sig


def discard_csr(sig, off, chan, pauli, chunk: int = 1 << 20):
    """Vectorised discard decisions for a CSR shot list: a shot's signature
    is the XOR of its faults' signatures (each the XOR of its basis
    components); processed in chunks of shots."""
    import numpy as np
    n = len(off) - 1
    out = np.zeros(n, dtype=bool)
    W = sig.shape[1]
    for s0 in range(0, n, chunk):
        s1 = min(n, s0 + chunk)
        f0, f1 = int(off[s0]), int(off[s1])
        if f1 == f0:
            continue
        ch = chan[f0:f1].astype(np.int64)
        pa = pauli[f0:f1]
        fs = np.zeros((f1 - f0, W), dtype=np.uint64)
        for k in range(NCOMP):
            on = ((pa >> k) & 1).astype(bool)
            fs[on] ^= sig[NCOMP * ch[on] + k]
        starts = off[s0:s1] - f0
        cnt = np.diff(off[s0:s1 + 1])
        nz = cnt > 0
        red = np.bitwise_xor.reduceat(fs, starts[nz], axis=0)
        acc = np.zeros((s1 - s0, W), dtype=np.uint64)
        acc[nz] = red
        out[s0:s1] = acc.any(axis=1)
    return out
