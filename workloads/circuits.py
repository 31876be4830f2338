"""Cultivation-like Clifford+T toy circuits on surface-code patches.

The paper's own circuits (unitary |T> encoding and verification, fold-
transversal H_XY checks, unitary decoding; Appendix "Circuits") are not
available, so this module writes a deterministic stand-in family with the
same stage structure (Section 2 and Appendix "Circuits"):

1. Injection + unitary encoding: the seed data qubit is prepared in |+>,
   rotated by T (or S for the |S> control), then a CSS encoder (CNOT fan-out
   over the support of X_L, then one H + CNOT fan-out per X-check row in
   reduced row echelon form) maps it onto the patch.
2. Noisy syndrome rounds: every Z check and every X check is measured with
   a fresh ancilla (reset, CNOTs, measure).  Z checks and X checks are
   extracted in separate sub-rounds so every outcome is deterministic.
3. Transversal T layers on all data qubits open a "frame"; inside the frame
   each X-check sub-round is wrapped as (frame)^-1 / X checks / frame so the
   noiseless outcomes stay deterministic while faults inside the frame are
   conjugated into non-Pauli operators (the non-Clifford content).
4. A noiseless tail: leave the frame, one noiseless round, the inverse
   encoder, a Z measurement of every non-seed data qubit, and the seed's
   logical state is compared with the target (Appendix "Post-selection and
   logical error").

Optionally (``ghz_checks``), rounds outside a frame end with GHZ-controlled
check gadgets shaped like the paper's controlled-H_XY checks (Section 2 and
Appendix "Circuits": GHZ ancillas, controlled-S on single qubits, CCZ on
qubit pairs, controlled-X): for an X check X_S the gadget measures
V X_S V^dagger = X_S with V = (S on every qubit of S) (CZ on consecutive
pairs of S), applied as controlled-V^dagger, controlled-X_S, controlled-V
with the controls spread over a GHZ(k) state.  Noiselessly the CS and CCZ
gates cancel and every GHZ outcome is 0; a fault between them is conjugated
into a non-Pauli operator, which is what the pre-screen's diagonal-gate
rule and the MPS have to handle.

Noise (Appendix "Noise model", read as in the project's design notes):
DEP1/DEP2 after every noisy 1q/2q gate, an X flip after every reset and
before every measurement; no idle noise; the noiseless tail has none.

Every noiseless measurement outcome is 0 by construction, matching the rule
that a shot is kept iff every measurement returns 0 (Section 4).
"""
from __future__ import annotations

from dataclasses import dataclass, field


# --------------------------------------------------------------------------
# patches


@dataclass
class Patch:
    d: int
    kind: str                      # "rot" | "unrot"
    data: list                     # coords of data qubits
    checks: list                   # (type 'X'|'Z', anc_coord, [data coords])
    xl: list                       # data coords of the X_L representative
    zl: list


def _gf2_rank(rows):
    rows = [r for r in rows if r]
    rank = 0
    rows = list(rows)
    for bit in range(max((r.bit_length() for r in rows), default=0)):
        piv = None
        for i in range(rank, len(rows)):
            if rows[i] >> bit & 1:
                piv = i
                break
        if piv is None:
            continue
        rows[rank], rows[piv] = rows[piv], rows[rank]
        for i in range(len(rows)):
            if i != rank and rows[i] >> bit & 1:
                rows[i] ^= rows[rank]
        rank += 1
    return rank


def rotated_patch(d: int) -> Patch:
    """Rotated surface code of distance d: d*d data + d*d-1 checks."""
    assert d >= 2
    data = [(2 * i + 1, 2 * j + 1) for j in range(d) for i in range(d)]
    dset = set(data)
    checks = []
    for j in range(d + 1):
        for i in range(d + 1):
            x, y = 2 * i, 2 * j
            typ = "X" if (i + j) % 2 == 0 else "Z"
            nb = [(x + dx, y + dy) for dx, dy in ((-1, -1), (1, -1), (-1, 1), (1, 1))
                  if (x + dx, y + dy) in dset]
            if len(nb) == 4:
                checks.append((typ, (x, y), nb))
            elif len(nb) == 2:
                top_bottom = y == 0 or y == 2 * d
                left_right = x == 0 or x == 2 * d
                if (top_bottom and typ == "X") or (left_right and typ == "Z"):
                    checks.append((typ, (x, y), nb))
    mid = 2 * (d // 2) + 1
    xl = [(mid, 2 * j + 1) for j in range(d)]          # X on a column
    zl = [(2 * i + 1, mid) for i in range(d)]          # Z on a row
    p = Patch(d, "rot", data, checks, xl, zl)
    _validate(p)
    return p


def unrotated_patch(d: int) -> Patch:
    """Unrotated (regular) surface code on a (2d-1)x(2d-1) checkerboard.

    Data at (x, y) with x + y even, checks at x + y odd: X checks on the rows
    with even y, Z checks on the rows with odd y.  d=5 gives 41 data + 40
    checks = 81 qubits on a 9x9 grid.
    """
    n = 2 * d - 1
    data = [(x, y) for y in range(n) for x in range(n) if (x + y) % 2 == 0]
    dset = set(data)
    checks = []
    for y in range(n):
        for x in range(n):
            if (x + y) % 2 == 1:
                typ = "X" if y % 2 == 0 else "Z"
                nb = [(x + dx, y + dy) for dx, dy in ((0, -1), (-1, 0), (1, 0), (0, 1))
                      if (x + dx, y + dy) in dset]
                checks.append((typ, (x, y), nb))
    mid = 2 * (d // 2)
    # X_L must commute with the Z checks (odd rows, horizontal neighbours
    # on even... ) -- pick the representative by search below.
    xl = [(mid, y) for y in range(0, n, 2)]
    zl = [(x, mid) for x in range(0, n, 2)]
    p = Patch(d, "unrot", data, checks, xl, zl)
    if not _validate(p, raise_=False):
        xl, zl = zl, xl
        p = Patch(d, "unrot", data, checks, xl, zl)
        _validate(p)
    return p


def _validate(p: Patch, raise_: bool = True) -> bool:
    idx = {q: i for i, q in enumerate(p.data)}

    def mask(qs):
        m = 0
        for q in qs:
            m |= 1 << idx[q]
        return m

    xs = [mask(nb) for t, _, nb in p.checks if t == "X"]
    zs = [mask(nb) for t, _, nb in p.checks if t == "Z"]
    xl, zl = mask(p.xl), mask(p.zl)
    ok = all(bin(a & b).count("1") % 2 == 0 for a in xs for b in zs)
    ok &= all(bin(xl & b).count("1") % 2 == 0 for b in zs)
    ok &= all(bin(zl & a).count("1") % 2 == 0 for a in xs)
    ok &= bin(xl & zl).count("1") % 2 == 1
    ok &= _gf2_rank(xs) + _gf2_rank(zs) == len(p.data) - 1
    ok &= _gf2_rank(xs + [xl]) == _gf2_rank(xs) + 1
    if raise_ and not ok:
        raise ValueError("invalid patch")
    return ok


def _rref_avoiding(rows, cols_order):
    """Reduced row echelon form of GF(2) rows, pivots taken in cols_order."""
    rows = [r for r in rows]
    pivots = []
    rank = 0
    for c in cols_order:
        piv = None
        for i in range(rank, len(rows)):
            if rows[i] >> c & 1:
                piv = i
                break
        if piv is None:
            continue
        rows[rank], rows[piv] = rows[piv], rows[rank]
        for i in range(len(rows)):
            if i != rank and rows[i] >> c & 1:
                rows[i] ^= rows[rank]
        pivots.append(c)
        rank += 1
    return rows[:rank], pivots


# --------------------------------------------------------------------------
# circuit writer


@dataclass
class Circuit:
    text: str
    n_qubits: int
    order: list                    # order[site] = qubit
    seed: int
    target: str
    n_channels: int
    n_meas: int
    coords: dict = field(default_factory=dict)   # qubit -> coord
    meta: dict = field(default_factory=dict)


class _Writer:
    def __init__(self):
        self.lines = []
        self.noisy = True
        self.n_channels = 0
        self.n_meas = 0

    def g1(self, name, q):
        self.lines.append(f"{name} {q}")
        if self.noisy:
            self.lines.append(f"DEP1 {q}")
            self.n_channels += 1

    def g2(self, name, a, b):
        self.lines.append(f"{name} {a} {b}")
        if self.noisy:
            self.lines.append(f"DEP2 {a} {b}")
            self.n_channels += 1

    def g3(self, name, a, b, c):
        self.lines.append(f"{name} {a} {b} {c}")
        if self.noisy:
            self.lines.append(f"DEP3 {a} {b} {c}")
            self.n_channels += 1

    def reset(self, q):
        self.lines.append(f"R {q}")
        if self.noisy:
            self.lines.append(f"XERR {q}")
            self.n_channels += 1

    def meas(self, q):
        if self.noisy:
            self.lines.append(f"XERR {q}")
            self.n_channels += 1
        self.lines.append(f"M {q}")
        self.n_meas += 1


_FRAME_GATES = {
    # target -> (gate that advances the frame by one layer, its inverse)
    "T": ("T", "TDG"),
    "S": ("S", "SDG"),
}


def _frame_ops(target: str, k: int, inverse: bool):
    """Gates realising (layer)^k or its inverse on one qubit."""
    fwd, inv = _FRAME_GATES[target]
    if target == "T":
        k %= 8
        if k == 0:
            return []
        if k == 2:
            return ["SDG"] if inverse else ["S"]
        if k == 4:
            return ["Z"]
        return [inv if inverse else fwd] * k
    k %= 4
    if k == 0:
        return []
    if k == 2:
        return ["Z"]
    return [inv if inverse else fwd] * k


def make_circuit(kind: str = "rot", d: int = 3, plain_rounds: int = 3,
                 t_layers: int = 1, framed_rounds: int = 1,
                 final_rounds: int = 1, target: str = "T",
                 order: str = "snake", ghz_checks: int = 0,
                 ghz_size: int = 3) -> Circuit:
    """Write one cultivation-like circuit (see the module docstring)."""
    patch = rotated_patch(d) if kind == "rot" else unrotated_patch(d)
    coords = list(patch.data) + [c[1] for c in patch.checks]
    # qubit ids in row-major coordinate order (y, then x)
    coords.sort(key=lambda c: (c[1], c[0]))
    qid = {c: i for i, c in enumerate(coords)}
    n = len(coords)
    rows = sorted({c[1] for c in coords})
    if order == "rainbow":
        # coordinate rows taken from the outside in (first, last, second,
        # second to last, ...), each left to right: a deliberately poor
        # linear order whose cuts cross the patch twice (Section 3.1, the
        # ordering problem), so the exact bond dimension grows
        nested = []
        lo, hi = 0, len(rows) - 1
        while lo <= hi:
            nested.append(rows[lo])
            lo += 1
            if lo <= hi:
                nested.append(rows[hi])
                hi -= 1
        rows = nested
    site_order = []
    for r, y in enumerate(rows):
        row = sorted((c for c in coords if c[1] == y), key=lambda c: c[0])
        if r % 2 == 1 and order == "snake":
            row = row[::-1]
        site_order.extend(qid[c] for c in row)
    site_of = {q: s for s, q in enumerate(site_order)}

    data = sorted((qid[c] for c in patch.data), key=lambda q: site_of[q])
    zchk = [(qid[a], sorted((qid[c] for c in nb), key=lambda q: site_of[q]))
            for t, a, nb in patch.checks if t == "Z"]
    xchk = [(qid[a], sorted((qid[c] for c in nb), key=lambda q: site_of[q]))
            for t, a, nb in patch.checks if t == "X"]
    zchk.sort(key=lambda c: site_of[c[0]])
    xchk.sort(key=lambda c: site_of[c[0]])

    # encoder: seed in the middle of the X_L column
    xl = [qid[c] for c in patch.xl]
    seed = xl[len(xl) // 2]
    dindex = {q: i for i, q in enumerate(data)}
    xrows = []
    for a, nb in xchk:
        m = 0
        for q in nb:
            m |= 1 << dindex[q]
        xrows.append(m)
    xl_cols = {dindex[q] for q in xl}
    cols = [dindex[q] for q in data if dindex[q] not in xl_cols]
    rref, pivots = _rref_avoiding(xrows, cols)
    assert len(pivots) == len(xrows), "X checks not independent off X_L"
    enc = []                       # encoder CNOT/H list (after seed prep)
    for q in xl:
        if q != seed:
            enc.append(("CX", seed, q))
    for row, pc in zip(rref, pivots):
        p = data[pc]
        enc.append(("H", p))
        for i in range(len(data)):
            if row >> i & 1 and i != pc:
                enc.append(("CX", p, data[i]))

    w = _Writer()
    L = w.lines
    L.append("# cultivation-like toy circuit, %s d=%d, target |%s>" % (kind, d, target))
    L.append(f"QUBITS {n}")
    L.append("ORDER " + " ".join(str(q) for q in site_order))
    L.append(f"SEED {seed}")
    L.append(f"TARGET {target}")

    # 1. injection + encoding
    w.g1("H", seed)
    w.g1("T" if target == "T" else "S", seed)
    for op in enc:
        if op[0] == "H":
            w.g1("H", op[1])
        else:
            w.g2("CX", op[1], op[2])
    first_use = set()

    ancillas = sorted([a for a, _ in zchk] + [a for a, _ in xchk], key=lambda q: site_of[q])

    def ghz_check(a0, nb):
        # GHZ(k) on the k free ancillas nearest to the check's own ancilla
        near = sorted(ancillas, key=lambda q: (abs(site_of[q] - site_of[a0]), site_of[q]))
        g = sorted(near[:ghz_size], key=lambda q: site_of[q])
        k = len(g)
        pairs = [(nb[i], nb[i + 1]) for i in range(0, len(nb) - 1, 2)]
        L.append("TICK")
        for q in g:
            w.reset(q)
        w.g1("H", g[0])
        for i in range(k - 1):
            w.g2("CX", g[i], g[i + 1])
        for j, q in enumerate(nb):                 # controlled V^dagger
            w.g2("CSDG", g[j % k], q)
        for j, (x, y) in enumerate(pairs):
            w.g3("CCZ", g[(j + 1) % k], x, y)
        for j, q in enumerate(nb):                 # controlled X_S
            w.g2("CX", g[(j + 2) % k], q)
        for j, (x, y) in enumerate(pairs):         # controlled V
            w.g3("CCZ", g[(j + 1) % k], x, y)
        for j, q in enumerate(nb):
            w.g2("CS", g[j % k], q)
        for i in reversed(range(k - 1)):
            w.g2("CX", g[i], g[i + 1])
        w.g1("H", g[0])
        for q in g:
            w.meas(q)

    def round_(frame):
        # every syndrome round is a segment of the space-time accounting
        L.append("SEGMENT")
        L.append("TICK")
        for a, nb in zchk:
            w.reset(a)
            for q in nb:
                w.g2("CX", q, a)
            w.meas(a)
        inv = _frame_ops(target, frame, True)
        fwd = _frame_ops(target, frame, False)
        for q in data:
            for g in inv:
                w.g1(g, q)
        for a, nb in xchk:
            w.reset(a)
            w.g1("H", a)
            for q in nb:
                w.g2("CX", a, q)
            w.g1("H", a)
            w.meas(a)
        for q in data:
            for g in fwd:
                w.g1(g, q)
        if frame == 0:
            for a, nb in xchk[:ghz_checks]:
                ghz_check(a, nb)

    for _ in range(plain_rounds):
        round_(0)
    frame = 0
    for _ in range(t_layers):
        L.append("SEGMENT")
        L.append("TICK")
        frame += 1
        for q in data:
            w.g1("T" if target == "T" else "S", q)
        for _ in range(framed_rounds):
            round_(frame)
    if frame:
        L.append("SEGMENT")
        L.append("TICK")
        for q in data:
            for g in _frame_ops(target, frame, True):
                w.g1(g, q)
    for _ in range(final_rounds):
        round_(0)

    # 4. noiseless tail
    w.noisy = False
    ghz_checks = 0
    round_(0)
    L.append("SEGMENT")
    L.append("TICK")
    for op in reversed(enc):
        if op[0] == "H":
            w.g1("H", op[1])
        else:
            w.g2("CX", op[1], op[2])
    for q in data:
        if q != seed:
            w.meas(q)
    text = "\n".join(L) + "\n"
    return Circuit(text=text, n_qubits=n, order=site_order, seed=seed,
                   target=target, n_channels=w.n_channels, n_meas=w.n_meas,
                   coords={qid[c]: c for c in coords},
                   meta=dict(kind=kind, d=d, plain_rounds=plain_rounds,
                             t_layers=t_layers, framed_rounds=framed_rounds,
                             final_rounds=final_rounds, ghz_checks=ghz_checks,
                             ghz_size=ghz_size))


# --------------------------------------------------------------------------
# named workloads


def config_circuit(name: str, target: str = "T") -> Circuit:
    """Circuits of the named workloads (17, 49 and 81 qubits; c3_rainbow is
    the 49-qubit circuit on the rainbow layout, which reaches bond
    dimension 128 noiselessly)."""
    if name in ("c1", "c2", "rot3"):
        return make_circuit("rot", 3, plain_rounds=3, t_layers=1,
                            framed_rounds=1, final_rounds=1, target=target)
    if name in ("c3", "rot5"):
        return make_circuit("rot", 5, plain_rounds=2, t_layers=2,
                            framed_rounds=2, final_rounds=0, target=target)
    if name in ("c3_rainbow", "rot5_rainbow"):
        return make_circuit("rot", 5, plain_rounds=2, t_layers=2,
                            framed_rounds=2, final_rounds=0, target=target,
                            order="rainbow")
    if name in ("c4", "unrot5"):
        return make_circuit("unrot", 5, plain_rounds=2, t_layers=2,
                            framed_rounds=3, final_rounds=0, target=target)
    if name == "tiny":
        return make_circuit("rot", 2, plain_rounds=1, t_layers=1,
                            framed_rounds=1, final_rounds=0, target=target)
    if name == "tiny_ghz":
        return make_circuit("rot", 2, plain_rounds=1, t_layers=1,
                            framed_rounds=1, final_rounds=0, target=target,
                            ghz_checks=1, ghz_size=2)
    if name in ("c1_ghz", "rot3_ghz"):
        return make_circuit("rot", 3, plain_rounds=2, t_layers=1,
                            framed_rounds=1, final_rounds=1, target=target,
                            ghz_checks=2, ghz_size=3)
    raise KeyError(name)
