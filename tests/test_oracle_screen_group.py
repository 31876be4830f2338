"""Pins of the offline screen's group rule (Section 4.2) by brute force.

The oracle's tableau keeps a list of generators and, at a diagonal
non-Clifford (T, T^dagger, CS, CS^dagger, CCZ), eliminates the X/Y
components on the gate's support by GF(2) pivoting.  The rule it implements
is "keep every element of the stabiliser group that commutes with the
gate", i.e. the largest subgroup with only I or Z on the support.  Here that
subgroup is formed literally: every element of the group (at most 2^7 on
these circuits) is held explicitly with its flip vector over the basis
faults, a Clifford maps each element, a diagonal gate keeps exactly the
elements without X on its support, a fault flips the elements it
anticommutes with, and an undecided Z measurement keeps the elements that
commute with Z_q and multiplies them by {I, +Z_q}.  A measurement is decided
iff Z_q is an element.  Decided sets and flip vectors must equal the
tableau's exactly; a tableau that dropped more than the maximal subgroup
(for example every generator with X on the support) decides fewer
measurements and fails the comparison, which the last test demonstrates.
"""
import random

import pytest

from oracle import prescreen as ops
from oracle.ir import parse
from workloads.circuits import config_circuit


def _bit(v, q):
    return (v >> q) & 1


def brute_force_screen(circ):
    """Decided flags and flip vectors from the explicit group."""
    n = circ.n
    # the group of |0...0>: every product of Z's, no flips
    group = {(0, s): 0 for s in range(1 << n)}
    decided = [False] * circ.n_meas
    flips = [0] * circ.n_meas

    def remap(fn):
        nonlocal group
        new = {}
        for (x, z), f in group.items():
            new[fn(x, z)] = f
        assert len(new) == len(group)
        group = new

    def keep(pred):
        nonlocal group
        group = {k: f for k, f in group.items() if pred(*k)}

    for op in circ.ops:
        kind = op[0]
        if kind == "g1":
            name, q = op[1], op[2]
            if name == "H":
                def h(x, z, q=q):
                    bx, bz = _bit(x, q), _bit(z, q)
                    x = (x & ~(1 << q)) | (bz << q)
                    z = (z & ~(1 << q)) | (bx << q)
                    return x, z
                remap(h)
            elif name in ("S", "SDG"):
                remap(lambda x, z, q=q: (x, z ^ (_bit(x, q) << q)))
            elif name in ("T", "TDG"):
                keep(lambda x, z, q=q: not _bit(x, q))
        elif kind == "g2":
            name, a, b = op[1], op[2], op[3]
            if name == "CX":
                remap(lambda x, z, a=a, b=b: (x ^ (_bit(x, a) << b), z ^ (_bit(z, b) << a)))
            elif name == "CZ":
                remap(lambda x, z, a=a, b=b: (x, z ^ (_bit(x, b) << a) ^ (_bit(x, a) << b)))
            else:                                   # CS, CS^dagger
                keep(lambda x, z, a=a, b=b: not (_bit(x, a) or _bit(x, b)))
        elif kind == "g3":                          # CCZ
            qs = op[2:5]
            keep(lambda x, z, qs=qs: not any(_bit(x, q) for q in qs))
        elif kind == "ch":
            c, qs = op[2], op[3]
            for j, q in enumerate(qs):
                bx = 1 << (ops.NCOMP * c + 2 * j)       # X on q flips elements with Z/Y on q
                bz = 1 << (ops.NCOMP * c + 2 * j + 1)   # Z on q flips elements with X/Y on q
                group = {(x, z): f ^ (bx if _bit(z, q) else 0) ^ (bz if _bit(x, q) else 0)
                         for (x, z), f in group.items()}
        elif kind == "m":
            q, mi = op[1], op[2]
            key = (0, 1 << q)
            if key in group:
                decided[mi] = True
                flips[mi] = group[key]
            else:
                kept = {k: f for k, f in group.items() if not _bit(k[0], q)}
                group = dict(kept)
                for (x, z), f in kept.items():
                    group[(x, z ^ (1 << q))] = f
    return decided, flips


GATES1 = ["H", "S", "SDG", "T", "TDG", "X", "Z"]


def random_screen_circuit(n, rounds, rng):
    """A random circuit over the screen's gate set: rounds of Hadamards,
    entangling Cliffords, diagonal non-Cliffords, channels of every kind and
    mid-circuit measurements with resets."""
    lines = [f"QUBITS {n}"]

    def pick(k):
        return rng.sample(range(n), k)

    for _ in range(rounds):
        for q in range(n):
            if rng.random() < 0.5:
                lines.append(f"H {q}")
        for _ in range(rng.randrange(3, 9)):
            a, b = pick(2)
            lines.append(f"{rng.choice(['CX', 'CX', 'CZ'])} {a} {b}")
            if rng.random() < 0.3:
                lines.append(f"{rng.choice(['S', 'SDG', 'X', 'Z'])} {a}")
        for _ in range(rng.randrange(1, 4)):
            r = rng.random()
            if r < 0.4:
                lines.append(f"{rng.choice(['T', 'TDG'])} {rng.randrange(n)}")
            elif r < 0.75 or n < 3:
                a, b = pick(2)
                lines.append(f"{rng.choice(['CS', 'CSDG'])} {a} {b}")
            else:
                a, b, c = pick(3)
                lines.append(f"CCZ {a} {b} {c}")
        for _ in range(rng.randrange(1, 4)):
            r = rng.random()
            if r < 0.4:
                lines.append(f"DEP1 {rng.randrange(n)}")
            elif r < 0.7:
                a, b = pick(2)
                lines.append(f"DEP2 {a} {b}")
            elif r < 0.85 and n >= 3:
                a, b, c = pick(3)
                lines.append(f"DEP3 {a} {b} {c}")
            else:
                lines.append(f"XERR {rng.randrange(n)}")
        for q in pick(rng.randrange(1, 3)):
            if rng.random() < 0.5:
                lines.append(f"H {q}")
            lines.append(f"M {q}")
            if rng.random() < 0.5:
                lines.append(f"R {q}")
    for q in range(n):
        lines.append(f"M {q}")
    return "\n".join(lines) + "\n"


def _circuits():
    out = []
    for name in ("tiny", "tiny_ghz"):
        for tg in ("T", "S"):
            out.append((f"{name}-{tg}", config_circuit(name, tg).text))
    rng = random.Random(0x5C4EE)
    for i in range(80):
        n = rng.choice([4, 5, 6, 7])
        out.append((f"random{i}", random_screen_circuit(n, rng.randrange(2, 6), rng)))
    return out


CIRCUITS = _circuits()


@pytest.mark.parametrize("name,text", CIRCUITS, ids=[c[0] for c in CIRCUITS])
def test_screen_equals_explicit_group(name, text):
    c = parse(text)
    assert c.n <= 7
    dec, fl = ops.analyse(c)
    bdec, bfl = brute_force_screen(c)
    assert dec == bdec
    for m in range(c.n_meas):
        if dec[m]:
            assert fl[m] == bfl[m], m


def test_random_circuits_exercise_the_elimination():
    # the comparison above only pins maximality where a diagonal gate meets
    # several generators with X on its support, and decided measurements
    # after it: count both
    multi = 0
    decided_after = 0
    orig = ops.Tableau.drop_x

    def counting(self, q):
        nonlocal multi
        if sum(1 for g in self.g if g[0] >> q & 1) >= 2:
            multi += 1
        return orig(self, q)

    ops.Tableau.drop_x = counting
    try:
        for name, text in CIRCUITS:
            c = parse(text)
            dec, _ = ops.analyse(c)
            decided_after += sum(dec)
    finally:
        ops.Tableau.drop_x = orig
    assert multi >= 80
    assert decided_after >= 200


def test_generator_wise_dropping_is_caught():
    # plant the plausible mistake in the oracle (on the CPU): drop every
    # generator with X on the qubit instead of keeping the products of
    # pairs of them; some decided set must then differ from the explicit
    # group's
    def generator_wise(self, q):
        self.g = [g for g in self.g if not (g[0] >> q & 1)]

    orig = ops.Tableau.drop_x
    ops.Tableau.drop_x = generator_wise
    try:
        differ = 0
        for name, text in CIRCUITS:
            c = parse(text)
            dec, _ = ops.analyse(c)
            bdec, _ = brute_force_screen(c)
            differ += dec != bdec
    finally:
        ops.Tableau.drop_x = orig
    assert differ >= 10
