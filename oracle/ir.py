"""Oracle's own parser of the project's circuit text format.

One op per line; '#' starts a comment.  Header lines: QUBITS n, ORDER
q0 q1 ... (qubit held by each MPS site), SEED q, TARGET T|S.  Ops:
H S SDG T TDG X Y Z q | CX CZ CS CSDG a b | CCZ a b c | M q | R q | DEP1 q |
DEP2 a b | DEP3 a b c | XERR q | TICK | SEGMENT.  Channels (DEP1, DEP2, DEP3, XERR)
are numbered in text order, as are measurements.  CS/CSDG are controlled-S
and controlled-S^dagger, CCZ the doubly controlled Z: the diagonal
non-Clifford gates of the paper's checks (Section 2, Section 4.2).  The
noise semantics follow Section 4 (uniform depolarising, any of the 4^k-1
non-identity Paulis with probability p/(4^k-1)).  SEGMENT starts a new
segment of the circuit for the space-time accounting (Appendix
"Space-time overhead"); it does not act on the state.
"""
from __future__ import annotations

from dataclasses import dataclass, field

ONE_Q = {"H", "S", "SDG", "T", "TDG", "X", "Y", "Z"}
TWO_Q = {"CX", "CZ", "CS", "CSDG"}
THREE_Q = {"CCZ"}


@dataclass
class OCircuit:
    n: int
    ops: list                          # tuples, see parse()
    order: list
    seed: int
    target: str
    n_channels: int
    n_meas: int
    channel_arity: list = field(default_factory=list)   # 1, 2 or 3 per channel
    channel_kind: list = field(default_factory=list)    # DEP1|DEP2|DEP3|XERR
    segments: list = field(default_factory=lambda: [0])  # first op index of each


def parse(text: str) -> OCircuit:
    """Parse circuit text into ('g1', name, q) / ('g2', name, a, b) /
    ('g3', name, a, b, c) / ('m', q, meas_idx) / ('r', q) /
    ('ch', kind, chan_idx, qubits)."""
    n = None
    order = None
    seed = 0
    target = "T"
    ops = []
    nch = 0
    nm = 0
    arity = []
    kinds = []
    segs = [0]
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        tok = line.split()
        op = tok[0].upper()
        args = tok[1:]
        if op == "QUBITS":
            n = int(args[0])
        elif op == "ORDER":
            order = [int(a) for a in args]
        elif op == "SEED":
            seed = int(args[0])
        elif op == "TARGET":
            target = args[0].upper()
        elif op == "TICK":
            continue
        elif op == "SEGMENT":
            if len(ops) != segs[-1]:
                segs.append(len(ops))
        elif op in ONE_Q:
            ops.append(("g1", op, int(args[0])))
        elif op in TWO_Q:
            a, b = int(args[0]), int(args[1])
            if a == b:
                raise ValueError("two-qubit gate on one qubit")
            ops.append(("g2", op, a, b))
        elif op in THREE_Q:
            a, b, c = int(args[0]), int(args[1]), int(args[2])
            if len({a, b, c}) != 3:
                raise ValueError("three-qubit gate on repeated qubits")
            ops.append(("g3", op, a, b, c))
        elif op == "M":
            ops.append(("m", int(args[0]), nm))
            nm += 1
        elif op == "R":
            ops.append(("r", int(args[0])))
        elif op in ("DEP1", "XERR"):
            ops.append(("ch", op, nch, (int(args[0]),)))
            arity.append(1)
            kinds.append(op)
            nch += 1
        elif op == "DEP2":
            ops.append(("ch", op, nch, (int(args[0]), int(args[1]))))
            arity.append(2)
            kinds.append(op)
            nch += 1
        elif op == "DEP3":
            ops.append(("ch", op, nch, (int(args[0]), int(args[1]), int(args[2]))))
            arity.append(3)
            kinds.append(op)
            nch += 1
        else:
            raise ValueError(f"unknown op {op!r}")
    if n is None:
        raise ValueError("missing QUBITS")
    if order is None:
        order = list(range(n))
    if sorted(order) != list(range(n)):
        raise ValueError("ORDER is not a permutation")
    return OCircuit(n=n, ops=ops, order=order, seed=seed, target=target,
                    n_channels=nch, n_meas=nm, channel_arity=arity,
                    channel_kind=kinds, segments=segs)
