"""Expected space-time volume of a post-selected circuit, oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written from the
paper's appendix "Space-time overhead": a section's volume is the number of
qubits it uses times its number of gate layers (its depth); the expected
volume sums the sections' volumes, each weighted by the fraction of shots
that reach it, assuming a shot stops as soon as a measurement rejects it.

Readings (the paper fixes no more):
* sections are the circuit's segments, cut at SEGMENT lines;
* a segment uses the qubits that any of its gates, measurements or resets
  acts on; its depth is the number of layers of an as-soon-as-possible
  schedule of those ops (each op one layer after the latest earlier op on
  any of its qubits); noise channels are not layers;
* a shot reaches segment s with probability prod_{m < m_s} p(e_m), the
  product of its expected-outcome probabilities over the measurements
  before the segment (m_s of them), and 0 once a measurement has rejected
  it (p < tau_rej);
* per fault weight w the reach probability is averaged over the bin's
  shots; over weights it is re-weighted with Bin_w(p) as in Eq. (reweight);
  bins beyond the last sampled weight add at most B times the volume
  (upper bound only);
* only segments that hold a noise channel count towards the total (the
  paper leaves the noiseless stage out).
"""
from __future__ import annotations

import numpy as np

from .estimators import binom_pmf


def _qubits(op):
    k = op[0]
    if k == "g1":
        return (op[2],)
    if k == "g2":
        return (op[2], op[3])
    if k == "g3":
        return (op[2], op[3], op[4])
    if k in ("m", "r"):
        return (op[1],)
    return op[3]                        # channel


def segments(circ):
    """Per segment: dict(first_meas, n_qubits, depth, noisy, volume)."""
    bounds = list(circ.segments) + [len(circ.ops)]
    out = []
    meas_before = 0
    for s in range(len(bounds) - 1):
        ops = circ.ops[bounds[s]:bounds[s + 1]]
        used = set()
        layer = {}
        depth = 0
        noisy = False
        first = meas_before
        for op in ops:
            if op[0] == "ch":
                noisy = True
                continue
            qs = _qubits(op)
            used.update(qs)
            t = 1 + max(layer.get(q, 0) for q in qs)
            for q in qs:
                layer[q] = t
            depth = max(depth, t)
            if op[0] == "m":
                meas_before += 1
        out.append(dict(first_meas=first, n_qubits=len(used), depth=depth, noisy=noisy,
                        volume=len(used) * depth))
    return out


def shot_survival(first_meas: list, meas_probs: list, rejected: bool) -> list:
    """Reach probability of each segment for one shot from its recorded
    expected-outcome probabilities (the last one rejected it if rejected)."""
    out = []
    for m_s in first_meas:
        if rejected and m_s > len(meas_probs) - 1:
            out.append(0.0)
        else:
            out.append(float(np.prod(meas_probs[:m_s])))
    return out


def expected_volume(bin_n, bin_surv, segs, M: int, p: float):
    """(reach probability per segment, expected volume of the noisy
    segments, the same plus the truncation bound): bin_surv[w][s] is the sum
    over the bin's shots of their reach probability of segment s."""
    nb = len(bin_n)
    reach = np.zeros(len(segs))
    for w in range(nb):
        if bin_n[w] > 0:
            reach += binom_pmf(M, w, p) * np.asarray(bin_surv[w], dtype=float) / bin_n[w]
    B = sum(binom_pmf(M, w, p) for w in range(nb, M + 1))
    vol = sum(sg["volume"] * r for sg, r in zip(segs, reach) if sg["noisy"])
    vmax = sum(sg["volume"] for sg in segs if sg["noisy"])
    return reach, vol, vol + B * vmax
