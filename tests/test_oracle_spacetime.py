"""Pins of the oracle's space-time accounting (oracle/spacetime.py): the
segment table of a circuit worked out by hand, the reach probabilities
against their definition on both simulators (state vector and MPS agree),
the last reach equal to P_acc, reach values of a Clifford circuit in
{0} U {2^-k}, and the expected volume at p -> 0 equal to the total noisy
volume.
"""
import math

import numpy as np
import pytest

from oracle import mps as omps
from oracle import sampler as osamp
from oracle import spacetime as st
from oracle import statevector as sv
from oracle.ir import parse
from workloads.circuits import config_circuit

HAND = """QUBITS 3
SEED 0
SEGMENT
H 0
CX 0 1
DEP2 0 1
SEGMENT
CX 1 2
H 0
M 2
SEGMENT
SEGMENT
M 0
"""


def test_segment_table_by_hand():
    segs = st.segments(parse(HAND))
    # a SEGMENT before any op and a repeated one open no empty segment
    assert [(g["first_meas"], g["n_qubits"], g["depth"], g["noisy"]) for g in segs] == [
        (0, 2, 2, True),      # H 0 | CX 0 1 (+ noise)
        (0, 3, 2, False),     # CX 1 2, H 0 | M 2
        (1, 1, 1, False),     # M 0
    ]
    assert [g["volume"] for g in segs] == [4, 6, 1]


def _faults(circ, seed, n, w):
    off, ch, pa = osamp.sample_csr(circ, seed, 0, n, weights=[w] * n)
    return osamp.csr_to_dicts(off, ch, pa)


@pytest.mark.parametrize("name", ["tiny", "tiny_ghz"])
def test_reach_from_both_simulators(name):
    circ = parse(config_circuit(name).text)
    segs = st.segments(circ)
    first = [g["first_meas"] for g in segs] + [circ.n_meas]
    for w in (0, 1, 2):
        for f in _faults(circ, 0x5EED0041 + w, 12, w):
            a = sv.run_shot(circ, f, record=True)
            b = omps.run_shot(circ, f, record=True)
            ra = st.shot_survival(first, a.meas_probs, a.rejected_at >= 0)
            rb = st.shot_survival(first, b.meas_probs, b.rejected_at >= 0)
            assert np.allclose(ra, rb, atol=1e-12)
            assert ra[0] == 1.0
            assert all(x >= y - 1e-15 for x, y in zip(ra, ra[1:]))      # non-increasing
            assert ra[-1] == pytest.approx(a.p_acc, abs=1e-12)          # to the end: P_acc


def test_reach_of_clifford_circuit_is_dyadic():
    circ = parse(config_circuit("tiny", target="S").text)
    first = [g["first_meas"] for g in st.segments(circ)]
    seen = set()
    for w in (1, 2, 3):
        for f in _faults(circ, 0x5EED0044 + w, 20, w):
            r = sv.run_shot(circ, f, record=True)
            for x in st.shot_survival(first, r.meas_probs, r.rejected_at >= 0):
                if x > 0:
                    k = -math.log2(x)
                    assert abs(k - round(k)) < 1e-9, x
                seen.add(round(x, 9))
    assert 0.0 in seen and 1.0 in seen


def test_expected_volume_limits():
    circ = parse(config_circuit("tiny").text)
    segs = st.segments(circ)
    noisy_total = sum(g["volume"] for g in segs if g["noisy"])
    K = len(segs)
    # one sampled bin (w = 0) whose shots all reach everything
    bin_n = [10.0]
    bin_surv = [[10.0] * K]
    reach, vol, vol_b = st.expected_volume(bin_n, bin_surv, segs, circ.n_channels, 0.0)
    assert np.allclose(reach, 1.0) and vol == noisy_total and vol_b == noisy_total
    # at p > 0 only Bin_0 of that reach is covered; B bounds the rest
    p = 1e-3
    reach, vol, vol_b = st.expected_volume(bin_n, bin_surv, segs, circ.n_channels, p)
    b0 = (1 - p) ** circ.n_channels
    assert np.allclose(reach, b0, rtol=1e-12)
    assert vol_b == pytest.approx(noisy_total, rel=1e-12)    # b0 + B = 1
