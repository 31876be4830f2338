"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself or with the GPU path: each
test checks a closed form, an invariant, a textbook or library routine, a
brute-force enumeration or a value printed in the paper.
"""
import itertools
import json
import math
import os
import random

import numpy as np
import pytest
from scipy import stats

from oracle import estimators as est
from oracle import mps as omps
from oracle import prescreen as ops
from oracle import sampler as osamp
from oracle import statevector as sv
from oracle.gates import G1, G2, ccz_sequence, fault_paulis, target_state
from oracle.ir import parse
from workloads.circuits import config_circuit, make_circuit

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one_qubit(prep: str, fault_kind: str = "") -> str:
    lines = ["QUBITS 1", "SEED 0", "TARGET T"] + [f"{g} 0" for g in prep.split()]
    if fault_kind:
        lines.append("DEP1 0")
    return "\n".join(lines) + "\n"


# ---------------------------------------------------------------- closed forms
def _embed(ops_, n=3):
    """Matrix of a gate list on n qubits (qubit 0 most significant)."""
    u = np.eye(2 ** n, dtype=complex)
    for g in ops_:
        if g[0] == "CX":
            c_, t_ = g[1], g[2]
            m = np.zeros((2 ** n, 2 ** n), dtype=complex)
            for x in range(2 ** n):
                y = x ^ (1 << (n - 1 - t_)) if x >> (n - 1 - c_) & 1 else x
                m[y, x] = 1
        else:
            m = np.array([[1]], dtype=complex)
            for q in range(n):
                m = np.kron(m, G1[g[0]] if q == g[1] else np.eye(2))
        u = m @ u
    return u


def test_controlled_phase_gates_from_definitions():
    # CCZ = diag(1,...,1,-1) (the MPS applies it as a CNOT + T network);
    # CS = diag(1,1,1,i): CS^2 = CZ, CS CS^dagger = I
    for a, b, c in itertools.permutations(range(3)):
        assert np.allclose(_embed(ccz_sequence(a, b, c)), np.diag([1] * 7 + [-1]), atol=1e-14)
    assert sum(1 for g in ccz_sequence(0, 1, 2) if g[0] in ("T", "TDG")) == 7
    assert np.allclose(G2["CS"] @ G2["CS"], G2["CZ"], atol=1e-15)
    assert np.allclose(G2["CS"] @ G2["CSDG"], np.eye(4), atol=1e-15)
    # bits 2j, 2j+1 of a fault code are the x, z bits of the j-th qubit
    got = dict((q, P) for q, P in fault_paulis(0b110110, (5, 6, 7)))
    assert np.allclose(got[5], G1["Z"]) and np.allclose(got[6], G1["X"])
    assert np.allclose(got[7], G1["Y"])
    assert [q for q, _ in fault_paulis(0b000100, (5, 6))] == [6]


def test_gates_unitary_and_t_state():
    for u in list(G1.values()) + list(G2.values()):
        assert np.allclose(u.conj().T @ u, np.eye(u.shape[0]), atol=1e-15)
    t = target_state("T")
    # |T> = T|+> = (|0> + e^{i pi/4}|1>)/sqrt(2)  (Introduction)
    assert np.allclose(t, np.array([1, np.exp(1j * np.pi / 4)]) / np.sqrt(2), atol=1e-15)
    ex = lambda P: np.real(np.conj(t) @ P @ t)
    assert abs(ex(G1["X"]) - 1 / math.sqrt(2)) < 1e-15
    assert abs(ex(G1["Y"]) - 1 / math.sqrt(2)) < 1e-15
    assert abs(ex(G1["Z"])) < 1e-15
    plus = np.array([1, 1]) / math.sqrt(2)
    assert abs(abs(np.conj(plus) @ t) ** 2 - math.cos(math.pi / 8) ** 2) < 1e-15


@pytest.mark.parametrize("engine", [sv, omps])
@pytest.mark.parametrize("code,infid", [(0, 0.0), (1, 0.5), (2, 1.0), (3, 0.5)])
def test_single_qubit_fidelity_closed_forms(engine, code, infid):
    # 1 - |<T|P|T>|^2: X and Y give 1/2, Z gives 1 (Appendix "Post-selection
    # and logical error": Pauli noise moves the overlap far from 1)
    c = parse(one_qubit("H T", "x"))
    r = engine.run_shot(c, {0: code} if code else {})
    assert r.p_acc == pytest.approx(1.0, abs=1e-14)
    assert r.infid == pytest.approx(infid, abs=1e-14)


def test_s_target_fidelity():
    c = parse("QUBITS 1\nSEED 0\nTARGET S\nH 0\nS 0\nT 0\n")
    r = sv.run_shot(c, {})
    # |<S|T|S>|^2 = |(1 + e^{i pi/4})/2|^2 = cos^2(pi/8)
    assert r.infid == pytest.approx(1 - math.cos(math.pi / 8) ** 2, abs=1e-14)


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("name", ["tiny", "c1", "tiny_ghz", "c1_ghz"])
@pytest.mark.parametrize("target", ["T", "S"])
def test_noiseless_circuits_are_deterministic(name, target):
    # every measurement has p(e_m) = 1 and the decoded seed equals the target
    c = parse(config_circuit(name, target).text)
    for engine in (sv, omps):
        r = engine.run_shot(c, {}, record=True)
        assert r.p_acc == pytest.approx(1.0, abs=1e-12)
        assert r.infid < 1e-12
        assert min(r.meas_probs) > 1 - 1e-12


def test_noiseless_49_qubit_circuit_on_mps():
    c = parse(config_circuit("c3").text)
    r = omps.run_shot(c, {}, record=True)
    assert r.p_acc == pytest.approx(1.0, abs=1e-10)
    assert r.infid < 1e-10
    assert r.chi_peak <= 2 ** 7


def _random_faults(circ, rng, w):
    f = {}
    for ch in rng.sample(range(circ.n_channels), w):
        k = circ.channel_kind[ch]
        f[ch] = 1 if k == "XERR" else rng.randrange(1, 4 if k == "DEP1" else 16)
    return f


def test_pacc_chain_rule_equals_projected_norm():
    # P_acc = prod_m p(e_m) = || prod_m Pi_m U psi ||^2
    c = parse(config_circuit("tiny").text)
    rng = random.Random(3)
    seen_partial = 0
    for _ in range(300):
        f = _random_faults(c, rng, rng.randrange(0, 4))
        r = sv.run_shot(c, f, tau_rej=0.0)
        psi = sv.final_state(c, f)
        assert r.p_acc == pytest.approx(float(np.vdot(psi, psi).real), abs=1e-12)
        seen_partial += 0.0 < r.p_acc < 1.0
    assert seen_partial > 0


@pytest.mark.parametrize("name,n_shots", [("tiny", 200), ("c1", 25), ("tiny_ghz", 150),
                                          ("c1_ghz", 12)])
def test_mps_agrees_with_state_vector(name, n_shots):
    c = parse(config_circuit(name).text)
    rng = random.Random(11)
    for _ in range(n_shots):
        f = _random_faults(c, rng, rng.randrange(0, 3))
        a = sv.run_shot(c, f, record=True)
        b = omps.run_shot(c, f, record=True)
        assert a.p_acc == pytest.approx(b.p_acc, abs=1e-12)
        assert a.infid == pytest.approx(b.infid, abs=1e-12)
        assert a.rejected_at == b.rejected_at


def _mps_vector(m, order):
    v = m.A[0]
    for k in range(1, len(m.A)):
        v = np.tensordot(v, m.A[k], axes=([-1], [0]))
    v = v.reshape((2,) * len(m.A))          # axes in site order
    perm = np.argsort(order)                 # qubit q sits at site perm[q]
    return np.transpose(v, perm).reshape(-1)


def _random_circuit(n, depth, rng, clifford):
    gates = ["H", "S"] + ([] if clifford else ["T", "TDG"])
    lines = [f"QUBITS {n}", "SEED 0", "TARGET T"]
    order = list(range(n))
    rng.shuffle(order)
    lines.append("ORDER " + " ".join(map(str, order)))
    for _ in range(depth):
        if rng.random() < 0.5:
            a, b = rng.sample(range(n), 2)
            lines.append(f"{rng.choice(['CX', 'CZ'])} {a} {b}")
        else:
            lines.append(f"{rng.choice(gates)} {rng.randrange(n)}")
    return "\n".join(lines) + "\n", order


def test_mps_amplitudes_match_state_vector_and_bond_bound():
    rng = random.Random(5)
    for _ in range(6):
        text, order = _random_circuit(8, 60, rng, clifford=False)
        c = parse(text)
        omps.run_shot(c, {})
        m = omps.run_shot.last
        psi = sv.final_state(c, {})
        assert np.allclose(_mps_vector(m, order), psi, atol=1e-12)
        for k, chi in enumerate(m.bonds(), start=1):
            assert chi <= 2 ** min(k, 8 - k)     # chi_k <= 2^min(k, N-k)


def _stabiliser_bond_dims(text, order):
    """chi_k = 2^(rank(G_A) - |A|) for a stabiliser state (textbook
    formula for the entanglement of stabiliser states)."""
    c = parse(text)
    n = c.n
    x = np.zeros((n, n), dtype=np.uint8)
    z = np.eye(n, dtype=np.uint8)
    for op in c.ops:
        if op[0] == "g1":
            q = op[2]
            if op[1] == "H":
                x[:, q], z[:, q] = z[:, q].copy(), x[:, q].copy()
            elif op[1] == "S":
                z[:, q] ^= x[:, q]
        elif op[0] == "g2":
            a, b = op[2], op[3]
            if op[1] == "CX":
                x[:, b] ^= x[:, a]
                z[:, a] ^= z[:, b]
            else:
                z[:, a] ^= x[:, b]
                z[:, b] ^= x[:, a]

    def rank2(mat):
        m = mat.copy() % 2
        r = 0
        for col in range(m.shape[1]):
            piv = next((i for i in range(r, m.shape[0]) if m[i, col]), None)
            if piv is None:
                continue
            m[[r, piv]] = m[[piv, r]]
            for i in range(m.shape[0]):
                if i != r and m[i, col]:
                    m[i] ^= m[r]
            r += 1
        return r

    dims = []
    for k in range(1, n):
        A = order[:k]
        GA = np.concatenate([x[:, A], z[:, A]], axis=1)
        dims.append(2 ** (rank2(GA) - k))
    return dims


def test_clifford_bond_dims_match_stabiliser_formula():
    rng = random.Random(7)
    for _ in range(8):
        text, order = _random_circuit(9, 70, rng, clifford=True)
        c = parse(text)
        omps.run_shot(c, {})
        assert omps.run_shot.last.bonds() == _stabiliser_bond_dims(text, order)


def test_clifford_measurement_probabilities_are_0_half_1():
    rng = random.Random(9)
    for _ in range(10):
        text, _ = _random_circuit(7, 40, rng, clifford=True)
        text += "".join(f"M {q}\n" for q in range(7))
        c = parse(text)
        r = sv.run_shot(c, {}, tau_rej=0.0, record=True)
        for p in r.meas_probs:
            assert min(abs(p), abs(p - 0.5), abs(p - 1.0)) < 1e-12


# ---------------------------------------------------------------- pre-screen
def _all_single_faults(c):
    for ch in range(c.n_channels):
        k = c.channel_kind[ch]
        codes = [1] if k == "XERR" else range(1, {"DEP1": 4, "DEP2": 16, "DEP3": 64}[k])
        for code in codes:
            yield {ch: code}


def test_prescreen_exhaustive_single_faults_ghz_gadgets():
    # CS, CS^dagger and CCZ inside the GHZ-controlled checks (Section 4.2:
    # the only non-Cliffords are diagonal); no discarded single fault may
    # have a nonzero acceptance probability.
    c = parse(config_circuit("tiny_ghz").text)
    assert any(o[0] == "g3" for o in c.ops)
    assert any(o[0] == "g2" and o[1] in ("CS", "CSDG") for o in c.ops)
    dec, fl = ops.analyse(c)
    n_disc = 0
    for f in _all_single_faults(c):
        if ops.discard(dec, fl, f):
            n_disc += 1
            assert sv.run_shot(c, f).p_acc == 0.0
    assert n_disc > 300


@pytest.mark.parametrize("gate", ["CS 0 1", "CSDG 1 0", "CCZ 0 1 2", "CCZ 2 0 1"])
def test_prescreen_diagonal_gates_undecide_what_they_entangle(gate):
    # a diagonal non-Clifford between |+> qubits makes the later X-basis
    # read-out of its support random: the measurement must not be decided,
    # otherwise the Z fault in front of it would be a false discard.
    text = f"QUBITS 3\nH 0\nH 1\nH 2\nDEP1 0\nDEP1 1\n{gate}\nH 0\nM 0\nH 1\nM 1\n"
    c = parse(text)
    dec, fl = ops.analyse(c)
    assert dec == [False, False]
    for f in _all_single_faults(c):
        r = sv.run_shot(c, f, tau_rej=0.0)
        assert r.p_acc > 0.1
        assert not ops.discard(dec, fl, f)


def test_prescreen_exact_on_clifford_three_qubit_channels():
    # every component of a three-qubit channel is injected: on a Clifford
    # circuit the screen is exact (discard iff P_acc = 0)
    text = ("QUBITS 4\nH 0\nCX 0 1\nCX 1 2\nH 3\nDEP3 0 1 2\nDEP3 3 2 0\n"
            "CX 1 2\nCX 0 1\nH 0\nH 3\nM 0\nM 1\nM 2\nM 3\n")
    c = parse(text)
    dec, fl = ops.analyse(c)
    assert all(dec)
    third_only = 0
    for f in _all_single_faults(c):
        d = ops.discard(dec, fl, f)
        assert d == (sv.run_shot(c, f).p_acc == 0.0)
        (code,) = f.values()
        third_only += d and code & 0b1111 == 0
    assert third_only > 0      # a fault on the third qubit alone is caught


@pytest.mark.parametrize("target", ["T", "S"])
def test_prescreen_exhaustive_single_faults(target):
    # Section 4.2: the screen cannot discard a shot that could be accepted;
    # for the pure-Clifford |S> control every measurement is decided and the
    # screen is exact.
    c = parse(config_circuit("tiny", target).text)
    dec, fl = ops.analyse(c)
    if target == "S":
        assert all(dec)
    for f in _all_single_faults(c):
        d = ops.discard(dec, fl, f)
        r = sv.run_shot(c, f)
        if d:
            assert r.p_acc == 0.0
        if target == "S":
            assert d == (r.p_acc == 0.0)


def test_prescreen_no_false_discards_multi_fault():
    c = parse(config_circuit("tiny").text)
    dec, fl = ops.analyse(c)
    rng = random.Random(2)
    n_disc = 0
    for _ in range(400):
        f = _random_faults(c, rng, rng.randrange(1, 5))
        if ops.discard(dec, fl, f):
            n_disc += 1
            assert sv.run_shot(c, f).p_acc == 0.0
    assert n_disc > 100


def test_prescreen_sampled_c1():
    c = parse(config_circuit("c1").text)
    dec, fl = ops.analyse(c)
    assert sum(dec) < c.n_meas          # the T frames leave some undecided
    rng = random.Random(4)
    for _ in range(40):
        f = _random_faults(c, rng, rng.randrange(1, 3))
        if ops.discard(dec, fl, f):
            assert omps.run_shot(c, f).p_acc == 0.0


# ---------------------------------------------------------------- sampler
def test_sampler_weight_distribution_is_binomial():
    c = parse(config_circuit("c1").text)
    M, p, n = c.n_channels, 0.01, 6000
    off, ch, pa = osamp.sample_csr(c, 123, 0, n, p=p)
    w = np.diff(off)
    kmax = 8
    obs = np.bincount(np.minimum(w, kmax), minlength=kmax + 1)
    pmf = stats.binom.pmf(np.arange(kmax), M, p)
    exp = np.append(pmf, 1 - pmf.sum()) * n
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert chi2 < stats.chi2.ppf(0.999, kmax)


def test_sampler_subsets_and_paulis_uniform():
    c = parse(config_circuit("tiny").text)
    M, n = c.n_channels, 4000
    off, ch, pa = osamp.sample_csr(c, 99, 0, n, weights=[3] * n)
    assert np.all(np.diff(off) == 3)
    for i in range(n):                    # distinct, sorted
        s = ch[off[i]:off[i + 1]]
        assert np.all(np.diff(s) > 0)
    cnt = np.bincount(ch, minlength=M)
    e = 3 * n / M
    assert ((cnt - e) ** 2 / e).sum() < stats.chi2.ppf(0.999, M - 1)
    two = np.array([c.channel_kind[x] == "DEP2" for x in ch])
    codes = np.bincount(pa[two], minlength=16)[1:]
    e2 = two.sum() / 15
    assert ((codes - e2) ** 2 / e2).sum() < stats.chi2.ppf(0.999, 14)
    assert codes.min() > 0


def test_binomial_table_matches_scipy():
    for M, p in [(243, 1e-3), (1863, 1e-3), (292, 0.05)]:
        cdf = osamp.binomial_cdf_table(M, p)
        ref = stats.binom.cdf(np.arange(len(cdf)), M, p)
        assert np.allclose(cdf, ref, rtol=1e-12, atol=1e-15)
        for w in range(6):
            assert est.binom_pmf(M, w, p) == pytest.approx(stats.binom.pmf(w, M, p), rel=1e-10)


# ---------------------------------------------------------------- estimators
def test_binomial_weights_sum_to_one_and_bound():
    M, p = 243, 1e-3
    tot = sum(est.binom_pmf(M, w, p) for w in range(M + 1))
    assert tot == pytest.approx(1.0, abs=1e-12)
    r = est.reweight([1, 1, 1], [1, 1, 1], [0, 0, 0], M, p)
    assert r["B"] == pytest.approx(1 - stats.binom.cdf(2, M, p), rel=1e-9)
    # all bins accepted with certainty -> p_acc = 1 - B
    assert r["p_acc"] == pytest.approx(1 - r["B"], abs=1e-12)


def test_loss_table_from_paper():
    g = json.load(open(os.path.join(GOLDEN, "loss_table.json")))
    for row in g["rows"].values():
        for pl, printed in zip(g["p_loss"], row["factor"]):
            assert abs(est.loss_multiplier(row["M"], pl) - printed) <= 0.005 + 1e-9


def test_weight_one_bin_brute_force_matches_sampling():
    # p_acc^(1) is the average of P_acc over a uniform channel and a
    # uniform non-identity Pauli; the subset sampler must estimate it.
    c = parse(config_circuit("tiny").text)
    exact = 0.0
    for ch in range(c.n_channels):
        k = c.channel_kind[ch]
        codes = [1] if k == "XERR" else list(range(1, 4 if k == "DEP1" else 16))
        exact += sum(sv.run_shot(c, {ch: code}).p_acc for code in codes) / len(codes)
    exact /= c.n_channels
    n = 3000
    off, chs, pa = osamp.sample_csr(c, 5, 0, n, weights=[1] * n)
    vals = [sv.run_shot(c, f).p_acc for f in osamp.csr_to_dicts(off, chs, pa)]
    sem = np.std(vals) / math.sqrt(n)
    assert abs(np.mean(vals) - exact) < 5 * sem
    # Eq. (reweight) to first order in p: p_acc = 1 - M p (1 - p_acc^(1))
    M, p = c.n_channels, 1e-6
    r = est.reweight([1, 1], [1.0, exact], [0, 0], M, p)
    assert r["p_acc"] == pytest.approx(1 - M * p * (1 - exact), abs=(M * p) ** 2)


def test_bin_sums_hand_example():
    # five shots by hand: weights 0, 2, 0, 1, 2 with P_acc 1, 1/2, 1/4, 0,
    # 3/4 and failure flags 0, 1, 0, 0, 1 give per weight the shot counts
    # (2, 1, 2), the P_acc sums (5/4, 0, 5/4) and the P_acc * fail sums
    # (0, 0, 1/2 + 3/4)
    n, a, e = est.bin_sums([0, 2, 0, 1, 2], [1.0, 0.5, 0.25, 0.0, 0.75], [0, 1, 0, 0, 1])
    assert n == [2.0, 1.0, 2.0]
    assert a == [1.25, 0.0, 1.25]
    assert e == [0.0, 0.0, 1.25]


def test_standard_errors_match_replicate_spread():
    # the standard error of Eq. (reweight) against the spread of the
    # estimator over replicate samples: per-bin values drawn from known
    # distributions (Beta for P_acc, Bernoulli failures), 4000 replicates
    rng = np.random.default_rng(11)
    M, p = 60, 0.03
    nw = [40, 25, 15, 8]
    shapes = [(50.0, 1.0), (3.0, 2.0), (1.0, 1.5), (0.7, 0.9)]
    pfail = [0.0, 0.1, 0.3, 0.5]
    R = 4000
    est_a, est_e, sem_a, sem_e = [], [], [], []
    for _ in range(R):
        n, a, e, a2, e2 = [], [], [], [], []
        for w in range(4):
            x = rng.beta(*shapes[w], size=nw[w])
            y = x * (rng.random(nw[w]) < pfail[w])
            n.append(float(nw[w]))
            a.append(float(x.sum()))
            e.append(float(y.sum()))
            a2.append(float((x * x).sum()))
            e2.append(float((y * y).sum()))
        r = est.reweight(n, a, e, M, p)
        sa, se = est.standard_errors(n, a, e, M, p, a2, e2)
        est_a.append(r["p_acc"])
        est_e.append(r["p_acc_le"])
        sem_a.append(sa)
        sem_e.append(se)
    assert abs(np.mean(sem_a) / np.std(est_a) - 1.0) < 0.05
    assert abs(np.mean(sem_e) / np.std(est_e) - 1.0) < 0.05


def test_standard_error_bound_is_exact_for_bernoulli_bins():
    # for 0/1 values the [0, 1] bound mean (1 - mean) is the variance
    # itself: the bound's standard error at the true means equals the
    # closed form sqrt(sum Bin_w^2 q_w (1 - q_w) / n_w)
    M, p = 30, 0.05
    q = [0.9, 0.4, 0.2]
    n = [50.0, 20.0, 10.0]
    a = [qi * ni for qi, ni in zip(q, n)]
    sa, _ = est.standard_errors(n, a, [0.0] * 3, M, p)
    ref = math.sqrt(sum(est.binom_pmf(M, w, p) ** 2 * q[w] * (1 - q[w]) / n[w]
                        for w in range(3)))
    assert abs(sa - ref) <= 1e-15 * ref
