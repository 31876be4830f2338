"""CPU tests of the library's host side through the C ABI (no GPU needed):
symbol table, parser errors, the fault sampler (bit-identical to the
oracle's twin), the offline-screen tables (decisions identical to the
oracle's tableau), re-weighting, and error paths of device entry points.
"""
import ctypes as C
import re
from pathlib import Path

import numpy as np
import pytest

import paper_2609_19116_amd as msc
from paper_2609_19116_amd import _lib
from tests.helpers import oracle_csr, oracle_discards
from oracle import estimators as est
from oracle import prescreen as ops
from oracle.ir import parse
from workloads.circuits import config_circuit

ROOT = Path(__file__).resolve().parent.parent


def test_library_exports_every_declared_symbol():
    header = (ROOT / "include" / "msc.h").read_text()
    names = set(re.findall(r"\b(msc_[a-z0-9_]+)\s*\(", header))
    assert len(names) >= 15
    L = _lib.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(_lib._SIGS) == names


def test_order_cost_constants_match_header():
    header = (ROOT / "include" / "msc.h").read_text()
    vals = dict(re.findall(r"#define (MSC_ORDER_COST_[A-Z]+)\s+([0-9.e+]+)", header))
    assert set(vals) == {"MSC_ORDER_COST_PSWAP", "MSC_ORDER_COST_MOVE", "MSC_ORDER_COST_TWOSITE"}
    for k, v in vals.items():
        assert getattr(_lib, k) == float(v), k


def test_struct_sizes_match_header():
    assert C.sizeof(_lib.ShotResult) == 64
    assert C.sizeof(_lib.SimOpts) == 64
    assert C.sizeof(_lib.CircuitInfo) == 72
    assert C.sizeof(_lib.Estimate) == 48
    assert C.sizeof(_lib.BatchStats) == 88
    assert C.sizeof(_lib.EngineStats) == 120


@pytest.mark.parametrize("text,frag", [
    ("H 0\n", "QUBITS"),
    ("QUBITS 2\nFOO 1\n", "unknown op"),
    ("QUBITS 2\nCX 0 0\n", "2q gate"),
    ("QUBITS 2\nH 5\n", "1q gate"),
    ("QUBITS 2\nH 0\nR 0\n", "not at start"),
    ("QUBITS 2\nORDER 0 0\n", "permutation"),
    ("QUBITS 2\nTARGET Q\n", "TARGET"),
    ("QUBITS 3\nCCZ 0 1 1\n", "CCZ"),
    ("QUBITS 3\nCCZ 0 1\n", "CCZ"),
    ("QUBITS 3\nDEP3 0 2 2\n", "DEP3"),
    ("QUBITS 3\nCS 1 1\n", "2q gate"),
])
def test_parse_errors(text, frag):
    with pytest.raises(msc.MscError) as e:
        msc.Circuit(text)
    assert frag in str(e.value)


def test_reset_after_measure_is_legal_and_compiles():
    c = msc.Circuit("QUBITS 2\nH 0\nCX 0 1\nM 1\nDEP1 0\nR 1\nCX 0 1\nM 1\n")
    inf = c.info()
    assert inf["n_meas"] == 2 and inf["n_channels"] == 1


@pytest.mark.parametrize("name", ["tiny", "c1", "c3", "c4", "tiny_ghz", "c1_ghz"])
def test_circuit_info(name):
    cc = config_circuit(name)
    inf = msc.Circuit(cc.text).info()
    assert inf["n_qubits"] == cc.n_qubits
    assert inf["n_channels"] == cc.n_channels
    assert inf["n_meas"] == cc.n_meas
    assert 0 < inf["n_decided"] < inf["n_meas"]
    assert inf["n_twosite"] >= inf["n_swaps"] >= 0
    assert inf["calibrated"] == 0


def test_ctx_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(msc.MscError) as e:
        msc.Ctx(0)
    assert e.value.code == _lib.MSC_E_DEVICE


@pytest.mark.parametrize("name,seed,n,p,weights", [
    ("c1", 0x5EED0001, 1000, 1e-3, None),
    ("c1", 0x5EED0002, 500, 0.0, "w04"),
    ("c3", 0x5EED0003, 200, 1e-3, None),
    ("c4", 0x5EED0004, 100, 1e-3, None),
    ("tiny", 17, 300, 0.2, None),
    ("c1_ghz", 0x5EED0006, 400, 2e-2, None),
])
def test_sampler_matches_oracle_twin(name, seed, n, p, weights):
    cc = config_circuit(name)
    c = msc.Circuit(cc.text)
    w = (np.arange(n) % 5) if weights == "w04" else None
    got = msc.sample_faults(c, seed, 3, n, weights=w, p=p)
    _, ref = oracle_csr(cc.text, seed, n, weights=w, p=p, first=3)
    for a, b in zip(got, ref):
        assert a.dtype == b.dtype and np.array_equal(a, b)


def test_sampler_capacity_error():
    c = msc.Circuit(config_circuit("tiny").text)
    off = np.zeros(11, dtype=np.int64)
    ch = np.zeros(1, dtype=np.int32)
    pa = np.zeros(1, dtype=np.uint8)
    nnz = C.c_int64()
    w = np.full(10, 3, dtype=np.int32)
    rc = _lib.lib().msc_sample_faults(c.h, 1, 0, 10, w.ctypes.data, 0.0, off.ctypes.data,
                                      ch.ctypes.data, pa.ctypes.data, 1, C.byref(nnz))
    assert rc == _lib.MSC_E_CAPACITY and nnz.value == 30


def _canonical_columns(sig):
    """Decided-measurement columns (ints over basis faults), each reduced
    modulo the span of the earlier columns.  Adding an earlier decided
    column to a later one leaves the discard rule unchanged (the shot is
    already discarded when the earlier measurement flips), so two tables
    define the same screen iff their canonical columns are equal."""
    nd = sig.shape[1] * 64
    cols = []
    for d in range(nd):
        bits = (sig[:, d >> 6] >> np.uint64(d & 63)) & np.uint64(1)
        cols.append(int("".join("1" if b else "0" for b in bits[::-1]) or "0", 2))
    basis = {}                       # pivot bit -> vector (reduced echelon)
    out = []
    for v in cols:
        for pb, bv in basis.items():
            if v >> pb & 1:
                v ^= bv
        out.append(v)
        if v:
            pb = v.bit_length() - 1
            for k in list(basis):
                if basis[k] >> pb & 1:
                    basis[k] ^= v
            basis[pb] = v
    return out


@pytest.mark.parametrize("name", ["tiny", "c1", "tiny_ghz", "c1_ghz"])
def test_prescreen_signatures_equal_oracle_table(name):
    cc = config_circuit(name)
    sig, dec = msc.prescreen_tables(msc.Circuit(cc.text))
    circ = parse(cc.text)
    odec, flips = ops.analyse(circ)
    assert list(dec) == [m for m, d in enumerate(odec) if d]
    ref = ops.signature_table(circ, odec, flips)
    assert sig.shape == ref.shape
    assert _canonical_columns(sig) == _canonical_columns(ref)


@pytest.mark.parametrize("name,n,p", [("c1", 3000, 1e-2), ("c3", 800, 3e-3), ("tiny", 1000, 0.1),
                                      ("c1_ghz", 1500, 1e-2)])
def test_prescreen_tables_match_oracle(name, n, p):
    cc = config_circuit(name)
    c = msc.Circuit(cc.text)
    sig, dec = msc.prescreen_tables(c)
    circ, ocsr = oracle_csr(cc.text, 0x5EED0005, n, p=p)
    ref = oracle_discards(circ, ocsr)
    off, ch, pa = ocsr
    got = np.zeros(n, dtype=bool)
    for i in range(n):
        acc = np.zeros(sig.shape[1], dtype=np.uint64)
        for cc_, code in zip(ch[off[i]:off[i + 1]], pa[off[i]:off[i + 1]]):
            for k in range(6):
                if code >> k & 1:
                    acc ^= sig[6 * cc_ + k]
        got[i] = acc.any()
    assert np.array_equal(got, ref)
    assert ref.any() and not ref.all()


def test_reweight_matches_oracle_estimators():
    rng = np.random.default_rng(1)
    n = rng.integers(10, 100, size=6).astype(float)
    a = n * rng.uniform(0.2, 1.0, size=6)
    e = a * rng.uniform(0.0, 0.1, size=6)
    for M, p in [(243, 1e-3), (1249, 5e-4), (1863, 2e-3)]:
        got = msc.reweight(n, a, e, M, [p])[0]
        ref = est.reweight(list(n), list(a), list(e), M, p)
        assert got["p_acc"] == pytest.approx(ref["p_acc"], rel=1e-12)
        assert got["p_acc_le"] == pytest.approx(ref["p_acc_le"], rel=1e-12)
        assert got["p_le"] == pytest.approx(ref["p_le"], rel=1e-12)
        assert got["trunc_bound"] == pytest.approx(ref["B"], rel=1e-9, abs=1e-15)
        # standard errors: from sums of squares, and from the [0, 1] bound
        a2 = a * rng.uniform(0.3, 1.0, size=6)
        e2 = e * rng.uniform(0.0, 0.1, size=6)
        n1 = n.copy()
        n1[2] = 1.0                           # one-shot bin: the bound
        a1 = a.copy()
        a1[2] = 0.4
        e1 = e.copy()
        e1[2] = 0.0
        for nn, aa, ee in ((n, a, e), (n1, a1, e1)):
            got = msc.reweight(nn, aa, ee, M, [p], a2, e2)[0]
            sa, se = est.standard_errors(list(nn), list(aa), list(ee), M, p, list(a2), list(e2))
            assert got["sem_p_acc"] == pytest.approx(sa, rel=1e-12)
            assert got["sem_p_acc_le"] == pytest.approx(se, rel=1e-12)
        got = msc.reweight(n, a, e, M, [p])[0]
        sa, se = est.standard_errors(list(n), list(a), list(e), M, p)
        assert got["sem_p_acc"] == pytest.approx(sa, rel=1e-12)
        assert got["sem_p_acc_le"] == pytest.approx(se, rel=1e-12)


def test_reweight_errors():
    with pytest.raises(msc.MscError):
        msc.reweight([1.0], [1.0], [0.0], 10, [1.5])
    with pytest.raises(msc.MscError):
        msc.reweight([1.0] * 5, [1.0] * 5, [0.0] * 5, 3, [0.1])


def test_device_calls_reject_null_context():
    L = _lib.lib()
    o = _lib.SimOpts(0, 64, 0.0, 1e-6, 1e-4, 0, 0)
    assert L.msc_simulate(None, None, C.byref(o), 0, None, None, None, None, 0, None) \
        == _lib.MSC_E_INVALID
    cnt = C.c_int64()
    assert L.msc_prescreen(None, None, 0, None, None, None, None, None, C.byref(cnt)) \
        == _lib.MSC_E_INVALID
    assert L.msc_twosite_contract(None, 1, 64, 1, None, None, None, None) == _lib.MSC_E_INVALID


def test_reciprocal_index_split_is_exact():
    """The shot kernels split an element index i into i / d and i % d as
    trunc(i * inv + inv / 2) with inv an approximation of 1/d (a hardware
    reciprocal refined by one Newton step: relative error far below
    2^-40).  The exact quotient of i + 1/2 lies at least 1/(2d) from an
    integer, so the split is exact for 0 <= i < 2^31 and 0 < d < 2^20:
    checked with inv off by +-2^-40 relative, on every divisor up to 2048
    and some large ones, at the indices next to every multiple of d up to
    2^16 and near 2^31."""
    rng = np.random.default_rng(7)
    for d in list(range(1, 2049)) + [4095, 65535, (1 << 20) - 1]:
        k = np.arange(0, (1 << 16) // d + 2, dtype=np.int64)
        near = np.concatenate([k * d - 1, k * d, k * d + d - 1])
        top = (1 << 31) - 1 - np.arange(0, 4 * d, max(1, d // 8), dtype=np.int64)
        i = np.concatenate([near[near >= 0], top, rng.integers(0, 1 << 31, 64)])
        for pert in (1.0 - 2.0 ** -40, 1.0 + 2.0 ** -40):
            inv = (1.0 / d) * pert
            q = np.trunc(i.astype(np.float64) * inv + 0.5 * inv).astype(np.int64)
            assert np.array_equal(q, i // d), d
