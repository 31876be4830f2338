"""GPU parity at the sizes of the named workloads.

- 17 qubits, 1000 shots, w ~ Bin(M, 1e-3), FP64 path (one launch): every
  shot against the oracle MPS, the first 40 also against the state vector.
- 17 qubits, 65536 shots, subset sampling w = 0..4, one persistent launch
  in FP32 and one in FP64: all shots FP32 vs FP64 within 1e-5, a stratified
  sample against the oracle.
- 81 qubits (unrotated d=5), 256 shots at p = 1e-3, screen + FP32 batch:
  validity of every record, w = 0 shots equal to the noiseless oracle result
  (P_acc = 1, f = 1), early-rejected shots against the oracle one by one.
- Offline screen on the 81-qubit circuit, 2^24 shots: bit-exact against the
  oracle's own vectorised evaluation.
"""
import numpy as np
import pytest

import paper_2609_19116_amd as msc
from paper_2609_19116_amd import MSC_FP32, MSC_FP64, results_numpy
from oracle import prescreen as ops
from tests.helpers import oracle_csr, oracle_results, say, to_dev
from tests.test_gpu_parity import TOL, _compare, _same_csr
from workloads.circuits import config_circuit
from oracle.ir import parse

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = msc.Ctx(0)
    yield c
    c.close()


def _cal(ctx, name):
    cc = config_circuit(name)
    c = msc.Circuit(cc.text)
    say(f"calibrate {name}")
    c.calibrate(ctx)
    return cc, c


def test_c1_1000_shots_fp64(ctx):
    cc, c = _cal(ctx, "c1")
    n = 1000
    csr = msc.sample_faults(c, 0x5EED0001, 0, n, p=1e-3)
    circ, ocsr = oracle_csr(cc.text, 0x5EED0001, n, p=1e-3)
    assert _same_csr(csr, ocsr)
    off, ch, pa = to_dev(*csr)
    say("c1 1000 shots fp64")
    res = results_numpy(msc.simulate(ctx, c, off, ch, pa, precision=MSC_FP64))
    ref = oracle_results(circ, ocsr)
    _compare(res, ref, TOL[MSC_FP64])
    ref_sv = oracle_results(circ, ocsr, engine="sv", idx=range(40))
    _compare(res[:40], ref_sv, TOL[MSC_FP64])


def test_c2_65536_shots_one_launch(ctx):
    cc, c = _cal(ctx, "c2")
    n = 65536
    w = (np.arange(n) % 5).astype(np.int32)
    csr = msc.sample_faults(c, 0x5EED0002, 0, n, weights=w)
    circ, ocsr = oracle_csr(cc.text, 0x5EED0002, 2000, weights=w[:2000])
    assert all(np.array_equal(a, b) for a, b in
               zip((csr[0][:2001], csr[1][:csr[0][2000]], csr[2][:csr[0][2000]]), ocsr))
    off, ch, pa = to_dev(*csr)
    say("c2 65536 shots fp32")
    r32 = results_numpy(msc.simulate(ctx, c, off, ch, pa, precision=MSC_FP32))
    say("c2 65536 shots fp64")
    r64 = results_numpy(msc.simulate(ctx, c, off, ch, pa, precision=MSC_FP64))
    acc = r64["p_acc"] > 0
    assert np.all(r32["p_acc"][~acc] == 0.0)
    assert (np.abs(r32["p_acc"] - r64["p_acc"])[acc] / r64["p_acc"][acc]).max() <= TOL[MSC_FP32]
    scale = np.maximum(r64["infid"], 1.0 - r64["infid"])
    assert (np.abs(r32["infid"] - r64["infid"])[acc] / scale[acc]).max() <= TOL[MSC_FP32]
    assert np.array_equal(r32["fail"], r64["fail"])
    assert np.array_equal(r32["rejected_at"], r64["rejected_at"])
    # per-bin acceptance of w = 0 is exactly one (Section 4.1)
    assert np.allclose(r64["p_acc"][w == 0], 1.0, atol=1e-12)
    pick = []
    for k in range(5):
        idx = np.nonzero(w[:2000] == k)[0]
        pick += list(idx[:10])
    ref = oracle_results(circ, ocsr, idx=pick)
    _compare(r64[pick], ref, TOL[MSC_FP64])
    _compare(r32[pick], ref, TOL[MSC_FP32])


def test_c4_81_qubits(ctx):
    cc, c = _cal(ctx, "c4")
    n = 256
    csr = msc.sample_faults(c, 0x5EED0004, 0, n, p=1e-3)
    off, ch, pa = to_dev(*csr)
    say("c4 screen + fp32")
    bits, idx, cnt = msc.prescreen(ctx, c, off, ch, pa)
    res = results_numpy(msc.simulate(ctx, c, off, ch, pa, shot_idx=idx, precision=MSC_FP32))
    assert cnt == len(res) > 10
    assert not np.any(res["status"] & (msc.SHOT_CHI_CAP | msc.SHOT_NOCONV))
    assert np.all(res["chi_peak"] <= 256)
    surv = idx.cpu().numpy()
    w = np.diff(csr[0])[surv]
    # w = 0: the noiseless circuit, for which the oracle gives P_acc = 1, f = 1
    assert np.allclose(res["p_acc"][w == 0], 1.0, atol=1e-5)
    assert np.all(res["infid"][w == 0] < 1e-5)
    circ, ocsr = oracle_csr(cc.text, 0x5EED0004, n, p=1e-3)
    assert _same_csr(csr, ocsr)
    rej = np.nonzero(res["rejected_at"] >= 0)[0]
    early = rej[np.argsort(res["rejected_at"][rej], kind="stable")[:3]]
    ref = oracle_results(circ, ocsr, idx=[int(surv[i]) for i in early])
    _compare(res[early], ref, TOL[MSC_FP32])


def test_screen_81_qubits_2p24_shots(ctx):
    cc = config_circuit("c4")
    c = msc.Circuit(cc.text)
    n = 1 << 24
    csr = msc.sample_faults(c, 0x5EED0005, 0, n, p=1e-3)
    off, ch, pa = to_dev(*csr)
    say("screen 2^24 shots")
    bits, _, cnt = msc.prescreen(ctx, c, off, ch, pa, with_index=False)
    got = bits.cpu().numpy().view(np.uint64)
    circ = parse(cc.text)
    dec, fl = ops.analyse(circ)
    sig = ops.signature_table(circ, dec, fl)
    ref_discard = ops.discard_csr(sig, *csr)
    ref_bits = np.packbits(~ref_discard, bitorder="little").view(np.uint64)
    assert np.array_equal(got, ref_bits)
    assert cnt == int((~ref_discard).sum())
