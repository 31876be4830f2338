"""GPU: the fused batch entry point against the separate stages and the oracle.

msc_run_batch runs sampling, screen, shots and the per-weight reduction on
one stream; its per-shot results must equal those of the separate calls bit
for bit, its bins the sums of those results, and its bins the oracle's on a
small circuit.  The accepted / wrong counts of rows 3 and 4 are compared
exactly with the oracle's acceptance draws applied to the same per-shot
results, and to the oracle's own results.
"""
import threading

import numpy as np
import pytest

import paper_2609_19116_amd as msc
from oracle import estimators as est
from paper_2609_19116_amd import MSC_FP32, MSC_FP64, results_numpy
from oracle import stats as ostats
from tests.helpers import oracle_csr, oracle_results, say
from workloads.circuits import config_circuit

pytestmark = pytest.mark.gpu

FIELDS = ("p_acc", "infid", "disc_weight", "chi_peak", "status", "rejected_at", "fail")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = msc.Ctx(0)
    yield c
    c.close()


def _separate(ctx, circ, seed, first, n, p, nb, **kw):
    """Bins from the separate stages: the sums of the per-shot results and
    the oracle's acceptance counts of those results."""
    import torch
    off, ch, pa = msc.sample_faults_device(ctx, circ, seed, first, n, p=p)
    bits, idx, cnt = msc.prescreen(ctx, circ, off, ch, pa)
    per = np.zeros(n, dtype=msc.SHOT_DTYPE)
    per["rejected_at"] = -1
    if cnt:
        res = results_numpy(msc.simulate(ctx, circ, off, ch, pa, shot_idx=idx, **kw))
        per[idx.cpu().numpy()] = res
    w = np.minimum(np.diff(off.cpu().numpy()), nb - 1)
    bins = np.zeros((7, nb))
    np.add.at(bins[0], w, 1.0)
    np.add.at(bins[1], w, per["p_acc"])
    np.add.at(bins[2], w, per["p_acc"] * per["fail"])
    _, bins[3], bins[4] = ostats.count_bins(seed, first, w, per["p_acc"], per["fail"], nb)
    np.add.at(bins[5], w, per["p_acc"] ** 2)
    np.add.at(bins[6], w, (per["p_acc"] * per["fail"]) ** 2)
    return bins, per, int(ch.numel()), cnt


@pytest.mark.parametrize("name,n,p,precision,prefix", [
    ("c1", 3000, 1e-2, MSC_FP64, False),
    ("c1_ghz", 2000, 1e-2, MSC_FP32, True),
    ("c3", 4096, 1e-3, MSC_FP32, True),
    ("tiny", 777, 0.05, MSC_FP64, True),
])
def test_run_batch_equals_separate_stages(ctx, name, n, p, precision, prefix):
    import torch
    circ = msc.Circuit(config_circuit(name).text)
    circ.calibrate(ctx)
    nb = 33
    seed, first = 0x5EED000B, 1000
    say(f"run_batch {name} n={n} p={p} precision={precision} prefix={prefix}")
    out = torch.empty(n * msc.SHOT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    bins, st = msc.run_batch(ctx, circ, seed, first, n, p, n_bins=nb, precision=precision,
                             prefix=prefix, out=out)
    ref_bins, per, nnz, cnt = _separate(ctx, circ, seed, first, n, p, nb, precision=precision,
                                        prefix=prefix)
    got = results_numpy(out)
    for f in FIELDS:
        assert np.array_equal(got[f], per[f]), f
    assert np.array_equal(bins[0], ref_bins[0])
    assert np.allclose(bins[1:3], ref_bins[1:3], rtol=1e-12, atol=1e-12)
    assert np.array_equal(bins[3:5], ref_bins[3:5])
    assert np.allclose(bins[5:7], ref_bins[5:7], rtol=1e-12, atol=1e-12)
    assert st["n_shots"] == n and st["nnz"] == nnz and st["n_survivors"] == cnt
    assert st["n_accepted"] == int((per["p_acc"] > 0).sum())
    assert st["n2q"] == int(per["n2q"].sum()) and st["chi_peak"] == int(per["chi_peak"].max())
    # a second call gives the same bits
    bins2, _ = msc.run_batch(ctx, circ, seed, first, n, p, n_bins=nb, precision=precision,
                             prefix=prefix)
    assert np.array_equal(bins, bins2)


def test_run_batch_bins_match_oracle(ctx):
    cc = config_circuit("c1")
    circ = msc.Circuit(cc.text)
    circ.calibrate(ctx)
    n, p, nb, seed = 150, 1e-2, 9, 0x5EED000C
    say("run_batch c1 vs oracle bins")
    bins, _ = msc.run_batch(ctx, circ, seed, 0, n, p, n_bins=nb, precision=MSC_FP64)
    ocirc, ocsr = oracle_csr(cc.text, seed, n, p=p)
    ref = oracle_results(ocirc, ocsr)        # screened shots carry P_acc 0
    w = np.minimum(np.diff(ocsr[0]), nb - 1)
    fail = (ref[:, 0] > 0) & (ref[:, 1] > 1e-4)
    rb = np.zeros((7, nb))
    np.add.at(rb[0], w, 1.0)
    np.add.at(rb[1], w, ref[:, 0])
    np.add.at(rb[2], w, ref[:, 0] * fail)
    _, rb[3], rb[4] = ostats.count_bins(seed, 0, w, ref[:, 0], fail, nb)
    np.add.at(rb[5], w, ref[:, 0] ** 2)
    np.add.at(rb[6], w, (ref[:, 0] * fail) ** 2)
    assert np.array_equal(bins[0], rb[0])
    assert np.abs(bins[1:3] - rb[1:3]).max() <= 1e-10 * n
    assert np.abs(bins[5:7] - rb[5:7]).max() <= 1e-10 * n
    # the counts take the same decision u < P_acc on both sides
    assert np.array_equal(bins[3:5], rb[3:5])
    # standard errors of Eq. (reweight) from the GPU's sums equal the oracle's
    M = circ.info()["n_channels"]
    for pp in (5e-4, 1e-3, 2e-3):
        got = msc.reweight(bins[0], bins[1], bins[2], M, [pp], bins[5], bins[6])[0]
        sa, se = est.standard_errors(list(rb[0]), list(rb[1]), list(rb[2]), M, pp,
                                     list(rb[5]), list(rb[6]))
        assert got["sem_p_acc"] == pytest.approx(sa, rel=1e-8)
        assert got["sem_p_acc_le"] == pytest.approx(se, rel=1e-8, abs=1e-15)
    assert bins[3].sum() > 0
    # the likelihood-ratio intervals from the GPU's counts equal the oracle's
    last = int(np.nonzero(rb[0])[0].max()) + 1
    pb = ostats.Problem(rb[0][:last], rb[3][:last], rb[4][:last], M, p)
    for f in (msc.MSC_STAT_PACC, msc.MSC_STAT_PLE):
        r = msc.lr_interval(bins[0][:last], bins[3][:last], bins[4][:last], M, p, f)
        o = ostats.lr_interval(pb, f)
        assert (r["estimate"], r["lo"], r["hi"], r["hi_trunc"]) == pytest.approx(
            o, rel=1e-8, abs=1e-12)


def test_run_batch_on_concurrent_contexts(ctx):
    circ = msc.Circuit(config_circuit("c3").text)
    circ.calibrate(ctx)
    n, p = 4096, 1e-3
    say("run_batch on 3 contexts in threads")
    ref = [msc.run_batch(ctx, circ, 0x5EED000D, b * n, n, p)[0] for b in range(3)]
    ctxs = [msc.Ctx(0) for _ in range(3)]
    got = [None] * 3

    def work(i):
        got[i] = msc.run_batch(ctxs[i], circ, 0x5EED000D, i * n, n, p)[0]

    th = [threading.Thread(target=work, args=(i,)) for i in range(3)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for c in ctxs:
        c.close()
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_run_batch_argument_errors(ctx):
    circ = msc.Circuit(config_circuit("tiny").text)
    with pytest.raises(msc.MscError):
        msc.run_batch(ctx, circ, 1, 0, 10, 0.1)          # not calibrated
    circ.calibrate(ctx)
    for kw in ({"n_bins": 0}, {"n_bins": 2000}):
        with pytest.raises(msc.MscError):
            msc.run_batch(ctx, circ, 1, 0, 10, 0.1, **kw)
    with pytest.raises(msc.MscError):
        msc.run_batch(ctx, circ, 1, 0, 10, 1.5)
    bins, st = msc.run_batch(ctx, circ, 1, 0, 0, 0.1, n_bins=4)
    assert not bins.any() and st["n_shots"] == 0
