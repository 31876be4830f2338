"""GPU: shots forked from checkpoints of the noiseless run.

A shot that forks from the checkpoint before its first fault skips only
fault-free ops that it would have run with the same kernel and arithmetic,
so every per-shot result must be bit-identical to the run from |0...0>;
the forked run must also still match the oracle.
"""
import numpy as np
import pytest

import paper_2609_19116_amd as msc
from paper_2609_19116_amd import MSC_FP32, MSC_FP64, results_numpy
from tests.helpers import oracle_csr, oracle_results, say, to_dev
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


@pytest.mark.parametrize("name,precision,lds_width,n,p", [
    ("c1", MSC_FP64, 0, 600, 1e-2),
    ("c1", MSC_FP32, 0, 600, 1e-2),
    ("c1_ghz", MSC_FP64, 0, 400, 1e-2),
    ("c3", MSC_FP32, 32, 1024, 1e-3),
    ("c3", MSC_FP32, 64, 512, 1e-3),
    ("c3", MSC_FP64, 32, 256, 2e-3),
    ("tiny", MSC_FP64, 0, 2000, 0.05),
])
def test_forked_shots_bit_identical(ctx, name, precision, lds_width, n, p):
    circ = msc.Circuit(config_circuit(name).text)
    circ.calibrate(ctx)
    off, ch, pa = msc.sample_faults_device(ctx, circ, 0x5EED0009, 0, n, p=p)
    bits, idx, cnt = msc.prescreen(ctx, circ, off, ch, pa)
    say(f"prefix {name} precision={precision} lds={lds_width} survivors={cnt}")
    kw = dict(shot_idx=idx, precision=precision, lds_width=lds_width)
    ref = results_numpy(msc.simulate(ctx, circ, off, ch, pa, **kw))
    got = results_numpy(msc.simulate(ctx, circ, off, ch, pa, prefix=True, **kw))
    say(f"  prefix build {ctx.last_kernel_ms('prefix'):.2f} ms")
    for f in FIELDS:
        assert np.array_equal(got[f], ref[f]), f
    assert got["n2q"].sum() < ref["n2q"].sum()
    w = np.diff(off.cpu().numpy())[idx.cpu().numpy()]
    if (w == 0).any():                         # fault-free shots only read out
        assert got["n2q"][w == 0].max() == 0


def test_forked_shots_match_oracle(ctx):
    cc = config_circuit("c1")
    circ = msc.Circuit(cc.text)
    circ.calibrate(ctx)
    n = 120
    w = np.arange(n) % 5
    csr = msc.sample_faults(circ, 0x5EED000A, 0, n, weights=w)
    ocirc, ocsr = oracle_csr(cc.text, 0x5EED000A, n, weights=w)
    ref = oracle_results(ocirc, ocsr)
    say("prefix c1 vs oracle")
    for prec, tol in ((MSC_FP64, 1e-10), (MSC_FP32, 1e-5)):
        res = results_numpy(msc.simulate(ctx, circ, *to_dev(*csr), precision=prec, prefix=True))
        assert np.abs(res["p_acc"] - ref[:, 0]).max() <= tol
        acc = ref[:, 0] > 0
        assert np.abs(res["infid"] - ref[:, 1])[acc].max() <= tol
        assert np.array_equal(res["rejected_at"], ref[:, 2].astype(np.int32))


def test_prefix_rebuilt_when_options_change(ctx):
    circ = msc.Circuit(config_circuit("tiny").text)
    circ.calibrate(ctx)
    off, ch, pa = msc.sample_faults_device(ctx, circ, 3, 0, 300, p=0.05)
    say("prefix option changes")
    outs = []
    for prec, tau in ((MSC_FP64, 0.0), (MSC_FP32, 0.0), (MSC_FP64, 1e-9)):
        a = results_numpy(msc.simulate(ctx, circ, off, ch, pa, precision=prec, tau_trunc=tau))
        b = results_numpy(msc.simulate(ctx, circ, off, ch, pa, precision=prec, tau_trunc=tau,
                                       prefix=True))
        for f in FIELDS:
            assert np.array_equal(a[f], b[f]), (prec, tau, f)
        outs.append(b)
    circ.calibrate(ctx)                       # drops the checkpoints
    c = results_numpy(msc.simulate(ctx, circ, off, ch, pa, precision=MSC_FP64, prefix=True))
    assert np.array_equal(c["p_acc"], outs[0]["p_acc"])
