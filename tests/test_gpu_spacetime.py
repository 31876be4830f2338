"""GPU: msc_run_batch in space-time mode (the screen skipped, every shot's
probability of reaching each segment recorded and summed per weight).

Checked: the reach sums equal the oracle's (MPS-oracle reach of the same
shots) on small circuits; the per-weight P_acc sums and counts equal the
screened batch's (skipping the screen changes no result, the online screen
rejects the same shots); checkpoint forking leaves the reach sums bit for
bit; the expected volume from the GPU's sums equals the oracle's.
"""
import numpy as np
import pytest

import paper_2609_19116_amd as msc
from paper_2609_19116_amd import MSC_FP32, MSC_FP64
from oracle import sampler as osamp
from oracle import spacetime as ost
from oracle import mps as omps
from oracle.ir import parse
from tests.helpers import say
from workloads.circuits import config_circuit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = msc.Ctx(0)
    yield c
    c.close()


@pytest.mark.parametrize("name,n,p,prefix", [("c1", 120, 1e-2, False), ("tiny_ghz", 300, 0.03, True)])
def test_reach_sums_match_oracle(ctx, name, n, p, prefix):
    cc = config_circuit(name)
    circ = msc.Circuit(cc.text)
    circ.calibrate(ctx)
    nb, seed = 9, 0x5EED0051
    say(f"space-time run_batch {name} n={n} p={p} prefix={prefix}")
    bins, st = msc.run_batch(ctx, circ, seed, 0, n, p, n_bins=nb, precision=MSC_FP64,
                             prefix=prefix, space_time=True)
    assert st["n_survivors"] == n
    ocirc = parse(cc.text)
    first = [g["first_meas"] for g in ost.segments(ocirc)]
    off, ch, pa = osamp.sample_csr(ocirc, seed, 0, n, p=p)
    shots = osamp.csr_to_dicts(off, ch, pa)
    ref = np.zeros((nb, len(first)))
    for i, f in enumerate(shots):
        r = omps.run_shot(ocirc, f, expected=circ.expected(), record=True)
        w = min(len(f), nb - 1)
        ref[w] += ost.shot_survival(first, r.meas_probs, r.rejected_at >= 0)
    assert np.abs(st["surv_bins"] - ref).max() <= 1e-10 * n
    # the first segment is reached by every shot
    assert np.array_equal(st["surv_bins"][:, 0], bins[0])


def test_space_time_mode_changes_no_result(ctx):
    circ = msc.Circuit(config_circuit("c3").text)
    circ.calibrate(ctx)
    n, p, nb, seed = 2048, 1e-3, 33, 0x5EED0052
    say("space-time vs screened run_batch c3")
    a, sa = msc.run_batch(ctx, circ, seed, 0, n, p, n_bins=nb, precision=MSC_FP32)
    b, sb = msc.run_batch(ctx, circ, seed, 0, n, p, n_bins=nb, precision=MSC_FP32,
                          space_time=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[3:], b[3:])
    assert np.allclose(a[1:3], b[1:3], rtol=0, atol=1e-12)
    assert sb["n_survivors"] == n and sa["n_survivors"] < n
    # forked shots give the same reach sums as shots run from |0...0>
    c, sc = msc.run_batch(ctx, circ, seed, 0, n, p, n_bins=nb, precision=MSC_FP32,
                          space_time=True, prefix=False)
    assert np.array_equal(sb["surv_bins"], sc["surv_bins"])
    assert np.array_equal(b, c)
    # reach is non-increasing along the circuit in every bin
    sv_ = sb["surv_bins"]
    assert np.all(sv_[:, 1:] <= sv_[:, :-1] + 1e-9)
    # expected volume from the GPU's sums equals the oracle's formula
    segs = circ.segments()
    M = circ.info()["n_channels"]
    osegs = ost.segments(parse(config_circuit("c3").text))
    r, v, vb = msc.expected_volume(b[0], sv_, segs, M, p)
    ro, vo, vbo = ost.expected_volume(b[0], sv_, osegs, M, p)
    assert np.allclose(r, ro, rtol=1e-12) and v == pytest.approx(vo, rel=1e-12)
    assert 0 < v <= vb
