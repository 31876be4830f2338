"""GPU: CAMPS shots (msc_simulate_camps) against the oracles.

The method is exact, so P_acc, the infidelity and the rejecting
measurement must equal the state vector's (small circuits) and the plain
MPS path's (larger ones); the residual's peak bond must equal the dense
CAMPS oracle's, which makes the same greedy choices; a Clifford circuit
keeps the residual a product state; the residual needs no larger bond
than the plain MPS on the noiseless run.
"""
import numpy as np
import pytest

import paper_2609_19116_amd as msc
from paper_2609_19116_amd import MSC_FP64, results_numpy
from oracle import camps as ocamps
from oracle import sampler as osamp
from oracle import statevector as sv
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


def _circ(ctx, name, target="T"):
    cc = config_circuit(name, target=target)
    c = msc.Circuit(cc.text)
    c.calibrate(ctx)
    return cc, c


@pytest.mark.parametrize("name", ["tiny", "tiny_ghz"])
def test_camps_equals_oracles_small(ctx, name):
    cc, circ = _circ(ctx, name)
    seed, n = 0x5EED0071, 24
    w = np.array([0, 1, 2, 3] * (n // 4), dtype=np.int32)
    say(f"camps {name} n={n}")
    off, ch, pa = msc.sample_faults_device(ctx, circ, seed, 0, n, weights=w)
    res = results_numpy(msc.simulate_camps(ctx, circ, off, ch, pa))
    ocirc = parse(cc.text)
    o_off, o_ch, o_pa = osamp.sample_csr(ocirc, seed, 0, n, weights=w)
    for i, f in enumerate(osamp.csr_to_dicts(o_off, o_ch, o_pa)):
        ref = sv.run_shot(ocirc, f)
        oc = ocamps.run_shot(ocirc, f)
        r = res[i]
        assert r["status"] & msc.SHOT_DONE or r["rejected_at"] >= 0
        assert r["rejected_at"] == ref.rejected_at, i
        assert abs(r["p_acc"] - ref.p_acc) < 1e-10, i
        if ref.p_acc > 0:
            assert abs(r["infid"] - ref.infid) < 1e-10, i
        assert r["chi_peak"] == oc.chi_peak, (i, r["chi_peak"], oc.chi_peak)


@pytest.mark.parametrize("name,n", [("c1", 160), ("c1_ghz", 96), ("c3", 48)])
def test_camps_equals_mps_path(ctx, name, n):
    cc, circ = _circ(ctx, name)
    seed = 0x5EED0072
    w = np.array([0, 1, 2, 3] * (n // 4), dtype=np.int32)
    say(f"camps vs mps {name} n={n}")
    off, ch, pa = msc.sample_faults_device(ctx, circ, seed, 0, n, weights=w)
    a = results_numpy(msc.simulate_camps(ctx, circ, off, ch, pa))
    b = results_numpy(msc.simulate(ctx, circ, off, ch, pa, precision=MSC_FP64))
    assert not (a["status"] & msc.SHOT_CHI_CAP).any()
    assert np.array_equal(a["rejected_at"], b["rejected_at"])
    assert np.allclose(a["p_acc"], b["p_acc"], atol=1e-9, rtol=0)
    acc = b["p_acc"] > 0
    assert np.allclose(a["infid"][acc], b["infid"][acc], atol=1e-9, rtol=0)
    assert np.array_equal(a["fail"], b["fail"])
    # the noiseless shot (w = 0): the residual needs no larger bond
    assert a["chi_peak"][0] <= b["chi_peak"][0]
    print(f"{name}: noiseless chi_peak camps {a['chi_peak'][0]} mps {b['chi_peak'][0]}; "
          f"max camps {a['chi_peak'].max()} mps {b['chi_peak'].max()}; "
          f"camps {ctx.last_kernel_ms('camps'):.1f} ms", flush=True)


@pytest.mark.parametrize("name,n", [("c1", 400), ("c3", 256)])
def test_camps_prefix_bit_identical(ctx, name, n):
    cc, circ = _circ(ctx, name)
    say(f"camps prefix {name} n={n}")
    off, ch, pa = msc.sample_faults_device(ctx, circ, 0x5EED0074, 0, n, p=3e-3)
    a = results_numpy(msc.simulate_camps(ctx, circ, off, ch, pa))
    ta = ctx.last_kernel_ms("camps")
    b = results_numpy(msc.simulate_camps(ctx, circ, off, ch, pa, prefix=True))
    tb = ctx.last_kernel_ms("camps")
    for f in ("p_acc", "infid", "chi_peak", "status", "rejected_at", "fail", "n2q", "sweeps"):
        assert np.array_equal(a[f], b[f]), f
    print(f"{name}: {ta:.1f} ms from |0...0>, {tb:.1f} ms forked", flush=True)


def test_camps_clifford_circuit_has_product_residual(ctx):
    cc, circ = _circ(ctx, "c1", target="S")
    n = 64
    w = np.array([0, 1, 2, 3] * (n // 4), dtype=np.int32)
    say("camps |S> c1")
    off, ch, pa = msc.sample_faults_device(ctx, circ, 0x5EED0073, 0, n, weights=w)
    a = results_numpy(msc.simulate_camps(ctx, circ, off, ch, pa))
    assert (a["chi_peak"] == 1).all()
    b = results_numpy(msc.simulate(ctx, circ, off, ch, pa, precision=MSC_FP64))
    assert np.allclose(a["p_acc"], b["p_acc"], atol=1e-10, rtol=0)


def test_camps_argument_errors(ctx):
    import torch
    cc, circ = _circ(ctx, "tiny")
    off, ch, pa = msc.sample_faults_device(ctx, circ, 1, 0, 4, weights=np.zeros(4, np.int32))
    with pytest.raises(msc.MscError):
        msc.simulate_camps(ctx, circ, off, ch, pa, chi_max=64)
    raw = msc.Circuit(cc.text)
    with pytest.raises(msc.MscError):
        msc.simulate_camps(ctx, raw, off, ch, pa)          # not calibrated
    out = msc.simulate_camps(ctx, circ, off, ch, pa,
                             shot_idx=torch.tensor([0, 9, -1], dtype=torch.int64, device="cuda"))
    r = results_numpy(out)
    assert r["status"][1] == 0 and r["status"][2] == 0 and r["status"][0] & msc.SHOT_DONE


def test_camps_cap_reruns_on_mps(ctx):
    """A residual bond cap that binds (2 here, on the 17-qubit circuit whose
    residual reaches 4) no longer ends the shot with P_acc 0: the shot is
    run again by the FP64 MPS path, whose record it then carries bit for
    bit (flagged MSC_SHOT_MPS_RERUN); every shot still equals the MPS path
    to 1e-10.  Forking needs the noiseless residual within the cap."""
    import torch
    cc, circ = _circ(ctx, "c1")
    seed, n = 0x5EED0072, 96
    w = np.array([0, 1, 2, 3] * (n // 4), dtype=np.int32)
    off, ch, pa = msc.sample_faults_device(ctx, circ, seed, 0, n, weights=w)
    prefix = False
    say("camps cap 2")
    res = results_numpy(msc.simulate_camps(ctx, circ, off, ch, pa, chi_max=2, prefix=prefix))
    mps = results_numpy(msc.simulate(ctx, circ, off, ch, pa, precision=MSC_FP64, chi_max=256,
                                     wave_chi=-1, prefix=prefix))
    rerun = (res["status"] & msc.SHOT_MPS_RERUN) != 0
    assert rerun.sum() >= 10, rerun.sum()
    assert not np.any(res["status"][~rerun] & msc.SHOT_CHI_CAP)
    for f in ("p_acc", "infid", "disc_weight", "chi_peak", "rejected_at", "fail", "n2q"):
        assert np.array_equal(res[f][rerun], mps[f][rerun]), f
    assert np.array_equal(res["status"][rerun], mps["status"][rerun] | msc.SHOT_MPS_RERUN)
    assert np.array_equal(res["rejected_at"], mps["rejected_at"])
    acc = mps["p_acc"] > 0
    assert np.abs(res["p_acc"] - mps["p_acc"])[acc].max() <= 1e-10 * mps["p_acc"][acc].max()
    # a selection of shots (device shot_idx) reruns the selected shot ids
    idx = torch.tensor(np.nonzero(rerun)[0][:5], dtype=torch.int64, device="cuda")
    sub = results_numpy(msc.simulate_camps(ctx, circ, off, ch, pa, shot_idx=idx, chi_max=2,
                                           prefix=prefix))
    assert np.all(sub["status"] & msc.SHOT_MPS_RERUN)
    assert np.array_equal(sub["p_acc"], mps["p_acc"][idx.cpu().numpy()])
    with pytest.raises(msc.MscError):
        msc.simulate_camps(ctx, circ, off, ch, pa, chi_max=2, prefix=True)
