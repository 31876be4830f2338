"""GPU parity of the wavefront kernel (one shot per wavefront, four per
workgroup, slots of a smaller bond cap).

The kernel runs the op stream of the workgroup kernel with one-wavefront
teams; a shot whose bond would outgrow its slot is run again from its start
by the workgroup kernel.  Per shot against the CPU oracle (P_acc and f within
1e-10 relative in FP64, 1e-5 in FP32, rejection index and failure flag
exact), with caps that never bind (16 on bond-16 circuits), caps that bind
for many shots (4, and 16 on the bond-32 circuit) and the automatic choice.
Prefix forking and the slot count change no bit of a result; the batch path
gives the bin sums of the workgroup kernel up to rounding.
"""
import numpy as np
import pytest

import paper_2609_19116_amd as msc
from paper_2609_19116_amd import MSC_FP32, MSC_FP64, results_numpy
from tests.helpers import oracle_csr, oracle_results, say, to_dev
from tests.test_gpu_parity import TOL, _compare, _same_csr
from workloads.circuits import config_circuit

pytestmark = pytest.mark.gpu

FIELDS = ["p_acc", "infid", "disc_weight", "chi_peak", "status", "rejected_at", "fail", "n2q",
          "flops", "sweeps"]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = msc.Ctx(0)
    yield c
    c.close()


_CIRC = {}
_REF = {}


def _circuit(ctx, name):
    if name not in _CIRC:
        cc = config_circuit(name)
        c = msc.Circuit(cc.text)
        say(f"calibrate {name}")
        c.calibrate(ctx)
        _CIRC[name] = (cc, c)
    return _CIRC[name]


def _stratified(ctx, name, n, seed):
    cc, c = _circuit(ctx, name)
    w = np.arange(n) % 5
    csr = msc.sample_faults(c, seed, 0, n, weights=w)
    key = (name, n, seed)
    if key not in _REF:
        circ, ocsr = oracle_csr(cc.text, seed, n, weights=w)
        assert _same_csr(csr, ocsr)
        _REF[key] = oracle_results(circ, ocsr)
    return c, csr, _REF[key]


@pytest.mark.parametrize("precision", [MSC_FP64, MSC_FP32])
@pytest.mark.parametrize("name,n", [("tiny", 120), ("c1", 160), ("tiny_ghz", 120),
                                    ("c1_ghz", 120)])
def test_wave_kernel_matches_oracle(ctx, name, n, precision):
    c, csr, ref = _stratified(ctx, name, n, 0x5EED0041)
    assert c.noiseless()["chi_peak"] <= 16
    off, ch, pa = to_dev(*csr)
    say(f"wave {name} precision={precision} wave_chi=16")
    res = results_numpy(msc.simulate(ctx, c, off, ch, pa, precision=precision, wave_chi=16))
    st = ctx.engine_stats()
    assert st["wave_slots"] > 0
    _compare(res, ref, TOL[precision])
    assert np.all(res["chi_peak"] <= 16)


@pytest.mark.parametrize("precision", [MSC_FP64, MSC_FP32])
@pytest.mark.parametrize("name,n,cap", [("c1", 160, 4), ("c1_ghz", 120, 2), ("c3", 30, 16)])
def test_wave_kernel_retries_match_oracle(ctx, name, n, cap, precision):
    # the cap binds: the shots that outgrow it run again in the workgroup
    # kernel, from their start
    c, csr, ref = _stratified(ctx, name, n, 0x5EED0042)
    off, ch, pa = to_dev(*csr)
    say(f"wave {name} precision={precision} wave_chi={cap}")
    res = results_numpy(msc.simulate(ctx, c, off, ch, pa, precision=precision, wave_chi=cap))
    st = ctx.engine_stats()
    assert st["wave_slots"] > 0 and st["wave_retries"] > 0
    _compare(res, ref, TOL[precision])
    # the retried shots ran with bonds above the cap
    assert np.any(res["chi_peak"] > cap)


@pytest.mark.parametrize("cap", [16, 4])
def test_wave_prefix_and_slots_change_no_bit(ctx, cap):
    c, csr, ref = _stratified(ctx, "c1", 160, 0x5EED0043)
    off, ch, pa = to_dev(*csr)
    say(f"wave prefix/slots wave_chi={cap}")
    kw = dict(precision=MSC_FP32, wave_chi=cap)
    base = results_numpy(msc.simulate(ctx, c, off, ch, pa, **kw))
    slots = results_numpy(msc.simulate(ctx, c, off, ch, pa, n_slots=7, **kw))
    pf = results_numpy(msc.simulate(ctx, c, off, ch, pa, prefix=True, **kw))
    pf2 = results_numpy(msc.simulate(ctx, c, off, ch, pa, prefix=True, n_slots=5, **kw))
    for f in FIELDS:
        assert np.array_equal(base[f], slots[f]), f
        assert np.array_equal(pf[f], pf2[f]), f
    # a forked shot skips (and does not count) the updates before its fork
    for f in FIELDS[:7]:
        assert np.array_equal(base[f], pf[f]), f
    _compare(base, ref, TOL[MSC_FP32])


def test_wave_kernel_automatic_choice(ctx):
    c, csr, _ = _stratified(ctx, "c1", 160, 0x5EED0041)
    off, ch, pa = to_dev(*csr)
    say("wave automatic choice")
    msc.simulate(ctx, c, off, ch, pa, precision=MSC_FP32)
    assert ctx.engine_stats()["wave_slots"] > 0            # bond-16 circuit: on
    msc.simulate(ctx, c, off, ch, pa, precision=MSC_FP32, lds_width=32)
    assert ctx.engine_stats()["wave_slots"] == 0           # an explicit LDS width: off
    msc.simulate(ctx, c, off, ch, pa, precision=MSC_FP32, wave_chi=-1)
    assert ctx.engine_stats()["wave_slots"] == 0
    c3, csr3, _ = _stratified(ctx, "c3", 30, 0x5EED0042)
    assert c3.noiseless()["chi_peak"] > 16
    o3, h3, p3 = to_dev(*csr3)
    msc.simulate(ctx, c3, o3, h3, p3, precision=MSC_FP32)
    assert ctx.engine_stats()["wave_slots"] == 0           # bond-32 circuit: off
    for bad in (1, -2, 65):
        with pytest.raises(msc.MscError):
            msc.simulate(ctx, c, off, ch, pa, precision=MSC_FP32, wave_chi=bad)


@pytest.mark.parametrize("space_time", [False, True])
def test_wave_batch_matches_workgroup_kernel(ctx, space_time):
    # the whole batch path (sampling, screen, shots, bin sums) with the
    # wavefront kernel and with the workgroup kernel: the same shots, bin sums
    # equal up to FP32 rounding
    cc, c = _circuit(ctx, "c1")
    say(f"wave batch space_time={space_time}")
    kw = dict(n_bins=17, precision=MSC_FP32, space_time=space_time)
    bw, sw = msc.run_batch(ctx, c, 0x5EED0044, 0, 8192, 2e-3, wave_chi=16, **kw)
    assert ctx.engine_stats()["wave_slots"] > 0
    bg, sg = msc.run_batch(ctx, c, 0x5EED0044, 0, 8192, 2e-3, wave_chi=-1, **kw)
    assert ctx.engine_stats()["wave_slots"] == 0
    assert np.array_equal(bw[0], bg[0])                     # shots per weight
    assert sw["n_survivors"] == sg["n_survivors"]
    np.testing.assert_allclose(bw[1], bg[1], rtol=1e-5, atol=1e-12)
    np.testing.assert_allclose(bw[2], bg[2], rtol=1e-4, atol=1e-9)
    if space_time:
        np.testing.assert_allclose(sw["surv_bins"], sg["surv_bins"], rtol=1e-5, atol=1e-12)


def test_wave_kernel_edge_cases(ctx):
    import torch
    c, csr, ref = _stratified(ctx, "c1", 160, 0x5EED0045)
    off, ch, pa = to_dev(*csr)
    say("wave edge cases")
    base = results_numpy(msc.simulate(ctx, c, off, ch, pa, precision=MSC_FP32, wave_chi=16))
    # one slot requested: one workgroup of four wavefronts, same bits
    one = results_numpy(msc.simulate(ctx, c, off, ch, pa, precision=MSC_FP32, wave_chi=16,
                                     n_slots=1))
    for f in FIELDS:
        assert np.array_equal(base[f], one[f]), f
    # BF16x3 runs the FP32 shot kernel (its split products are the engine's);
    # at the same threshold every bit equals the FP32 run
    b3 = results_numpy(msc.simulate(ctx, c, off, ch, pa, precision=msc.MSC_BF16X3,
                                    tau_trunc=1e-4, wave_chi=16))
    f32 = results_numpy(msc.simulate(ctx, c, off, ch, pa, precision=MSC_FP32, tau_trunc=1e-4,
                                     wave_chi=16))
    for f in FIELDS:
        assert np.array_equal(b3[f], f32[f]), f
    # a bond cap below the circuit's bonds binds in the slots themselves: no
    # reruns, the cap flagged as in the workgroup kernel
    capped = results_numpy(msc.simulate(ctx, c, off, ch, pa, precision=MSC_FP64, chi_max=4))
    st = ctx.engine_stats()
    assert st["wave_slots"] > 0 and st["wave_retries"] == 0
    assert np.all(capped["chi_peak"] <= 4)
    assert np.any(capped["status"] & msc.SHOT_CHI_CAP)
    assert np.all(np.isfinite(capped["p_acc"])) and np.all(np.isfinite(capped["infid"]))
    # shot indices outside the CSR give the empty record, as in the workgroup kernel
    idx = torch.tensor([0, -1, 5, 10 ** 9, 7], dtype=torch.int64, device="cuda")
    sel = results_numpy(msc.simulate(ctx, c, off, ch, pa, shot_idx=idx, precision=MSC_FP32,
                                     wave_chi=16))
    assert sel["rejected_at"][1] == -1 and sel["rejected_at"][3] == -1
    assert sel["p_acc"][1] == 0.0 and sel["p_acc"][3] == 0.0 and sel["status"][1] == 0
    for k, i in ((0, 0), (2, 5), (4, 7)):
        for f in FIELDS:
            assert sel[f][k] == base[f][i], (f, i)
