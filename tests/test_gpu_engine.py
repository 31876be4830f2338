"""GPU parity of the batched engine for large two-site updates.

The engine takes every two-site update whose theta has a side above
large_side: ragged MFMA contractions, FP64 Gram matrices on MFMA, FP64
Jacobi eigen-decompositions of their overlapping blocks and the new site
tensors, for all parked shots at once.  Forcing it onto small updates
(large_side = 2) runs it on every shape of the small circuits; the results
are compared per shot with the CPU oracle (P_acc and f within 1e-10
relative in FP64, 1e-5 in FP32, rejection index and failure flag exact) and
with the shot kernel alone (large_side = -1); the workgroup kernel runs
every shot here (wave_chi = -1), the one that parks.  Graph replay, the slot
count and prefix forking change no bit of a result.  The 81-qubit circuit reaches bond 64
(theta sides 128) and the 49-qubit circuit on the rainbow layout bond 128
(sides 256); with large_side = 64 the engine takes their wide updates, and
their shots are compared with oracle values stored by
tests/golden/make_large_chi.py.
"""
import json
import os

import numpy as np
import pytest

import paper_2609_19116_amd as msc
from paper_2609_19116_amd import MSC_FP32, MSC_FP64, results_numpy
from tests.helpers import oracle_csr, oracle_results, say, to_dev
from tests.test_gpu_parity import TOL, _compare, _same_csr
from workloads.circuits import config_circuit

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
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


def _circuit(ctx, name):
    if name not in _CIRC:
        cc = config_circuit(name)
        c = msc.Circuit(cc.text)
        say(f"calibrate {name}")
        c.calibrate(ctx)
        _CIRC[name] = (cc, c)
    return _CIRC[name]


_REF = {}


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
def test_engine_on_every_update_matches_oracle(ctx, name, n, precision):
    c, csr, ref = _stratified(ctx, name, n, 0x5EED0031)
    off, ch, pa = to_dev(*csr)
    say(f"engine {name} precision={precision} large_side=2")
    res = results_numpy(msc.simulate(ctx, c, off, ch, pa, precision=precision, large_side=2,
                                     wave_chi=-1))
    st = ctx.engine_stats()
    assert st["updates"] > 0 and st["contract_flops"] > 0 and st["gram_flops"] > 0
    _compare(res, ref, TOL[precision])
    say(f"shot kernel alone {name} precision={precision}")
    alone = results_numpy(msc.simulate(ctx, c, off, ch, pa, precision=precision,
                                       large_side=-1, wave_chi=-1))
    assert ctx.engine_stats()["updates"] == 0
    acc = alone["p_acc"] > 0
    # the two factorisations may pick different bases of degenerate singular
    # subspaces (the SVD gauge), which can change later centre moves and so
    # the update count, never a gauge-invariant result
    assert np.array_equal(res["rejected_at"], alone["rejected_at"])
    assert np.array_equal(res["fail"], alone["fail"])
    rel = np.abs(res["p_acc"] - alone["p_acc"])[acc] / alone["p_acc"][acc]
    assert rel.max() <= TOL[precision]


@pytest.mark.parametrize("lds_width", [32, 64])
def test_engine_graphs_and_prefix_change_no_bit(ctx, lds_width):
    c, csr, ref = _stratified(ctx, "c1", 160, 0x5EED0032)
    off, ch, pa = to_dev(*csr)
    say(f"engine graphs/prefix lds_width={lds_width}")
    kw = dict(precision=MSC_FP32, large_side=4, lds_width=lds_width, wave_chi=-1)
    base = results_numpy(msc.simulate(ctx, c, off, ch, pa, **kw))
    assert ctx.engine_stats()["rounds"] > 0
    g1 = results_numpy(msc.simulate(ctx, c, off, ch, pa, use_graphs=True, **kw))
    g2 = results_numpy(msc.simulate(ctx, c, off, ch, pa, use_graphs=True, **kw))
    pf = results_numpy(msc.simulate(ctx, c, off, ch, pa, prefix=True, **kw))
    slots = results_numpy(msc.simulate(ctx, c, off, ch, pa, n_slots=7, **kw))
    for other in (g1, g2, slots):
        for f in FIELDS:
            assert np.array_equal(base[f], other[f]), f
    # a forked shot skips (and does not count) the updates before its fork
    for f in FIELDS[:7]:
        assert np.array_equal(base[f], pf[f]), f
    _compare(base, ref, TOL[MSC_FP32])


@pytest.mark.parametrize("precision", [MSC_FP64, MSC_FP32])
def test_engine_c3_stratified(ctx, precision):
    c, csr, ref = _stratified(ctx, "c3", 30, 0x5EED0033)
    off, ch, pa = to_dev(*csr)
    say(f"engine c3 precision={precision} large_side=8")
    res = results_numpy(msc.simulate(ctx, c, off, ch, pa, precision=precision, large_side=8,
                                     wave_chi=-1))
    assert ctx.engine_stats()["updates"] > 0
    _compare(res, ref, TOL[precision])


def _golden(name):
    with open(os.path.join(GOLDEN, f"large_chi_{name}.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("precision", [MSC_FP64, MSC_FP32])
@pytest.mark.parametrize("use_graphs", [False, True])
@pytest.mark.parametrize("name,chi", [("c4", 64), ("c3_rainbow", 128)])
def test_engine_golden_large_bonds(ctx, name, chi, precision, use_graphs):
    # the 81-qubit circuit (bond 64) and the 49-qubit circuit on the rainbow
    # layout (bond 128), shots stored by the oracle-only golden script
    import torch
    g = _golden(name)
    assert g["noiseless"]["chi_peak"] == chi
    cc, c = _circuit(ctx, name)
    n = g["candidates"]
    w = np.full(n, g["weight_of_every_shot"], dtype=np.int32)
    csr = msc.sample_faults(c, int(g["seed"], 16), 0, n, weights=w)
    shots = [s["shot"] for s in g["shots"]]
    ref = np.array([(s["p_acc"], s["infid"], s["rejected_at"]) for s in g["shots"]])
    assert sum(1 for s in g["shots"] if s["p_acc"] > 0) >= 16
    off, ch, pa = to_dev(*csr)
    idx = torch.tensor(shots, dtype=torch.int64, device="cuda")
    say(f"engine golden {name} precision={precision} graphs={use_graphs}")
    res = results_numpy(msc.simulate(ctx, c, off, ch, pa, shot_idx=idx, precision=precision,
                                     use_graphs=use_graphs, large_side=64, wave_chi=-1))
    assert ctx.engine_stats()["updates"] > 0
    _compare(res, ref, TOL[precision])
    acc = ref[:, 0] > 0
    assert np.all(res["chi_peak"][acc] >= chi)
    assert not np.any(res["status"] & (msc.SHOT_CHI_CAP | msc.SHOT_NOCONV))


def test_autotune_cache_roundtrip_and_tile_independence(ctx, tmp_path):
    # the autotuner times every tile shape per bucket and writes the JSON
    # cache; any tile shape leaves each output's summation order unchanged,
    # so the results under the tuned shapes are bit-identical
    c, csr, ref = _stratified(ctx, "c1", 160, 0x5EED0034)
    off, ch, pa = to_dev(*csr)
    path = tmp_path / "tune.json"
    say("autotune FP32 and FP64")
    e32 = msc.autotune(ctx, MSC_FP32, reps=2, cache_path=path)
    e64 = msc.autotune(ctx, MSC_FP64, reps=2, cache_path=path)
    doc = json.loads(path.read_text())
    assert {(e["precision"], e["bucket"]) for e in doc["entries"]} == \
        {(p, b) for p in (MSC_FP32, MSC_FP64) for b in range(4)}
    for e in e32 + e64:
        assert e["rows"] > 0 and e["b"] > 0 and e["gram"] > 0 and e["contract_us"] > 0
    kw = dict(precision=MSC_FP32, large_side=4, wave_chi=-1)
    base = results_numpy(msc.simulate(ctx, c, off, ch, pa, **kw))
    tuned = results_numpy(msc.simulate(ctx, c, off, ch, pa, autotune_cache=path, **kw))
    for f in FIELDS:
        assert np.array_equal(base[f], tuned[f]), f
    _compare(tuned, ref, TOL[MSC_FP32])
    with pytest.raises(msc.MscError):
        msc.simulate(ctx, c, off, ch, pa, autotune_cache=tmp_path / "missing.json", **kw)
    bad = tmp_path / "bad.json"
    bad.write_text('{"entries": [{"precision": 1, "bucket": 0, "rows": 48, "b": 32, "gram": 64}]}')
    with pytest.raises(msc.MscError):
        msc.simulate(ctx, c, off, ch, pa, autotune_cache=bad, **kw)


@pytest.mark.parametrize("name,chi", [("c4", 64), ("c3_rainbow", 128)])
def test_engine_bf16x3_golden_large_bonds(ctx, name, chi):
    # BF16x3 split-precision contractions in the engine (FP32 tensors, FP64
    # Gram and factorisation): the error against the FP64 oracle is stated
    # by the method at ~1e-5 relative; checked at 1e-4
    import torch
    g = _golden(name)
    cc, c = _circuit(ctx, name)
    n = g["candidates"]
    w = np.full(n, g["weight_of_every_shot"], dtype=np.int32)
    csr = msc.sample_faults(c, int(g["seed"], 16), 0, n, weights=w)
    ref = np.array([(s["p_acc"], s["infid"], s["rejected_at"]) for s in g["shots"]])
    off, ch, pa = to_dev(*csr)
    idx = torch.tensor([s["shot"] for s in g["shots"]], dtype=torch.int64, device="cuda")
    say(f"engine golden {name} BF16x3")
    res = results_numpy(msc.simulate(ctx, c, off, ch, pa, shot_idx=idx,
                                     precision=msc.MSC_BF16X3, large_side=64, wave_chi=-1))
    assert ctx.engine_stats()["updates"] > 0
    _compare(res, ref, 1e-4)
    acc = ref[:, 0] > 0
    assert np.all(res["chi_peak"][acc] >= chi)


# gate ids of msc_engine_update and the oracle's 4x4 matrices over |q_A q_B>
_ENGINE_GATES = {2: "CX", 4: "CZ", 1: "SWAP", 5: "CS"}


def _theta(A, B, gname):
    """theta = G (A B) in FP64 as the (chi_l 2) x (2 chi_r) matrix, from the
    oracle's gate matrix."""
    from oracle.gates import G2
    g = G2[gname].reshape(2, 2, 2, 2)
    pre = np.einsum("aic,cjb->aijb", A, B)
    th = np.einsum("xyij,aijb->axyb", g, pre)
    cl, cr = A.shape[0], B.shape[2]
    return th.reshape(2 * cl, 2 * cr)


@pytest.mark.parametrize("precision,tau,tol", [(MSC_FP64, 1e-12, 1e-12), (MSC_FP32, 1e-5, 2e-5),
                                               (msc.MSC_BF16X3, 1e-4, 1e-4)])
@pytest.mark.parametrize("dir", [1, 0])
@pytest.mark.parametrize("cl,cm,cr,gid", [(64, 40, 48, 2), (24, 16, 20, 4), (16, 24, 40, 1)])
def test_engine_update_against_lapack_svd(ctx, precision, tau, tol, dir, cl, cm, cr, gid):
    """One batched engine update on random tensors whose theta has a rank
    below both sides (the CX and CZ products have operator Schmidt rank 2,
    so rank <= 2 chi_m; SWAP: <= 4 chi_m): the kept bond is LAPACK's
    numerical rank at the same threshold, A' B' reproduces theta / |theta|,
    the isometric factor is isometric and the other factor's norms are
    LAPACK's singular values (all to `tol`, relative to sigma_0).  theta's
    sides 128 x 96 flag more than 64 overlapping vectors (the workspace
    route); the others fewer (the LDS eigen-decomposition, whose rotated
    vectors are polished by one-sided Jacobi: without it, null directions
    kept norms near eps sigma_0^3 / sigma_min^2 and passed the threshold)."""
    rng = np.random.default_rng(0x5EED0051 + 7 * cl + dir)
    batch = 5
    A = rng.normal(size=(batch, cl, 2, cm)) + 1j * rng.normal(size=(batch, cl, 2, cm))
    B = rng.normal(size=(batch, cm, 2, cr)) + 1j * rng.normal(size=(batch, cm, 2, cr))
    A /= np.sqrt(cl * cm)
    B /= np.sqrt(cm * cr)
    say(f"engine update precision={precision} dir={dir} shape={cl}x{cm}x{cr} gate={gid}")
    outa, outb = msc.engine_update(ctx, A, B, dir, gid, 1024, tau, precision=precision)
    for i in range(batch):
        th = _theta(A[i], B[i], _ENGINE_GATES[gid])
        s = np.linalg.svd(th, compute_uv=False)
        r = int(np.sum(s > tau * s[0]))
        a, b = outa[i], outb[i]
        assert a.shape[2] == r and b.shape[0] == r, (i, a.shape, b.shape, r)
        U = a.reshape(2 * cl, r)
        V = b.reshape(r, 2 * cr)
        nk = np.sqrt(np.sum(s[:r] ** 2))
        err = np.linalg.norm(U @ V - th / nk) / np.linalg.norm(th / nk)
        assert err <= tol, (i, err)
        if dir:
            iso = np.abs(U.conj().T @ U - np.eye(r)).max()
            sv = np.linalg.norm(V, axis=1)
        else:
            iso = np.abs(V @ V.conj().T - np.eye(r)).max()
            sv = np.linalg.norm(U, axis=0)
        assert iso <= tol, (i, iso)
        dev = np.abs(np.sort(sv)[::-1] - s[:r] / nk).max() / (s[0] / nk)
        assert dev <= tol, (i, dev)
        if i == 0:
            say(f"  r={r} reconstruction {err:.2e} isometry {iso:.2e} sigma {dev:.2e}")


def test_engine_update_degenerate_spectrum(ctx):
    """theta with all singular values equal (isometric A and B, the
    stabiliser-like case): nothing overlaps, every vector is kept, and the
    factors reproduce theta."""
    cl, cm, cr = 32, 64, 32
    A = np.eye(2 * cl, cm).reshape(1, cl, 2, cm).astype(np.complex128)
    B = np.eye(cm, 2 * cr).reshape(1, cm, 2, cr).astype(np.complex128)
    for precision in (MSC_FP64, MSC_FP32):
        outa, outb = msc.engine_update(ctx, A, B, 1, 2, 1024, 1e-12 if precision == MSC_FP64
                                       else 1e-5, precision=precision)
        th = _theta(A[0], B[0], "CX")
        a, b = outa[0], outb[0]
        assert a.shape[2] == 64
        U, V = a.reshape(2 * cl, 64), b.reshape(64, 2 * cr)
        assert np.abs(U @ V - th / np.linalg.norm(th)).max() <= 1e-6


def test_engine_update_errors(ctx):
    A = np.zeros((1, 4, 2, 4), dtype=np.complex128)
    B = np.zeros((1, 4, 2, 4), dtype=np.complex128)
    for kw in ({"dir": 2, "gate": 2}, {"dir": 1, "gate": 9}):
        with pytest.raises(RuntimeError):
            msc.engine_update(ctx, A, B, kw["dir"], kw["gate"], 16, 1e-12)
    with pytest.raises(RuntimeError):
        msc.engine_update(ctx, A, B, 1, 2, 16, 0.0)
