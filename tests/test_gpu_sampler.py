"""GPU parity of the device fault sampler (Section 4.1, subset sampling).

The device CSR must equal the host sampler's bit for bit; the host sampler
is itself checked against the oracle's twin on the CPU.
"""
import ctypes as C

import numpy as np
import pytest

import paper_2609_19116_amd as msc
from paper_2609_19116_amd import _lib
from tests.helpers import oracle_csr, say
from workloads.circuits import config_circuit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = msc.Ctx(0)
    yield c
    c.close()


def _host(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("name,seed,first,n,p,weights", [
    ("c1", 0x5EED0001, 3, 1000, 1e-3, None),
    ("c1", 0x5EED0002, 0, 777, 0.0, "w04"),
    ("c3", 0x5EED0003, 4096, 4096, 1e-3, None),
    ("c4", 0x5EED0004, 0, 3001, 1e-3, None),
    ("c1_ghz", 0x5EED0006, 11, 2500, 2e-2, None),
    ("tiny", 17, 0, 4097, 0.2, None),
    ("c1", 5, 0, 300, 0.0, "heavy"),
    ("tiny", 9, 0, 1, 1.0, None),
])
def test_device_sampler_equals_host(ctx, name, seed, first, n, p, weights):
    circ = msc.Circuit(config_circuit(name).text)
    M = circ.info()["n_channels"]
    w = None
    if weights == "w04":
        w = (np.arange(n) % 5).astype(np.int32)
    elif weights == "heavy":                 # weights up to and past M
        w = np.linspace(0, M + 20, n).astype(np.int32)
    say(f"device sampler {name} n={n} p={p} weights={weights}")
    d = msc.sample_faults_device(ctx, circ, seed, first, n, weights=w, p=p)
    h = msc.sample_faults(circ, seed, first, n, weights=w, p=p)
    for a, b in zip(d, h):
        assert np.array_equal(_host(a), b)


def test_device_sampler_matches_oracle_directly(ctx):
    cc = config_circuit("c1_ghz")
    circ = msc.Circuit(cc.text)
    n = 400
    say("device sampler vs oracle twin c1_ghz")
    d = msc.sample_faults_device(ctx, circ, 0x5EED0007, 5, n, p=3e-2)
    _, ref = oracle_csr(cc.text, 0x5EED0007, n, p=3e-2, first=5)
    for a, b in zip(d, ref):
        assert np.array_equal(_host(a), b)


def test_device_sampler_large_batch(ctx):
    circ = msc.Circuit(config_circuit("c3").text)
    n = 1 << 21
    say(f"device sampler c3 n={n}")
    d = msc.sample_faults_device(ctx, circ, 0x5EED0008, 0, n, p=2e-3)
    h = msc.sample_faults(circ, 0x5EED0008, 0, n, p=2e-3)
    for a, b in zip(d, h):
        assert np.array_equal(_host(a), b)


def test_device_sampler_capacity_and_empty(ctx):
    import torch
    circ = msc.Circuit(config_circuit("c1").text)
    n, cap, guard = 64, 40, 64
    w = torch.full((n,), 3, dtype=torch.int32, device="cuda")
    off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    chan = torch.full((cap + guard,), -7, dtype=torch.int32, device="cuda")
    pa = torch.full((cap + guard,), 200, dtype=torch.uint8, device="cuda")
    nnz = C.c_int64()
    say("device sampler capacity error")
    rc = _lib.lib().msc_sample_faults_device(ctx.h, circ.h, 1, 0, n, w.data_ptr(), 0.0,
                                             off.data_ptr(), chan.data_ptr(), pa.data_ptr(),
                                             cap, C.byref(nnz))
    assert rc == _lib.MSC_E_CAPACITY and nnz.value == 3 * n
    assert np.array_equal(_host(off), 3 * np.arange(n + 1))
    assert np.all(_host(chan)[cap:] == -7) and np.all(_host(pa)[cap:] == 200)
    h = msc.sample_faults(circ, 1, 0, n, weights=np.full(n, 3))
    k = cap // 3 * 3                          # whole shots that fit
    assert np.array_equal(_host(chan)[:k], h[1][:k])
    off0 = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    rc = _lib.lib().msc_sample_faults_device(ctx.h, circ.h, 1, 0, 0, None, 0.1, off0.data_ptr(),
                                             None, None, 0, C.byref(nnz))
    assert rc == 0 and nnz.value == 0 and int(off0.item()) == 0
