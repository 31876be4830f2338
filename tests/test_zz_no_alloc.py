"""msc_prescreen_noalloc through the C ABI: the offline screen with the
library's fixed per-device scratch instead of allocations, against
msc_prescreen on the same device CSR (bit-exact bitmap, survivor list and
count), on two calls in a row with the second smaller, plus its size and
state errors."""
import ctypes as C

import numpy as np
import pytest

import paper_2609_19116_amd as msc
from paper_2609_19116_amd import _lib
from tests.helpers import say
from workloads.circuits import config_circuit

pytestmark = pytest.mark.gpu

def _noalloc():
    return _lib.lib().msc_prescreen_noalloc


def _screen_noalloc(ctx, circ, off, ch, pa):
    import torch
    n = off.numel() - 1
    bits = torch.full(((n + 63) // 64,), -1, dtype=torch.int64, device=off.device)
    idx = torch.full((max(n, 1),), -7, dtype=torch.int64, device=off.device)
    cnt = C.c_int64(-1)
    rc = _noalloc()(ctx.h, circ.h, n, _lib._ptr(off), _lib._ptr(ch), _lib._ptr(pa),
                    _lib._ptr(bits), _lib._ptr(idx), C.byref(cnt))
    return rc, bits, idx, cnt.value


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = msc.Ctx(0)
    yield c
    c.close()


def test_noalloc_screen_equals_prescreen_twice(ctx):
    c = msc.Circuit(config_circuit("c4").text)
    say("noalloc: calibrate the 81-qubit circuit (uploads its tables)")
    c.calibrate(ctx)
    for seed, n in ((0x5EED0005, 1 << 20), (0x5EED0015, 50_001)):
        off, ch, pa = msc.sample_faults_device(ctx, c, seed, 0, n, p=1e-3)
        say(f"noalloc: screen n={n} seed={seed:#x}")
        ref_bits, ref_idx, ref_cnt = msc.prescreen(ctx, c, off, ch, pa)
        rc, bits, idx, cnt = _screen_noalloc(ctx, c, off, ch, pa)
        assert rc == 0, _lib.lib().msc_last_error().decode()
        assert cnt == ref_cnt > 0
        assert np.array_equal(bits.cpu().numpy(), ref_bits.cpu().numpy())
        assert np.array_equal(idx[:cnt].cpu().numpy(), ref_idx.cpu().numpy())
        # nothing written past the survivors
        assert bool((idx[cnt:] == -7).all())


def test_noalloc_screen_errors(ctx):
    import torch
    c = msc.Circuit(config_circuit("c1").text)
    off = torch.zeros(2, dtype=torch.int64, device="cuda")
    ch = torch.zeros(1, dtype=torch.int32, device="cuda")
    pa = torch.ones(1, dtype=torch.uint8, device="cuda")
    # tables not uploaded yet: a state error, no device work
    rc, _, _, _ = _screen_noalloc(ctx, c, off, ch, pa)
    assert rc == _lib.MSC_E_STATE
    c.calibrate(ctx)
    # above the fixed maximum: rejected on the host
    cnt = C.c_int64()
    rc = _noalloc()(ctx.h, c.h, (1 << 26) + 1, _lib._ptr(off), _lib._ptr(ch), _lib._ptr(pa),
                    _lib._ptr(off), None, C.byref(cnt))
    assert rc == _lib.MSC_E_INVALID
    # a channel index outside the circuit: the kernel's own range check
    # reports it (the index is never used to address a table)
    M = c.info()["n_channels"]
    off = torch.tensor([0, 1], dtype=torch.int64, device="cuda")
    ch = torch.tensor([M + 5], dtype=torch.int32, device="cuda")
    say("noalloc: out-of-range channel")
    rc, _, _, _ = _screen_noalloc(ctx, c, off, ch, pa)
    assert rc == _lib.MSC_E_INVALID
    assert "outside" in _lib.lib().msc_last_error().decode()
    # a valid call right after it still matches the allocating screen
    off, ch, pa = msc.sample_faults_device(ctx, c, 3, 0, 4096, p=1e-2)
    ref_bits, ref_idx, ref_cnt = msc.prescreen(ctx, c, off, ch, pa)
    rc, bits, idx, cnt = _screen_noalloc(ctx, c, off, ch, pa)
    assert rc == 0 and cnt == ref_cnt
    assert np.array_equal(bits.cpu().numpy(), ref_bits.cpu().numpy())
    assert np.array_equal(idx[:cnt].cpu().numpy(), ref_idx.cpu().numpy())
