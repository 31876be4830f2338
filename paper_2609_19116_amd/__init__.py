"""Batched exact-MPS simulation of noisy magic-state-cultivation shots on
MI355X: Python binding of the C ABI in include/msc.h.

The functions below have the names of the C entry points (without the
``msc_`` prefix) and only marshal arguments; every step of the method runs
in libmsc.so (host C++ and HIP kernels for gfx950).  Device arrays are torch
tensors on the context's GPU.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from ._lib import (BatchStats, EngineStats, TuneEntry, MSC_BF16X3, MSC_FP32, MSC_FP64, MSC_STAT_PACC,  # noqa: F401
                   MSC_ORDER_COST_MOVE, MSC_ORDER_COST_PSWAP, MSC_ORDER_COST_TWOSITE,
                   MSC_STAT_PLE, SEGMENT_DTYPE, SHOT_CHI_CAP, SHOT_DONE, SHOT_DTYPE, SHOT_NOCONV, SHOT_MPS_RERUN,
                   SHOT_REJECTED, CircuitInfo, Estimate, Interval, MscError, SimOpts, _check,
                   _ptr, lib)

__all__ = ["Ctx", "Circuit", "sample_faults", "sample_faults_device", "prescreen", "simulate",
           "simulate_camps", "camps_candidates",
           "run_batch", "reweight", "profile_loglik", "lr_interval", "ratio_credible",
           "loss_factor", "expected_volume", "order_search", "twosite_contract", "engine_update", "prescreen_tables",
           "autotune", "version", "MscError",
           "MSC_FP64", "MSC_FP32", "MSC_BF16X3", "order_cost", "MSC_STAT_PACC", "MSC_STAT_PLE", "SHOT_DTYPE"]


def version() -> str:
    return lib().msc_version().decode()


class Ctx:
    """msc_ctx: one GPU, one stream, device scratch.  ``stream`` (optional) is
    a torch.cuda.Stream of that GPU for the context to run on; by default
    the context creates a stream of its own."""

    def __init__(self, device: int = 0, stream=None):
        h = C.c_void_p()
        raw = None if stream is None else C.c_void_p(stream.cuda_stream)
        _check(lib().msc_ctx_create(device, raw, C.byref(h)))
        self.h = h
        self.device = device
        self.stream = stream

    def close(self) -> None:
        if self.h:
            lib().msc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_kernel_ms(self, which: str) -> float:
        return lib().msc_ctx_last_kernel_ms(self.h, which.encode())

    def engine_stats(self) -> dict:
        """msc_ctx_engine_stats: the large-update engine in the last shot run."""
        st = EngineStats()
        _check(lib().msc_ctx_engine_stats(self.h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in EngineStats._fields_}


class Circuit:
    """msc_circuit: parsed and compiled circuit."""

    def __init__(self, text: str, order=None):
        h = C.c_void_p()
        b = text.encode()
        o = None
        if order is not None:
            o = np.ascontiguousarray(order, dtype=np.int32)
        _check(lib().msc_circuit_load(b, len(b), _ptr(o), C.byref(h)))
        self.h = h

    def __del__(self):
        try:
            if self.h:
                lib().msc_circuit_free(self.h)
                self.h = None
        except Exception:
            pass

    def info(self) -> dict:
        i = CircuitInfo()
        _check(lib().msc_circuit_get_info(self.h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in CircuitInfo._fields_}

    def expected(self) -> np.ndarray:
        out = np.zeros(self.info()["n_meas"], dtype=np.uint8)
        _check(lib().msc_circuit_expected(self.h, _ptr(out)))
        return out

    def calibrate(self, ctx: Ctx) -> None:
        _check(lib().msc_circuit_calibrate(ctx.h, self.h))

    def segments(self) -> np.ndarray:
        """The circuit's segments (SEGMENT_DTYPE records)."""
        n = C.c_int32()
        lib().msc_circuit_segments(self.h, 0, None, C.byref(n))
        out = np.zeros(n.value, dtype=SEGMENT_DTYPE)
        _check(lib().msc_circuit_segments(self.h, n.value, _ptr(out), C.byref(n)))
        return out

    def noiseless(self) -> dict:
        """The calibration's noiseless-run record (bond peak, updates, flops)."""
        r = np.zeros(1, dtype=SHOT_DTYPE)
        _check(lib().msc_circuit_noiseless(self.h, _ptr(r)))
        return {k: r[k][0].item() for k in SHOT_DTYPE.names}


def order_search(ctx: Ctx, text: str, seed: int, budget: int, start=None):
    """Local search for the qubit -> site order; returns (order int32 [n],
    start cost, best cost) with cost = flops of the noiseless run plus the
    fixed op costs (order_cost)."""
    b = text.encode()
    st = None if start is None else np.ascontiguousarray(start, dtype=np.int32)
    n = Circuit(text).info()["n_qubits"]
    out = np.zeros(n, dtype=np.int32)
    cost = np.zeros(2, dtype=np.float64)
    _check(lib().msc_order_search(ctx.h, b, len(b), _ptr(st), seed, budget, _ptr(out),
                                  _ptr(cost)))
    return out, float(cost[0]), float(cost[1])


def order_cost(circ: Circuit) -> float:
    """msc_order_cost: the order-search cost of a calibrated circuit."""
    out = C.c_double()
    _check(lib().msc_order_cost(circ.h, C.byref(out)))
    return out.value


def sample_faults(circ: Circuit, seed: int, first_shot: int, n_shots: int,
                  weights=None, p: float = 0.0):
    """Host CSR (shot_off int64, chan int32, pauli uint8) of the shots."""
    off = np.zeros(n_shots + 1, dtype=np.int64)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.int32)
    cap = max(16, 4 * n_shots)
    while True:
        chan = np.zeros(cap, dtype=np.int32)
        pa = np.zeros(cap, dtype=np.uint8)
        nnz = C.c_int64()
        rc = lib().msc_sample_faults(circ.h, seed, first_shot, n_shots, _ptr(w), p, _ptr(off),
                                     _ptr(chan), _ptr(pa), cap, C.byref(nnz))
        if rc == -4:   # capacity: retry with the size the library asked for
            cap = nnz.value
            continue
        _check(rc)
        return off, chan[:nnz.value].copy(), pa[:nnz.value].copy()


def sample_faults_device(ctx: Ctx, circ: Circuit, seed: int, first_shot: int, n_shots: int,
                         weights=None, p: float = 0.0, nnz_cap=None):
    """Device CSR (shot_off int64, chan int32, pauli uint8 torch tensors on
    the context's GPU), bit-identical to sample_faults.  ``weights`` may be
    a host array or a device int32 tensor."""
    import torch
    dev = torch.device("cuda", ctx.device)
    M = circ.info()["n_channels"]
    w = None
    if weights is not None:
        if isinstance(weights, torch.Tensor):
            w = weights.to(device=dev, dtype=torch.int32).contiguous()
            need = int(w.clamp(0, M).sum().item()) if n_shots else 0
        else:
            wn = np.ascontiguousarray(weights, dtype=np.int32)
            need = int(np.clip(wn[:n_shots], 0, M).sum())
            w = torch.from_numpy(wn).to(dev)
        cap = need if nnz_cap is None else nnz_cap
    else:
        mean = n_shots * M * p
        cap = int(mean + 8.0 * np.sqrt(mean + 1.0) + 64) if nnz_cap is None else nnz_cap
    off = torch.empty(n_shots + 1, dtype=torch.int64, device=dev)
    while True:
        chan = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        pa = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
        nnz = C.c_int64()
        rc = lib().msc_sample_faults_device(ctx.h, circ.h, seed, first_shot, n_shots, _ptr(w), p,
                                            _ptr(off), _ptr(chan), _ptr(pa), cap, C.byref(nnz))
        if rc == -4 and nnz_cap is None:   # capacity: retry with the exact size
            cap = nnz.value
            continue
        _check(rc)
        return off, chan[:nnz.value], pa[:nnz.value]


def prescreen_tables(circ: Circuit):
    """(sig uint64[6*M, words], decided int32[n_decided])."""
    inf = circ.info()
    sig = np.zeros((6 * inf["n_channels"], inf["words"]), dtype=np.uint64)
    dec = np.zeros(max(1, inf["n_decided"]), dtype=np.int32)
    _check(lib().msc_prescreen_tables(circ.h, _ptr(sig), _ptr(dec)))
    return sig, dec[:inf["n_decided"]]


def prescreen(ctx: Ctx, circ: Circuit, off, chan, pauli, with_index: bool = True):
    """Device screen: returns (survive_bits uint64 tensor, survivor index
    int64 tensor or None, count)."""
    import torch
    n = off.numel() - 1
    dev = off.device
    bits = torch.zeros((n + 63) // 64, dtype=torch.int64, device=dev)
    idx = torch.empty(max(n, 1), dtype=torch.int64, device=dev) if with_index else None
    cnt = C.c_int64()
    _check(lib().msc_prescreen(ctx.h, circ.h, n, _ptr(off), _ptr(chan), _ptr(pauli), _ptr(bits),
                               _ptr(idx), C.byref(cnt)))
    return bits, (idx[:cnt.value] if idx is not None else None), cnt.value


def _opts(precision, chi_max, tau_trunc, tau_rej, tau_fail, n_slots, lds_width, prefix,
          large_side=0, use_graphs=False, autotune_cache=None, wave_chi=0) -> SimOpts:
    cache = None if autotune_cache is None else str(autotune_cache).encode()
    return SimOpts(precision, chi_max, tau_trunc, tau_rej, tau_fail, n_slots, lds_width,
                   1 if prefix else 0, large_side, 1 if use_graphs else 0, wave_chi, cache)


def simulate(ctx: Ctx, circ: Circuit, off, chan, pauli, shot_idx=None, precision=MSC_FP64,
             chi_max: int = 256, tau_trunc: float = 0.0, tau_rej: float = 1e-6,
             tau_fail: float = 1e-4, n_slots: int = 0, lds_width: int = 0, prefix: bool = False,
             out=None, large_side: int = 0, use_graphs: bool = False, autotune_cache=None,
             wave_chi: int = 0):
    """Simulate shots (device CSR); returns a uint8 device tensor holding
    msc_shot_result records (view them with ``results_numpy``).
    ``large_side`` (0: 256, -1: off) hands wider two-site updates to the
    batched engine; ``use_graphs`` replays its rounds from a HIP graph;
    ``autotune_cache`` names an msc_autotune file of tile shapes;
    ``wave_chi`` (0: automatic, -1: off) runs one shot per wavefront in
    slots of that bond cap."""
    import torch
    n_shots = off.numel() - 1
    n = shot_idx.numel() if shot_idx is not None else n_shots
    if out is None:
        out = torch.empty(max(n, 1) * SHOT_DTYPE.itemsize, dtype=torch.uint8, device=off.device)
    o = _opts(precision, chi_max, tau_trunc, tau_rej, tau_fail, n_slots, lds_width, prefix,
              large_side, use_graphs, autotune_cache, wave_chi)
    _check(lib().msc_simulate(ctx.h, circ.h, C.byref(o), n_shots, _ptr(off), _ptr(chan),
                              _ptr(pauli), _ptr(shot_idx), n, _ptr(out)))
    return out[: n * SHOT_DTYPE.itemsize]


def simulate_camps(ctx: Ctx, circ: Circuit, off, chan, pauli, shot_idx=None,
                   chi_max: int = 32, tau_trunc: float = 0.0, tau_rej: float = 1e-6,
                   tau_fail: float = 1e-4, n_slots: int = 0, prefix: bool = False, out=None):
    """Simulate shots with the Clifford-augmented MPS (FP64); same records
    as ``simulate`` with chi_peak the magic residual's peak bond.  With
    ``prefix`` shots fork from checkpoints of the noiseless CAMPS run."""
    import torch
    n_shots = off.numel() - 1
    n = shot_idx.numel() if shot_idx is not None else n_shots
    if out is None:
        out = torch.empty(max(n, 1) * SHOT_DTYPE.itemsize, dtype=torch.uint8, device=off.device)
    o = _opts(MSC_FP64, chi_max, tau_trunc, tau_rej, tau_fail, n_slots, 0, prefix)
    _check(lib().msc_simulate_camps(ctx.h, circ.h, C.byref(o), n_shots, _ptr(off), _ptr(chan),
                                    _ptr(pauli), _ptr(shot_idx), n, _ptr(out)))
    return out[: n * SHOT_DTYPE.itemsize]


def camps_candidates():
    """The disentangler's 19 candidates: (unitaries complex [19, 4, 4],
    Pauli maps uint8 [19, 16])."""
    n = C.c_int32()
    _check(lib().msc_camps_candidates(None, None, C.byref(n)))
    m = np.zeros(32 * n.value, dtype=np.float64)
    t = np.zeros(16 * n.value, dtype=np.uint8)
    _check(lib().msc_camps_candidates(_ptr(m), _ptr(t), C.byref(n)))
    u = m.reshape(n.value, 16, 2)
    return (u[..., 0] + 1j * u[..., 1]).reshape(n.value, 4, 4), t.reshape(n.value, 16)


def run_batch(ctx: Ctx, circ: Circuit, seed: int, first_shot: int, n_shots: int, p: float,
              n_bins: int = 65, precision=MSC_FP32, chi_max: int = 256, tau_trunc: float = 0.0,
              tau_rej: float = 1e-6, tau_fail: float = 1e-4, n_slots: int = 0,
              lds_width: int = 0, prefix: bool = True, out=None, space_time: bool = False,
              large_side: int = 0, use_graphs: bool = False, autotune_cache=None,
              wave_chi: int = 0):
    """One batch of the whole path (sampling, screen, shots, bin sums) on the
    context's stream with one synchronisation.  Returns (bins float64
    [7, n_bins]: shots, sum P_acc, sum P_acc * fail, accepted count, wrong
    count, sum P_acc^2, sum (P_acc * fail)^2 per weight; stats dict).  With ``space_time`` the offline screen
    is skipped and stats["surv_bins"] holds float64 [n_bins, n_seg]: per
    weight the summed probabilities of reaching each segment.
    ``out`` (optional uint8 device tensor of n_shots records) receives the
    per-shot results, indexed by shot."""
    o = _opts(precision, chi_max, tau_trunc, tau_rej, tau_fail, n_slots, lds_width, prefix,
              large_side, use_graphs, autotune_cache, wave_chi)
    bins = np.zeros(7 * n_bins, dtype=np.float64)
    st = BatchStats()
    if out is not None:
        assert out.numel() >= n_shots * SHOT_DTYPE.itemsize
    surv = None
    if space_time:
        surv = np.zeros(n_bins * len(circ.segments()), dtype=np.float64)
    _check(lib().msc_run_batch(ctx.h, circ.h, C.byref(o), seed, first_shot, n_shots, p, n_bins,
                               _ptr(bins), C.byref(st), _ptr(out), _ptr(surv)))
    stats = {f: getattr(st, f) for f, _ in BatchStats._fields_}
    if space_time:
        stats["surv_bins"] = surv.reshape(n_bins, -1)
    return bins.reshape(7, n_bins), stats


def results_numpy(out) -> np.ndarray:
    return np.frombuffer(out.cpu().numpy().tobytes(), dtype=SHOT_DTYPE)


def twosite_contract(ctx: Ctx, chi: int, batch: int, A, B, gate, theta,
                     precision: int = MSC_FP32) -> None:
    _check(lib().msc_twosite_contract(ctx.h, precision, chi, batch, _ptr(A), _ptr(B), _ptr(gate),
                                      _ptr(theta)))


def engine_update(ctx: Ctx, A, B, dir: int, gate: int, chi_max: int, tau: float,
                  precision: int = MSC_FP64):
    """msc_engine_update: one two-site update per batch element through the
    batched engine.  A: complex (batch, chi_l, 2, chi_m), B: complex (batch,
    chi_m, 2, chi_r) (numpy); returns the lists of new A' (chi_l, 2, r) and
    B' (r, 2, chi_r) as complex numpy arrays."""
    A = np.asarray(A)
    B = np.asarray(B)
    batch, cl, _, cm = A.shape
    cr = B.shape[3]
    assert B.shape == (batch, cm, 2, cr)
    planar = lambda X: np.ascontiguousarray(
        np.stack([X.real, X.imag], axis=1).reshape(X.shape[0], -1), dtype=np.float64)
    a, b = planar(A), planar(B)
    rmax = min(chi_max, 2 * min(cl, cr))
    ao = np.zeros((batch, 2, cl * 2 * rmax))
    bo = np.zeros((batch, 2, rmax * 2 * cr))
    r = np.zeros(batch, dtype=np.int32)
    _check(lib().msc_engine_update(ctx.h, precision, cl, cm, cr, batch, dir, gate, chi_max, tau,
                                   _ptr(a), _ptr(b), _ptr(ao), _ptr(bo), _ptr(r)))
    outa, outb = [], []
    for i in range(batch):
        k = int(r[i])
        outa.append((ao[i, 0, :cl * 2 * k] + 1j * ao[i, 1, :cl * 2 * k]).reshape(cl, 2, k))
        outb.append((bo[i, 0, :k * 2 * cr] + 1j * bo[i, 1, :k * 2 * cr]).reshape(k, 2, cr))
    return outa, outb


def autotune(ctx: Ctx, precision: int = MSC_FP32, reps: int = 5, cache_path=None) -> list:
    """msc_autotune: the engine's fastest tile shapes per bucket of theta
    sides (written to ``cache_path`` as JSON if given)."""
    out = (TuneEntry * 4)()
    path = None if cache_path is None else str(cache_path).encode()
    _check(lib().msc_autotune(ctx.h, precision, reps, path, C.cast(out, C.c_void_p)))
    return [{f: getattr(o, f) for f, _ in TuneEntry._fields_} for o in out]


def reweight(bin_n, bin_acc, bin_fail, M: int, p_grid, bin_acc2=None, bin_fail2=None) -> list:
    """Eq. (reweight) per p, with standard errors (from the sums of squares
    when given, else the [0, 1] variance bound)."""
    n = np.ascontiguousarray(bin_n, dtype=np.float64)
    a = np.ascontiguousarray(bin_acc, dtype=np.float64)
    e = np.ascontiguousarray(bin_fail, dtype=np.float64)
    a2 = None if bin_acc2 is None else np.ascontiguousarray(bin_acc2, dtype=np.float64)
    e2 = None if bin_fail2 is None else np.ascontiguousarray(bin_fail2, dtype=np.float64)
    pg = np.ascontiguousarray(p_grid, dtype=np.float64)
    out = (Estimate * len(pg))()
    _check(lib().msc_reweight(_ptr(n), _ptr(a), _ptr(e), _ptr(a2), _ptr(e2), len(n), M,
                              _ptr(pg), len(pg), C.cast(out, C.c_void_p)))
    return [{f: getattr(o, f) for f, _ in Estimate._fields_} for o in out]


def _counts(bin_n, bin_acc, bin_err):
    return tuple(np.ascontiguousarray(x, dtype=np.float64) for x in (bin_n, bin_acc, bin_err))


def profile_loglik(bin_n, bin_acc, bin_err, M: int, p: float, functional: int, theta: float,
                   d_e: int = 0) -> float:
    n, k, m = _counts(bin_n, bin_acc, bin_err)
    out = C.c_double()
    _check(lib().msc_profile_loglik(_ptr(n), _ptr(k), _ptr(m), len(n), M, p, d_e, functional,
                                    theta, C.byref(out)))
    return out.value


def lr_interval(bin_n, bin_acc, bin_err, M: int, p: float, functional: int, R: float = 100.0,
                d_e: int = 0) -> dict:
    n, k, m = _counts(bin_n, bin_acc, bin_err)
    out = Interval()
    _check(lib().msc_lr_interval(_ptr(n), _ptr(k), _ptr(m), len(n), M, p, d_e, functional, R,
                                 C.byref(out)))
    return {f: getattr(out, f) for f, _ in Interval._fields_}


def ratio_credible(bin_n, bin_acc, bin_err, M: int, p: float, s_acc: float, s_err: float,
                   level: float = 0.95, h: float = 2e-3, d_e: int = 0):
    n, k, m = _counts(bin_n, bin_acc, bin_err)
    lo, hi = C.c_double(), C.c_double()
    _check(lib().msc_ratio_credible(_ptr(n), _ptr(k), _ptr(m), len(n), M, p, d_e, s_acc, s_err,
                                    level, h, C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def expected_volume(bin_n, surv_bins, segs, M: int, p: float):
    """(reach probability per segment, expected volume of the noisy
    segments, the same plus the truncation bound) at error rate p."""
    n = np.ascontiguousarray(bin_n, dtype=np.float64)
    sv = np.ascontiguousarray(surv_bins, dtype=np.float64)
    sg = np.ascontiguousarray(segs, dtype=SEGMENT_DTYPE)
    reach = np.zeros(len(sg))
    vol = np.zeros(2)
    _check(lib().msc_expected_volume(_ptr(n), _ptr(sv), len(n), _ptr(sg), len(sg), M, p,
                                     _ptr(reach), _ptr(vol)))
    return reach, float(vol[0]), float(vol[1])


def loss_factor(M: int, p_loss: float) -> float:
    out = C.c_double()
    _check(lib().msc_loss_factor(M, p_loss, C.byref(out)))
    return out.value
