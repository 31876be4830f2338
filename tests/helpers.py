"""Shared test helpers: oracle runs on CSR shot lists and GPU plumbing."""
from __future__ import annotations

import sys

import numpy as np

from oracle import mps as omps
from oracle import prescreen as ops
from oracle import sampler as osamp
from oracle import statevector as sv
from oracle.ir import parse


def say(*a) -> None:
    """Print and flush the case before a GPU step."""
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_csr(text: str, seed: int, n: int, weights=None, p: float = 0.0, first: int = 0):
    circ = parse(text)
    return circ, osamp.sample_csr(circ, seed, first, n, weights=weights, p=p)


def oracle_results(circ, csr, engine: str = "mps", idx=None):
    """Per-shot (p_acc, infid, rejected_at) from the oracle."""
    off, ch, pa = csr
    shots = osamp.csr_to_dicts(off, ch, pa)
    eng = omps if engine == "mps" else sv
    out = []
    for i in (range(len(shots)) if idx is None else idx):
        r = eng.run_shot(circ, shots[i])
        out.append((r.p_acc, r.infid, r.rejected_at))
    return np.array(out, dtype=np.float64)


def oracle_discards(circ, csr) -> np.ndarray:
    dec, fl = ops.analyse(circ)
    off, ch, pa = csr
    return np.array([ops.discard(dec, fl, f) for f in osamp.csr_to_dicts(off, ch, pa)])


def to_dev(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]
