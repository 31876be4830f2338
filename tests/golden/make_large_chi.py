"""Writes the large-bond golden files from the oracle alone.

For a named workload it draws faults with the oracle's sampler twin
(SplitMix64 keyed by seed and shot, a uniform w-subset of the channels and
uniform non-identity Paulis; w given per shot), keeps the shots that the
oracle's offline screen does not discard, runs the oracle's FP64 MPS (LAPACK
SVD, no bond cap) on them in shot order and records P_acc, 1 - f, the
rejecting measurement and the bond peak of every shot until `--accepted`
accepted faulty shots are found.  The noiseless run is recorded first
(P_acc = 1, f = 1 on these deterministic circuits).

    python tests/golden/make_large_chi.py c4 --seed 0x5EED0004 --weight 1
    python tests/golden/make_large_chi.py c3_rainbow --seed 0x5EED0023 --weight 1

Nothing here calls the library: the values are the oracle's.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _run(args):
    name, faults = args
    from oracle import mps as omps
    from oracle.ir import parse
    from workloads.circuits import config_circuit
    circ = parse(config_circuit(name).text)
    t0 = time.time()
    r = omps.run_shot(circ, faults)
    return r.p_acc, r.infid, r.rejected_at, r.chi_peak, time.time() - t0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--seed", type=lambda x: int(x, 0), required=True)
    ap.add_argument("--weight", type=int, default=1)
    ap.add_argument("--candidates", type=int, default=4000,
                    help="shots drawn; the screen keeps a fraction of them")
    ap.add_argument("--accepted", type=int, default=16)
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

    from oracle import prescreen as ops
    from oracle import sampler as osamp
    from oracle.ir import parse
    from workloads.circuits import config_circuit

    text = config_circuit(args.name).text
    circ = parse(text)
    n = args.candidates
    weights = [args.weight] * n
    off, ch, pa = osamp.sample_csr(circ, args.seed, 0, n, weights=weights)
    shots = osamp.csr_to_dicts(off, ch, pa)
    dec, fl = ops.analyse(circ)
    surv = [i for i, f in enumerate(shots) if not ops.discard(dec, fl, f)]
    print(f"{args.name}: {len(surv)} of {n} shots survive the screen", flush=True)

    records = []
    with Pool(args.procs) as pool:
        noiseless = pool.apply(_run, ((args.name, {}),))
        print(f"noiseless: {noiseless}", flush=True)
        assert abs(noiseless[0] - 1.0) < 1e-10 and noiseless[1] < 1e-10
        pos = 0
        n_acc = 0
        while n_acc < args.accepted and pos < len(surv):
            chunk = surv[pos:pos + args.procs]
            pos += len(chunk)
            for i, r in zip(chunk, pool.map(_run, [(args.name, shots[i]) for i in chunk])):
                records.append({"shot": i, "p_acc": r[0], "infid": r[1], "rejected_at": r[2],
                                "chi_peak": r[3]})
                print(f"shot {i}: p_acc {r[0]:.6g} infid {r[1]:.3g} rej {r[2]} chi {r[3]} "
                      f"({r[4]:.0f}s)", flush=True)
            n_acc = sum(1 for x in records if x["p_acc"] > 0)
    acc = [x for x in records if x["p_acc"] > 0]
    assert len(acc) >= args.accepted, "not enough accepted faulty shots among the survivors"
    # keep the simulated shots up to the last needed accepted one
    last = acc[args.accepted - 1]["shot"]
    records = [x for x in records if x["shot"] <= last]
    out = {
        "workload": args.name,
        "seed": hex(args.seed),
        "weight_of_every_shot": args.weight,
        "candidates": n,
        "noiseless": {"p_acc": noiseless[0], "infid": noiseless[1], "chi_peak": noiseless[3]},
        "oracle": "oracle.mps.run_shot (FP64, LAPACK SVD, keep sigma > 1e-12 sigma_0, no cap)",
        "command": " ".join(["python", "tests/golden/make_large_chi.py"] + sys.argv[1:]),
        "shots": records,
    }
    path = os.path.join(HERE, f"large_chi_{args.name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: {len(records)} shots, {len(acc)} accepted", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
