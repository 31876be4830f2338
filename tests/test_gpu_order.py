"""GPU: the qubit-order search (msc_order_search).

The search's cost is the noiseless run's algorithmic flops under an order
plus fixed costs per product swap, centre move and two-site update of the
compiled op stream; checked here: the contract (a permutation, a cost the calibration
reproduces, no worse than the start, deterministic in the seed), the
optimum of an exhaustive enumeration of all 5040 orders of the 7-qubit
circuit, and that simulating under the order found changes no result:
per-shot P_acc, infidelity and rejection equal the oracle's state vector
(which has no order) on sampled shots.
"""
import itertools

import numpy as np
import pytest

import paper_2609_19116_amd as msc
from paper_2609_19116_amd import MSC_FP64, results_numpy
from tests.helpers import oracle_csr, oracle_results, say
from workloads.circuits import config_circuit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = msc.Ctx(0)
    yield c
    c.close()


def _cost(ctx, text, order):
    c = msc.Circuit(text, order=order)
    c.calibrate(ctx)
    return msc.order_cost(c)


def test_order_search_contract(ctx):
    text = config_circuit("c1").text
    say("order search c1 budget 40")
    order, c0, c1 = msc.order_search(ctx, text, 0x5EED0031, 40)
    n = msc.Circuit(text).info()["n_qubits"]
    assert sorted(order.tolist()) == list(range(n))
    assert c1 <= c0
    assert _cost(ctx, text, order) == c1
    start = np.array(next(ln for ln in text.splitlines() if ln.startswith("ORDER")).split()[1:],
                     dtype=np.int32)
    assert _cost(ctx, text, start) == c0
    again = msc.order_search(ctx, text, 0x5EED0031, 40)
    assert np.array_equal(again[0], order) and again[1:] == (c0, c1)
    # budget 1 only evaluates the start
    o1, a, b = msc.order_search(ctx, text, 1, 1)
    assert np.array_equal(o1, start) and a == b == c0


def test_order_search_against_exhaustive_tiny(ctx):
    text = config_circuit("tiny").text
    n = 7
    say("exhaustive orders of tiny (5040 calibrations)")
    costs = {}
    for perm in itertools.permutations(range(n)):
        costs[perm] = _cost(ctx, text, np.array(perm, dtype=np.int32))
    allc = np.array(sorted(costs.values()))
    say("order search tiny budget 400")
    order, c0, c1 = msc.order_search(ctx, text, 0x5EED0032, 400)
    assert c1 == costs[tuple(order.tolist())]
    # the local search lands in the cheapest 1 % of all orders
    assert c1 <= allc[len(allc) // 100], (c1, allc[0], allc[len(allc) // 100])
    print(f"tiny: start {c0:.4g}  found {c1:.4g}  optimum {allc[0]:.4g}  "
          f"median {np.median(allc):.4g}", flush=True)


def test_results_unchanged_under_found_order(ctx):
    cc = config_circuit("c1")
    say("order search c1 budget 25, then 120 FP64 shots vs the state vector")
    order, _, _ = msc.order_search(ctx, cc.text, 0x5EED0033, 25)
    circ = msc.Circuit(cc.text, order=order)
    circ.calibrate(ctx)
    seed, n = 0x5EED0034, 120
    w = np.array([0, 1, 2, 3] * (n // 4), dtype=np.int32)
    off, ch, pa = msc.sample_faults_device(ctx, circ, seed, 0, n, weights=w)
    res = results_numpy(msc.simulate(ctx, circ, off, ch, pa, precision=MSC_FP64))
    ocirc, ocsr = oracle_csr(cc.text, seed, n, weights=w)
    ref = oracle_results(ocirc, ocsr, engine="sv")
    assert np.allclose(res["p_acc"], ref[:, 0], atol=1e-10, rtol=0)
    acc = ref[:, 0] > 0
    assert np.allclose(res["infid"][acc], ref[acc, 1], atol=1e-10, rtol=0)
    assert np.array_equal(res["rejected_at"], ref[:, 2].astype(np.int32))


def test_order_search_errors(ctx):
    with pytest.raises(msc.MscError):
        msc.order_search(ctx, "QUBITS 2\nCX 0 1\n", 1, 0)        # budget < 1
    with pytest.raises(msc.MscError):
        msc.order_search(ctx, "QUBITS 2\nFOO 0\n", 1, 5)         # parse error
    with pytest.raises(msc.MscError):
        msc.order_search(ctx, "QUBITS 3\nH 0\n", 1, 5, start=[0, 0, 1])


def test_benchmark_layout_changes_no_result(ctx):
    # the 49-qubit workload under the order the benchmark's layout search
    # finds (the benchmark's own procedure and defaults) against its snake
    # order, FP64, sampled shots
    from bench import benchmark_layout
    cc = config_circuit("c3")
    say("benchmark layout search on c3 (3 starts + 4 refinements x 128 evaluations), then "
        "128 FP64 shots on both layouts")
    order, info = benchmark_layout(msc, ctx, cc.text)
    c0, c1 = info["snake_cost"], info["searched_cost"]
    assert c1 <= c0
    snake = msc.Circuit(cc.text)
    snake.calibrate(ctx)
    searched = msc.Circuit(cc.text, order=order)
    searched.calibrate(ctx)
    n = 128
    w = np.array([0, 1, 2, 3] * (n // 4), dtype=np.int32)
    off, ch, pa = msc.sample_faults_device(ctx, snake, 0x5EED0035, 0, n, weights=w)
    a = results_numpy(msc.simulate(ctx, snake, off, ch, pa, precision=MSC_FP64))
    b = results_numpy(msc.simulate(ctx, searched, off, ch, pa, precision=MSC_FP64))
    assert np.array_equal(a["rejected_at"], b["rejected_at"])
    assert np.allclose(a["p_acc"], b["p_acc"], atol=1e-9, rtol=0)
    acc = a["p_acc"] > 0
    assert np.allclose(a["infid"][acc], b["infid"][acc], atol=1e-9, rtol=0)
    assert np.array_equal(a["fail"], b["fail"])
    print(f"c3: order cost snake {c0:.4g} searched {c1:.4g}; mean shot flops "
          f"{a['flops'].mean():.4g} -> {b['flops'].mean():.4g}", flush=True)
