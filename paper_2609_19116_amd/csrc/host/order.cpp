// Search for the qubit -> MPS-site order.
//
// Section 3.1: an MPS needs a linear order of the qubits, and a poor order
// both lengthens the routing of two-qubit gates and raises the bond
// dimension; the paper picks its layouts by hand and names an automatic
// search as future work.  Here the cost of an order is what the simulation
// actually spends on it: the algorithmic flops (as the shot kernel counts
// them) of the circuit's noiseless run compiled with that order, evaluated
// on the GPU by the calibration run, plus a fixed cost per op of the
// compiled stream (product swaps, centre moves, two-site updates): the shot
// kernel is latency-bound, and an op's latency, not its flops, dominates
// the small ops that routing adds.  An order whose noiseless run exceeds
// the kernel's bond cap costs +inf.
//
// The search is a first-improvement local search from the start order:
// each step proposes one move between two sites i and j -- exchange them,
// reverse the run between them, or move site i to j (one third each) --
// drawn from a SplitMix64 stream (Steele, Lea, Flood 2014) keyed by the
// seed, and keeps it iff the cost falls.  The distance |i - j| is
// 1 + floor(-4 ln u) for a uniform u (mean 5, beyond 16 in 2 % of the
// moves): mostly local moves, whose candidates' noiseless runs cost about
// as much as the current one's, with the occasional long move that lets
// the search leave a local optimum.  Every proposal costs one evaluation;
// the search stops after `budget` evaluations.
#include <algorithm>
#include <cmath>
#include <vector>

#include "../msc_internal.h"

namespace {

struct Mix {
    uint64_t s;
    explicit Mix(uint64_t seed) : s(seed) {}
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    // uniform in [0, n) by rejection of the biased top range
    int below(int n) {
        const uint64_t lim = ~0ull - (~0ull % static_cast<uint64_t>(n));
        uint64_t x;
        do x = next();
        while (x >= lim);
        return static_cast<int>(x % static_cast<uint64_t>(n));
    }
};

}  // namespace

using namespace msc;

// flops of the calibrated circuit's noiseless run plus the fixed op costs
static double calibrated_cost(const msc_circuit* c) {
    return c->noiseless.flops + MSC_ORDER_COST_PSWAP * static_cast<double>(c->n_product_swaps) +
           MSC_ORDER_COST_MOVE * static_cast<double>(c->n_moves) +
           MSC_ORDER_COST_TWOSITE * static_cast<double>(c->n_twosite);
}

extern "C" int msc_order_cost(const msc_circuit* c, double* out) {
    if (!c || !out) return set_error(MSC_E_INVALID, "null argument");
    if (!c->calibrated) return set_error(MSC_E_STATE, "circuit not calibrated");
    *out = calibrated_cost(c);
    return MSC_OK;
}

// cost of one order: flops of the noiseless run plus the fixed op costs,
// +inf if it cannot run
static int order_cost(msc_ctx* ctx, const char* text, size_t len, const std::vector<int32_t>& order,
                      double* cost) {
    msc_circuit* c = nullptr;
    int rc = msc_circuit_load(text, len, order.data(), &c);
    if (rc) return rc;
    rc = msc_circuit_calibrate(ctx, c);
    if (rc == MSC_OK)
        *cost = calibrated_cost(c);
    else if (rc == MSC_E_NONDETERMINISTIC && (c->noiseless.status & MSC_SHOT_CHI_CAP)) {
        *cost = INFINITY;
        rc = MSC_OK;
    }
    msc_circuit_free(c);
    return rc;
}

extern "C" int msc_order_search(msc_ctx* ctx, const char* text, size_t len,
                                const int32_t* start, uint64_t seed, int32_t budget,
                                int32_t* order_out, double* cost_out) {
    if (!ctx || !text || !order_out || !cost_out || budget < 1)
        return set_error(MSC_E_INVALID, "null argument or budget < 1");
    msc_circuit* c0 = nullptr;
    int rc = msc_circuit_load(text, len, start, &c0);
    if (rc) return rc;
    std::vector<int32_t> cur = c0->order;
    msc_circuit_free(c0);
    const int n = static_cast<int>(cur.size());
    double best;
    if ((rc = order_cost(ctx, text, len, cur, &best))) return rc;
    cost_out[0] = best;
    Mix rng(seed ^ 0x6F72646572ull);
    for (int32_t ev = 1; ev < budget && n >= 2; ++ev) {
        std::vector<int32_t> cand = cur;
        const int kind = rng.below(3);
        int i = rng.below(n);
        const double u = (static_cast<double>(rng.next() >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        const int d = std::min(n - 1, 1 + static_cast<int>(-4.0 * std::log(u)));
        int j = rng.below(2) ? i + d : i - d;
        if (j < 0 || j >= n) j = (j < 0) ? i + d : i - d;
        j = std::max(0, std::min(n - 1, j));
        if (j == i) j = i + 1 < n ? i + 1 : i - 1;
        if (kind == 0) {
            std::swap(cand[i], cand[j]);
        } else if (kind == 1) {
            if (i > j) std::swap(i, j);
            std::reverse(cand.begin() + i, cand.begin() + j + 1);
        } else {
            const int32_t q = cand[i];
            cand.erase(cand.begin() + i);
            cand.insert(cand.begin() + j, q);
        }
        double cost;
        if ((rc = order_cost(ctx, text, len, cand, &cost))) return rc;
        if (cost < best) {
            best = cost;
            cur = cand;
        }
    }
    std::copy(cur.begin(), cur.end(), order_out);
    cost_out[1] = best;
    return MSC_OK;
}

extern "C" int msc_circuit_noiseless(const msc_circuit* c, msc_shot_result* out) {
    if (!c || !out) return set_error(MSC_E_INVALID, "null argument");
    if (!c->calibrated) return set_error(MSC_E_STATE, "circuit not calibrated");
    *out = c->noiseless;
    return MSC_OK;
}
