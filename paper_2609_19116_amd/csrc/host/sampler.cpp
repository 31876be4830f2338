// Subset-sampling fault draws (Section 4.1) and Eq. (reweight).
//
// Faults are a pure function of (seed, shot index): SplitMix64 (Steele, Lea,
// Flood 2014) seeded with mix(seed ^ mix(shot)), Lemire's bounded integers,
// Floyd's uniform w-subset, and, when no weights are given, w drawn from
// Bin(M, p) by inverting an FP64 cumulative table built with the ratio
// recurrence from (1-p)^M (repeated squaring).  Every step uses only IEEE
// basic operations, so the draws are bit-reproducible across machines.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "../msc_internal.h"

namespace msc {
namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Rng {
    uint64_t s;
    Rng(uint64_t seed, uint64_t shot) : s(mix64(seed ^ mix64(shot))) {}
    uint64_t next() {
        s += kGolden;
        return mix64(s);
    }
    uint64_t bounded(uint64_t n) {
        unsigned __int128 m = static_cast<unsigned __int128>(next()) * n;
        uint64_t lo = static_cast<uint64_t>(m);
        if (lo < n) {
            uint64_t t = (0 - n) % n;
            while (lo < t) {
                m = static_cast<unsigned __int128>(next()) * n;
                lo = static_cast<uint64_t>(m);
            }
        }
        return static_cast<uint64_t>(m >> 64);
    }
    double uniform01() { return static_cast<double>(next() >> 11) * (1.0 / 9007199254740992.0); }
};

double pow_int(double x, int64_t k) {
    double r = 1.0, b = x;
    while (k) {
        if (k & 1) r *= b;
        b *= b;
        k >>= 1;
    }
    return r;
}

}  // namespace

std::vector<double> binomial_cdf(int64_t M, double p) {
    double q = 1.0 - p;
    double b = pow_int(q, M);
    double ratio = q > 0 ? p / q : INFINITY;
    std::vector<double> cdf;
    double acc = 0.0;
    for (int64_t w = 0; w <= M; ++w) {
        acc += b;
        cdf.push_back(acc);
        if (w < M) b = b * static_cast<double>(M - w) / static_cast<double>(w + 1) * ratio;
        if (b == 0.0 && static_cast<double>(w) > static_cast<double>(M) * p) break;
    }
    return cdf;
}

namespace {

struct ShotDraw {
    std::vector<int32_t> chan;
    std::vector<uint8_t> pauli;
};

void draw_shot(const msc_circuit* c, uint64_t seed, uint64_t shot, int64_t w_given,
               const std::vector<double>* cdf, std::vector<int32_t>& chans,
               std::vector<uint8_t>& paulis) {
    Rng rng(seed, shot);
    const int64_t M = c->n_channels;
    int64_t w;
    if (w_given >= 0) {
        w = w_given;
    } else {
        double u = rng.uniform01();
        w = static_cast<int64_t>(cdf->size()) - 1;
        for (size_t i = 0; i < cdf->size(); ++i)
            if (u < (*cdf)[i]) { w = static_cast<int64_t>(i); break; }
    }
    w = std::min<int64_t>(w, M);
    chans.clear();
    // Floyd: for j in [M-w, M): t = uniform in [0, j]; add t, or j if taken
    for (int64_t j = M - w; j < M; ++j) {
        int64_t t = static_cast<int64_t>(rng.bounded(static_cast<uint64_t>(j + 1)));
        bool have = std::find(chans.begin(), chans.end(), static_cast<int32_t>(t)) != chans.end();
        chans.push_back(static_cast<int32_t>(have ? j : t));
    }
    std::sort(chans.begin(), chans.end());
    paulis.clear();
    for (int32_t ch : chans) {
        int k = c->chan_kind[ch];
        uint8_t code;
        if (k == CH_XERR) code = 1;
        else if (k == CH_DEP1) code = static_cast<uint8_t>(1 + rng.bounded(3));
        else if (k == CH_DEP2) code = static_cast<uint8_t>(1 + rng.bounded(15));
        else code = static_cast<uint8_t>(1 + rng.bounded(63));
        paulis.push_back(code);
    }
}

}  // namespace
}  // namespace msc

using namespace msc;

extern "C" int msc_sample_faults(const msc_circuit* c, uint64_t seed, uint64_t first_shot,
                                 int64_t n_shots, const int32_t* weights, double p,
                                 int64_t* shot_off, int32_t* chan, uint8_t* pauli,
                                 int64_t nnz_cap, int64_t* nnz_out) {
    if (!c || n_shots < 0 || !shot_off || !nnz_out) return set_error(MSC_E_INVALID, "null argument");
    if (!weights && !(p >= 0.0 && p <= 1.0)) return set_error(MSC_E_INVALID, "p outside [0,1]");
    std::vector<double> cdf;
    if (!weights) cdf = binomial_cdf(c->n_channels, p);
    // draw in parallel chunks, then lay out the CSR in order
    const int64_t nthreads = std::max<int64_t>(1, std::min<int64_t>(16, n_shots / 4096));
    std::vector<std::vector<int32_t>> tch(nthreads);
    std::vector<std::vector<uint8_t>> tpa(nthreads);
    std::vector<std::vector<int64_t>> tcnt(nthreads);
    auto work = [&](int64_t t) {
        int64_t lo = n_shots * t / nthreads, hi = n_shots * (t + 1) / nthreads;
        std::vector<int32_t> cs;
        std::vector<uint8_t> ps;
        tcnt[t].reserve(hi - lo);
        for (int64_t i = lo; i < hi; ++i) {
            int64_t wg = weights ? weights[i] : -1;
            if (weights && wg < 0) wg = 0;
            draw_shot(c, seed, first_shot + static_cast<uint64_t>(i), wg,
                      weights ? nullptr : &cdf, cs, ps);
            tch[t].insert(tch[t].end(), cs.begin(), cs.end());
            tpa[t].insert(tpa[t].end(), ps.begin(), ps.end());
            tcnt[t].push_back(static_cast<int64_t>(cs.size()));
        }
    };
    if (nthreads == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        for (int64_t t = 0; t < nthreads; ++t) th.emplace_back(work, t);
        for (auto& x : th) x.join();
    }
    int64_t total = 0;
    for (auto& v : tch) total += static_cast<int64_t>(v.size());
    *nnz_out = total;
    if (total > nnz_cap) return set_error(MSC_E_CAPACITY, "nnz_cap too small");
    if (total > 0 && (!chan || !pauli)) return set_error(MSC_E_INVALID, "null chan/pauli");
    int64_t pos = 0, s = 0;
    shot_off[0] = 0;
    for (int64_t t = 0; t < nthreads; ++t) {
        std::copy(tch[t].begin(), tch[t].end(), chan + pos);
        std::copy(tpa[t].begin(), tpa[t].end(), pauli + pos);
        for (int64_t cnt : tcnt[t]) {
            pos += cnt;
            shot_off[++s] = pos;
        }
    }
    return MSC_OK;
}

// ---------------------------------------------------------------------------
// Eq. (reweight): p_acc = sum_w Bin_w(p) p_acc^(w), and the same with
// p_acc^(w) p_le^(w); B = sum_{w > w_max} Bin_w(p) (Appendix
// "Systematics"), summed over the tail itself so that tiny bounds keep full
// relative precision.  Bin_w(p) = exp(lgamma terms + w log p + (M-w) log1p(-p)).
double msc::log_bin(int64_t M, int64_t w, double p) {
    if (p <= 0.0) return w == 0 ? 0.0 : -INFINITY;
    if (p >= 1.0) return w == M ? 0.0 : -INFINITY;
    return std::lgamma(static_cast<double>(M + 1)) - std::lgamma(static_cast<double>(w + 1)) -
           std::lgamma(static_cast<double>(M - w + 1)) + static_cast<double>(w) * std::log(p) +
           static_cast<double>(M - w) * std::log1p(-p);
}

extern "C" int msc_reweight(const double* bin_n, const double* bin_acc, const double* bin_fail,
                            const double* bin_acc2, const double* bin_fail2, int32_t n_bins,
                            int64_t M, const double* p_grid, int32_t n_p, msc_estimate* out) {
    if (!bin_n || !bin_acc || !bin_fail || !p_grid || !out || n_bins < 1 || n_p < 0 || M < 0)
        return set_error(MSC_E_INVALID, "bad reweight arguments");
    if ((bin_acc2 == nullptr) != (bin_fail2 == nullptr))
        return set_error(MSC_E_INVALID, "give both sums of squares or neither");
    if (n_bins > M + 1) return set_error(MSC_E_INVALID, "more bins than M+1");
    // variance of one shot's value in a bin: the unbiased sample variance
    // from the sums, else the Bhatia-Davis bound of a [0, 1] variable
    auto var = [](double n, double s, const double* s2, int32_t w) {
        const double mu = s / n;
        if (s2 && n >= 2.0) return std::max(0.0, (s2[w] - s * mu) / (n - 1.0));
        return std::max(0.0, mu * (1.0 - mu));
    };
    for (int32_t k = 0; k < n_p; ++k) {
        double p = p_grid[k];
        if (!(p >= 0.0 && p <= 1.0)) return set_error(MSC_E_INVALID, "p outside [0,1]");
        double pacc = 0.0, num = 0.0, tail = 0.0, va = 0.0, ve = 0.0;
        for (int64_t w = M; w >= n_bins; --w) tail += std::exp(log_bin(M, w, p));
        for (int32_t w = 0; w < n_bins; ++w) {
            double b = std::exp(log_bin(M, w, p));
            const double n = bin_n[w];
            if (n <= 0.0) continue;
            pacc += b * bin_acc[w] / n;
            num += b * bin_fail[w] / n;
            va += b * b * var(n, bin_acc[w], bin_acc2, w) / n;
            ve += b * b * var(n, bin_fail[w], bin_fail2, w) / n;
        }
        out[k].p_acc = pacc;
        out[k].p_acc_le = num;
        out[k].p_le = pacc > 0.0 ? num / pacc : NAN;
        out[k].trunc_bound = tail;
        out[k].sem_p_acc = std::sqrt(va);
        out[k].sem_p_acc_le = std::sqrt(ve);
    }
    return MSC_OK;
}
