// Likelihood statistics of the subset-sampling estimator: the per-bin
// likelihood of Eq. (loglik-split), the profile likelihood and likelihood-
// ratio intervals of Eq. (profile) with the one-sided truncation bound
// (Appendix "Error analysis of the subset-sampling estimator"), the credible
// interval of a rate ratio (Appendix "Credible intervals for rate ratios")
// and the loss multiplier (Appendix "Losses").
//
// Method.  A bin's three exclusive outcomes (rejected; accepted and
// correct; accepted and wrong) have probabilities x = (1 - a, a (1 - e),
// a e) with a = p_acc^(w) and e = p_le^(w).  In these coordinates the joint
// log-likelihood sum_w sum_j n_wj log x_wj is concave, and both reported
// functionals fix a linear form of x: p_acc = theta is
// sum_w Bin_w (x_w1 + x_w2) = theta, and p_le = theta is
// sum_w Bin_w ((1 - theta) x_w2 - theta x_w1) = 0.  The constrained maximum
// is the maximum of the Lagrangian at the multiplier lambda that meets the
// constraint (a concave problem with one linear constraint has no duality
// gap), and for fixed lambda the bins decouple: each maximises
// sum_j n_j log x_j - sum_j c_j x_j over the simplex, whose solution is
// x_j = n_j / (c_j + s) for the outcomes with counts, one scalar s per bin
// fixed by sum_j x_j = 1, while a zero-count outcome takes the slack when
// its cost is the lowest.  The constraint value falls monotonically with
// lambda, so lambda is found by bisection.
#include <algorithm>
#include <cmath>
#include <functional>
#include <vector>

#include "../msc_internal.h"

namespace msc {
namespace {

struct Bin {
    double n[3];  // rejected, accepted and correct, accepted and wrong
    double b;     // Bin_w(p)
    bool fixed;   // p_le^(w) = 0 imposed (w < d_e): outcome 2 is excluded
};

struct Data {
    std::vector<Bin> bins;
    double B = 0.0;               // sum_{w >= n_bins} Bin_w(p)
    double unsampled_mass = 0.0;  // sum of Bin_w over bins with n_w = 0
    double unaccepted = 0.0;      // sum over bins with k_w = 0 of Bin_w (1 - R^(-1/n_w))
    int n_unsampled = 0;
    double lmax = 0.0;            // log-likelihood at the maximum
    double acc_hat = 0.0;         // sum_w Bin_w k_w / n_w
    double err_hat = 0.0;         // sum_w Bin_w m_w / n_w
};

double xlogy(double x, double y) { return x == 0.0 ? 0.0 : x * std::log(y); }

int load(const double* bn, const double* bk, const double* bm, int32_t n_bins, int64_t M, double p,
         int32_t d_e, Data& d) {
    if (!bn || !bk || !bm || n_bins < 1 || M < 0 || d_e < 0)
        return set_error(MSC_E_INVALID, "bad statistics arguments");
    if (n_bins > M + 1) return set_error(MSC_E_INVALID, "more bins than M+1");
    if (!(p >= 0.0 && p <= 1.0)) return set_error(MSC_E_INVALID, "p outside [0,1]");
    for (int64_t w = M; w >= n_bins; --w) d.B += std::exp(log_bin(M, w, p));
    for (int32_t w = 0; w < n_bins; ++w) {
        const double n = bn[w], k = bk[w], m = bm[w];
        if (!(n >= 0.0 && k >= 0.0 && m >= 0.0 && k <= n && m <= k) || n != std::floor(n) ||
            k != std::floor(k) || m != std::floor(m))
            return set_error(MSC_E_INVALID, "counts must be integers with 0 <= m <= k <= n");
        const double b = std::exp(log_bin(M, w, p));
        if (n == 0.0) {
            d.unsampled_mass += b;
            ++d.n_unsampled;
            continue;
        }
        const bool fixed = w < d_e;
        if (fixed && m > 0.0)
            return set_error(MSC_E_INVALID, "a bin below d_e holds a logical failure");
        Bin x{{n - k, k - m, m}, b, fixed};
        d.bins.push_back(x);
        for (int j = 0; j < 3; ++j) d.lmax += xlogy(x.n[j], x.n[j] / n);
        d.acc_hat += b * k / n;
        d.err_hat += b * m / n;
    }
    return MSC_OK;
}

// argmax over the simplex of sum_j n_j log x_j - lam sum_j g_j x_j
// (outcome 2 excluded for fixed bins); returns its log-likelihood
double tilted(const Bin& bn, double lam, const double g[3], double x[3]) {
    const int nj = bn.fixed ? 2 : 3;
    int ref = -1;  // the outcome with counts and the lowest cost
    for (int j = 0; j < nj; ++j)
        if (bn.n[j] > 0.0 && (ref < 0 || lam * (g[j] - g[ref]) < 0.0)) ref = j;
    double dc[3] = {0.0, 0.0, 0.0};  // cost minus the reference cost
    for (int j = 0; j < nj; ++j) dc[j] = lam * (g[j] - g[ref]);
    // sum_j n_j / (dc_j + s) = 1: Newton from the left (the function is
    // convex and decreasing, so the iterates rise monotonically to the root)
    double s = 0.0;
    for (int j = 0; j < nj; ++j)
        if (bn.n[j] > 0.0) s = std::max(s, bn.n[j] - dc[j]);
    for (int it = 0; it < 300; ++it) {
        double G = 0.0, dG = 0.0;
        for (int j = 0; j < nj; ++j) {
            if (bn.n[j] <= 0.0) continue;
            const double t = 1.0 / (dc[j] + s);
            G += bn.n[j] * t;
            dG += bn.n[j] * t * t;
        }
        const double step = (G - 1.0) / dG;
        if (!(step > 0.0)) break;
        const double ns = s + step;
        if (ns == s) break;
        s = ns;
    }
    int z = -1;  // zero-count outcome with the lowest cost
    for (int j = 0; j < nj; ++j)
        if (bn.n[j] == 0.0 && (z < 0 || dc[j] < dc[z])) z = j;
    x[0] = x[1] = x[2] = 0.0;
    if (z >= 0 && -dc[z] > s) s = -dc[z];
    double used = 0.0, ll = 0.0;
    for (int j = 0; j < nj; ++j) {
        if (bn.n[j] <= 0.0) continue;
        x[j] = bn.n[j] / (dc[j] + s);
        used += x[j];
        ll += bn.n[j] * std::log(x[j]);
    }
    if (z >= 0) x[z] = std::max(0.0, 1.0 - used);
    return ll;
}

// the linear form of the constraint: coefficients per outcome of bin bn
void coeffs(const Bin& bn, int functional, double theta, double g[3]) {
    g[0] = 0.0;
    if (functional == MSC_STAT_PACC) {
        g[1] = bn.b;
        g[2] = bn.b;
    } else {
        g[1] = -bn.b * theta;
        g[2] = bn.b * (1.0 - theta);
    }
}

// C(lam) and the log-likelihood of the Lagrangian maximiser
void evaluate(const Data& d, int functional, double theta, double lam, double* C, double* ll) {
    double c = 0.0, l = 0.0;
    for (const Bin& bn : d.bins) {
        double g[3], x[3];
        coeffs(bn, functional, theta, g);
        l += tilted(bn, lam, g, x);
        c += g[0] * x[0] + g[1] * x[1] + g[2] * x[2];
    }
    *C = c;
    *ll = l;
}

// Eq. (profile): max_{f = theta} l - max l; -inf where theta is infeasible
double profile(const Data& d, int functional, double theta) {
    if (d.bins.empty()) return -INFINITY;
    const double target = functional == MSC_STAT_PACC ? theta : 0.0;
    double c0, l0;
    evaluate(d, functional, theta, 0.0, &c0, &l0);
    if (c0 == target) return l0 - d.lmax;
    // C falls with lam: bracket the root by doubling away from 0
    const double dir = c0 > target ? 1.0 : -1.0;
    double a = 0.0, b = dir, cb, lb;
    for (;;) {
        evaluate(d, functional, theta, b, &cb, &lb);
        if ((dir > 0.0 && cb <= target) || (dir < 0.0 && cb >= target)) break;
        if (std::fabs(b) > 1e300) return -INFINITY;
        a = b;
        b *= 2.0;
    }
    if (cb == target) return lb - d.lmax;
    double lm = lb;
    for (int it = 0; it < 200; ++it) {
        const double m = 0.5 * (a + b);
        if (m == a || m == b) break;
        double cm;
        evaluate(d, functional, theta, m, &cm, &lm);
        if (cm == target) return lm - d.lmax;
        if ((cm > target) == (dir > 0.0)) a = m;
        else b = m;
    }
    double cm;
    evaluate(d, functional, theta, 0.5 * (a + b), &cm, &lm);
    return lm - d.lmax;
}

double estimate(const Data& d, int functional) {
    if (functional == MSC_STAT_PACC) return d.acc_hat;
    return d.acc_hat > 0.0 ? d.err_hat / d.acc_hat : 0.0;
}

void theta_range(const Data& d, int functional, double* lo, double* hi) {
    *lo = 0.0;
    if (functional == MSC_STAT_PACC) {
        double s = 0.0;
        for (const Bin& bn : d.bins) s += bn.b;
        *hi = s;
    } else {
        bool any_free = false;
        for (const Bin& bn : d.bins) any_free |= !bn.fixed;
        *hi = any_free ? 1.0 : 0.0;
    }
}

// endpoints of {theta : profile >= -log R} by bisection from the estimate
void interval(const Data& d, int functional, double R, double* est, double* lo, double* hi) {
    const double th = estimate(d, functional), cut = -std::log(R);
    double tlo, thi;
    theta_range(d, functional, &tlo, &thi);
    auto inside = [&](double t) { return profile(d, functional, t) >= cut; };
    auto edge = [&](double a, double b) {  // a inside, b outside
        for (int it = 0; it < 60; ++it) {
            const double c = 0.5 * (a + b);
            if (inside(c)) a = c;
            else b = c;
        }
        return 0.5 * (a + b);
    };
    *est = th;
    *hi = inside(thi) ? thi : edge(th, thi);
    *lo = inside(tlo) ? tlo : edge(th, tlo);
}

// samples exp(logf) on the lattice j h from the point nearest x0 outwards
// until logf is 18 below its maximum on both sides
int64_t lattice(const std::function<double(double)>& logf, double x0, double h,
                std::vector<double>& out) {
    const int64_t j0 = std::llround(x0 / h);
    std::vector<double> up, down;
    double mx = logf(static_cast<double>(j0) * h);
    const double v0 = mx;
    for (int64_t j = j0 + 1;; ++j) {
        const double v = logf(static_cast<double>(j) * h);
        up.push_back(v);
        mx = std::max(mx, v);
        if (v < mx - 18.0 && j > j0 + 2) break;
        if (up.size() > 50000000) break;
    }
    for (int64_t j = j0 - 1;; --j) {
        const double v = logf(static_cast<double>(j) * h);
        down.push_back(v);
        mx = std::max(mx, v);
        if (v < mx - 18.0 && j < j0 - 2) break;
        if (down.size() > 50000000) break;
    }
    out.clear();
    for (size_t i = down.size(); i-- > 0;) out.push_back(std::exp(down[i] - mx));
    out.push_back(std::exp(v0 - mx));
    for (double v : up) out.push_back(std::exp(v - mx));
    return j0 - static_cast<int64_t>(down.size());
}

}  // namespace
}  // namespace msc

using namespace msc;

extern "C" int msc_profile_loglik(const double* bin_n, const double* bin_acc, const double* bin_err,
                                  int32_t n_bins, int64_t M, double p, int32_t d_e,
                                  int32_t functional, double theta, double* out) {
    if (functional != MSC_STAT_PACC && functional != MSC_STAT_PLE)
        return set_error(MSC_E_INVALID, "unknown functional");
    if (!out || !std::isfinite(theta)) return set_error(MSC_E_INVALID, "bad theta or output");
    Data d;
    if (int e = load(bin_n, bin_acc, bin_err, n_bins, M, p, d_e, d)) return e;
    double lo, hi;
    theta_range(d, functional, &lo, &hi);
    *out = (theta < lo || theta > hi) ? -INFINITY : profile(d, functional, theta);
    return MSC_OK;
}

extern "C" int msc_lr_interval(const double* bin_n, const double* bin_acc, const double* bin_err,
                               int32_t n_bins, int64_t M, double p, int32_t d_e,
                               int32_t functional, double R, msc_interval* out) {
    if (functional != MSC_STAT_PACC && functional != MSC_STAT_PLE)
        return set_error(MSC_E_INVALID, "unknown functional");
    if (!out || !(R > 1.0) || !std::isfinite(R)) return set_error(MSC_E_INVALID, "bad R or output");
    Data d;
    if (int e = load(bin_n, bin_acc, bin_err, n_bins, M, p, d_e, d)) return e;
    if (d.bins.empty()) return set_error(MSC_E_INVALID, "no sampled bin");
    msc_interval r{};
    interval(d, functional, R, &r.estimate, &r.lo, &r.hi);
    r.trunc_bound = d.B;
    r.hi_trunc = r.hi + d.B;
    for (const Bin& bn : d.bins) {
        const double n = bn.n[0] + bn.n[1] + bn.n[2];
        if (bn.n[1] + bn.n[2] == 0.0) r.unaccepted += bn.b * -std::expm1(-std::log(R) / n);
    }
    r.unsampled_mass = d.unsampled_mass;
    r.n_unsampled = d.n_unsampled;
    r.n_bins_used = static_cast<int32_t>(d.bins.size());
    *out = r;
    return MSC_OK;
}

extern "C" int msc_ratio_credible(const double* bin_n, const double* bin_acc,
                                  const double* bin_err, int32_t n_bins, int64_t M, double p,
                                  int32_t d_e, double s_acc, double s_err, double level,
                                  double h, double* lo, double* hi) {
    if (!lo || !hi || !(level > 0.0 && level < 1.0) || !(h > 0.0 && h <= 0.1))
        return set_error(MSC_E_INVALID, "bad level, lattice step or output");
    if (!(s_acc >= 0.0 && s_err >= 0.0 && s_err <= s_acc))
        return set_error(MSC_E_INVALID, "need 0 <= s_err <= s_acc");
    Data d;
    if (int e = load(bin_n, bin_acc, bin_err, n_bins, M, p, d_e, d)) return e;
    const double th = estimate(d, MSC_STAT_PLE);
    if (!(th > 0.0)) return set_error(MSC_E_INVALID, "the profile of T needs a failure");
    // T: profile posterior with a prior flat in log(theta)
    auto log_t = [&](double x) {
        const double t = std::exp(x);
        if (t > 1.0) return -1e300;
        const double v = profile(d, MSC_STAT_PLE, t);
        return v > -1e300 ? v : -1e300;
    };
    // S: Jeffreys Beta posterior; density of log S is f_S(e^x) e^x
    const double al = s_err + 0.5, be = s_acc - s_err + 0.5;
    const double lbeta = std::lgamma(al) + std::lgamma(be) - std::lgamma(al + be);
    auto log_s = [&](double x) {
        const double s = std::exp(x);
        if (s >= 1.0) return -1e300;
        return (al - 1.0) * x + (be - 1.0) * std::log1p(-s) - lbeta + x;
    };
    std::vector<double> dt, ds;
    const int64_t jt = lattice(log_t, std::log(th), h, dt);
    const int64_t js = lattice(log_s, std::log(al / (al + be)), h, ds);
    // log R = log T - log S: g[q] = sum_i dt[i] ds[LS - 1 - (q - i)]
    const int64_t LT = static_cast<int64_t>(dt.size()), LS = static_cast<int64_t>(ds.size());
    std::vector<double> g(static_cast<size_t>(LT + LS - 1), 0.0);
    for (int64_t i = 0; i < LT; ++i)
        for (int64_t r = 0; r < LS; ++r) g[static_cast<size_t>(i + r)] += dt[i] * ds[LS - 1 - r];
    const int64_t j_first = jt - (js + LS - 1);
    std::vector<double> c(g.size());
    double acc = 0.0;
    for (size_t q = 0; q < g.size(); ++q) {
        acc += g[q];
        c[q] = acc;
    }
    for (double& v : c) v /= acc;
    auto edge = [&](size_t q) { return (static_cast<double>(j_first + static_cast<int64_t>(q)) + 0.5) * h; };
    auto pct = [&](double q) {
        const size_t i = static_cast<size_t>(std::lower_bound(c.begin(), c.end(), q) - c.begin());
        if (i == 0) return std::exp(edge(0));
        if (i >= c.size()) return std::exp(edge(c.size() - 1));
        const double f = (q - c[i - 1]) / (c[i] - c[i - 1]);
        return std::exp(edge(i - 1) + f * (edge(i) - edge(i - 1)));
    };
    const double a = 0.5 * (1.0 - level);
    *lo = pct(a);
    *hi = pct(1.0 - a);
    return MSC_OK;
}

extern "C" int msc_loss_factor(int64_t M, double p_loss, double* out) {
    if (!out || M < 0 || !(p_loss >= 0.0 && p_loss < 1.0))
        return set_error(MSC_E_INVALID, "need M >= 0 and 0 <= p_loss < 1");
    // (1 - p_l)^(-M) = exp(-M log1p(-p_l))
    *out = std::exp(-static_cast<double>(M) * std::log1p(-p_loss));
    return MSC_OK;
}

extern "C" int msc_expected_volume(const double* bin_n, const double* surv_bins, int32_t n_bins,
                                   const msc_segment* segs, int32_t n_seg, int64_t M, double p,
                                   double* reach, double* volume) {
    if (!bin_n || !surv_bins || !segs || !reach || !volume || n_bins < 1 || n_seg < 1 || M < 0)
        return set_error(MSC_E_INVALID, "bad expected-volume arguments");
    if (n_bins > M + 1) return set_error(MSC_E_INVALID, "more bins than M+1");
    if (!(p >= 0.0 && p <= 1.0)) return set_error(MSC_E_INVALID, "p outside [0,1]");
    for (int32_t s = 0; s < n_seg; ++s) reach[s] = 0.0;
    for (int32_t w = 0; w < n_bins; ++w) {
        if (!(bin_n[w] > 0.0)) continue;
        const double b = std::exp(log_bin(M, w, p));
        for (int32_t s = 0; s < n_seg; ++s)
            reach[s] += b * surv_bins[static_cast<size_t>(w) * n_seg + s] / bin_n[w];
    }
    double B = 0.0;
    for (int64_t w = M; w >= n_bins; --w) B += std::exp(log_bin(M, w, p));
    double vol = 0.0, vmax = 0.0;
    for (int32_t s = 0; s < n_seg; ++s) {
        if (!segs[s].noisy) continue;
        const double v = static_cast<double>(segs[s].n_qubits) * segs[s].depth;
        vol += v * reach[s];
        vmax += v;
    }
    volume[0] = vol;
    volume[1] = vol + B * vmax;
    return MSC_OK;
}
