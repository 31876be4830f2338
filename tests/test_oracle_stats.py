"""Pins of the oracle's likelihood statistics (oracle/stats.py) against what
the mathematics fixes: the multinomial the split of Eq. (loglik-split)
decomposes, one-bin cases that reduce to the binomial likelihood-ratio
interval, a brute-force profile over two bins, the asymptotic chi-square
law of the profile at the truth (the coverage the error analysis quotes for
R = 100), the exact posterior of a ratio of Beta variates, and the
counter-based acceptance draws.
"""
import math
import warnings

import numpy as np
import pytest
from scipy import integrate, optimize
from scipy import stats as sst

from oracle import sampler as osamp
from oracle import stats as S

pytestmark = pytest.mark.filterwarnings("ignore:Values in x were outside bounds")


def test_split_equals_multinomial():
    rng = np.random.default_rng(1)
    for _ in range(200):
        n = int(rng.integers(0, 500))
        k = int(rng.integers(0, n + 1))
        m = int(rng.integers(0, k + 1))
        a, e = rng.uniform(1e-6, 1 - 1e-6, 2)
        assert math.isclose(S.loglik_bin(n, k, m, a, e), S.loglik_multinomial(n, k, m, a, e),
                            rel_tol=1e-12, abs_tol=1e-9)


def _binomial_lr(succ, trials, R=100.0):
    """Textbook one-parameter likelihood-ratio interval by root finding."""
    def ll(q):
        return (succ * math.log(q) if succ else 0.0) + \
            ((trials - succ) * math.log1p(-q) if trials - succ else 0.0)
    hat = succ / trials
    cut = ll(min(max(hat, 1e-300), 1 - 1e-16)) - math.log(R)
    lo = 0.0 if succ == 0 else optimize.brentq(lambda q: ll(q) - cut, 1e-300, hat, xtol=1e-15)
    hi = 1.0 if succ == trials else optimize.brentq(lambda q: ll(q) - cut, hat, 1 - 1e-16,
                                                    xtol=1e-15)
    return lo, hi


@pytest.mark.parametrize("n,k,m", [(200, 37, 3), (50, 50, 0), (80, 0, 0), (1000, 400, 399)])
def test_single_bin_reduces_to_binomial_intervals(n, k, m):
    # with M = 0 the only bin is w = 0 with Bin_0 = 1: p_acc is a binomial
    # proportion over n shots, p_le one over the k accepted ones
    pb = S.Problem([n], [k], [m], M=0, p=0.0)
    est, lo, hi, hib = S.lr_interval(pb, S.P_ACC)
    blo, bhi = _binomial_lr(k, n)
    assert est == pytest.approx(k / n)
    assert lo == pytest.approx(blo, abs=1e-9) and hi == pytest.approx(bhi, abs=1e-9)
    assert hib == hi                       # nothing above w = M
    if k > 0:
        est, lo, hi, _ = S.lr_interval(pb, S.P_LE)
        blo, bhi = _binomial_lr(m, k)
        assert est == pytest.approx(m / k)
        assert lo == pytest.approx(blo, abs=1e-9) and hi == pytest.approx(bhi, abs=1e-9)


def test_two_bin_profile_matches_brute_force_pacc():
    n, k, m = [50, 80], [40, 10], [0, 2]
    pb = S.Problem(n, k, m, M=20, p=0.05)
    b = pb.b
    e2 = m[1] / k[1]
    lle = m[1] * math.log(e2) + (k[1] - m[1]) * math.log(1 - e2)
    lmax = pb.loglik(pb.mle())
    for frac in (0.3, 0.5, 0.9):
        th = frac * b.sum()
        a1 = np.linspace(1e-9, 1 - 1e-9, 2_000_001)
        a2 = (th - b[0] * a1) / b[1]
        ok = (a2 > 0) & (a2 < 1)
        a1, a2 = a1[ok], a2[ok]
        v = (k[0] * np.log(a1) + (n[0] - k[0]) * np.log1p(-a1)
             + k[1] * np.log(a2) + (n[1] - k[1]) * np.log1p(-a2))
        brute = v.max() + lle - lmax
        assert S.profile_loglik(pb, S.P_ACC, th) == pytest.approx(brute, abs=1e-7)


def test_two_bin_profile_matches_brute_force_ple():
    # maximise over (a1, a2, e1) on a grid with e2 fixed by the constraint
    n, k, m = np.array([60, 40]), np.array([30, 25]), np.array([2, 6])
    pb = S.Problem(n, k, m, M=10, p=0.1)
    b = pb.b
    lmax = pb.loglik(pb.mle())
    g = np.linspace(0.002, 0.998, 250)
    a1, a2, e1 = np.meshgrid(g, g, g, indexing="ij")
    for th in (0.06, 0.15, 0.3):
        e2 = (th * (b[0] * a1 + b[1] * a2) - b[0] * a1 * e1) / (b[1] * a2)
        ok = (e2 > 0) & (e2 < 1)
        with np.errstate(divide="ignore", invalid="ignore"):
            v = (k[0] * np.log(a1) + (n[0] - k[0]) * np.log1p(-a1)
                 + k[1] * np.log(a2) + (n[1] - k[1]) * np.log1p(-a2)
                 + m[0] * np.log(e1) + (k[0] - m[0]) * np.log1p(-e1)
                 + m[1] * np.log(e2) + (k[1] - m[1]) * np.log1p(-e2))
        brute = np.where(ok, v, -np.inf).max() - lmax
        prof = S.profile_loglik(pb, S.P_LE, th)
        # the optimiser can only beat the grid, and only by its resolution
        assert prof >= brute - 1e-9
        assert prof - brute < 0.05


def test_truncation_bound_added_upward_only():
    pb = S.Problem([100, 100], [90, 20], [0, 3], M=50, p=0.02)
    B = sum(S.binom_pmf(50, w, 0.02) for w in range(2, 51))
    for f in (S.P_ACC, S.P_LE):
        est, lo, hi, hib = S.lr_interval(pb, f)
        assert hib == pytest.approx(hi + B, rel=1e-14)
        assert lo <= est <= hi


def test_below_de_fixes_ple_to_zero_and_keeps_pacc():
    # imposing p_le^(w) = 0 on a bin leaves its p_acc estimate and interval
    # untouched (orthogonality of the split)
    n, k, m = [100, 100], [70, 30], [0, 4]
    free = S.Problem(n, k, m, M=30, p=0.01, d_e=0)
    fixd = S.Problem(n, k, m, M=30, p=0.01, d_e=1)
    a = S.lr_interval(free, S.P_ACC)
    b = S.lr_interval(fixd, S.P_ACC)
    assert a == pytest.approx(b, rel=1e-9)
    with pytest.raises(ValueError):
        S.Problem(n, k, [1, 4], M=30, p=0.01, d_e=1)


def test_profile_at_truth_follows_chi_square():
    # Wilks: -2 x (profile at the true value) ~ chi2_1; R = 100 gives the
    # error analysis's 99.76 % coverage
    rng = np.random.default_rng(7)
    M, p = 40, 0.05
    n = np.array([200, 300, 300])
    a_true = np.array([0.9, 0.5, 0.2])
    e_true = np.array([0.0, 0.1, 0.3])
    b = np.array([S.binom_pmf(M, w, p) for w in range(3)])
    theta = {S.P_ACC: float(b @ a_true), S.P_LE: float(b @ (a_true * e_true) / (b @ a_true))}
    stats = {f: [] for f in theta}
    reps = 150
    for _ in range(reps):
        k = rng.binomial(n, a_true)
        m = rng.binomial(k, e_true)
        pb = S.Problem(n, k, m, M, p)
        for f, th in theta.items():
            stats[f].append(-2.0 * S.profile_loglik(pb, f, th))
    for f in theta:
        d = np.array(stats[f])
        assert (d > 2 * math.log(100.0)).sum() <= 3          # expected 0.36 misses
        assert abs(d.mean() - 1.0) < 0.35                     # chi2_1 mean
        # distribution test against chi2_1
        assert sst.kstest(d, sst.chi2(1).cdf).pvalue > 1e-3


def _beta_ratio_percentiles(a1, b1, a2, b2, qs):
    """Percentiles of X / Y, X ~ Beta(a1, b1), Y ~ Beta(a2, b2) independent,
    from P(X/Y <= r) = int F_X(r y) f_Y(y) dy."""
    X, Y = sst.beta(a1, b1), sst.beta(a2, b2)
    lo, hi = Y.ppf(1e-13), Y.ppf(1 - 1e-13)

    def cdf(r):
        return integrate.quad(lambda y: X.cdf(min(1.0, r * y)) * Y.pdf(y), lo, hi,
                              limit=500, epsabs=1e-13, epsrel=1e-12)[0]
    return [optimize.brentq(lambda r: cdf(r) - q, 1e-5, 1e4, xtol=1e-14) for q in qs]


def test_ratio_credible_single_bin_is_a_beta_ratio():
    # one bin: the profile of p_le is e^m (1-e)^(k-m), so with the prior flat
    # in log(theta) the posterior of T is Beta(m, k - m + 1); S is Jeffreys
    n, k, m, sa, se = 400, 120, 7, 3000, 20
    pb = S.Problem([n], [k], [m], M=0, p=0.0)
    lo, hi = S.ratio_credible(pb, sa, se, h=1e-2)
    ex = _beta_ratio_percentiles(m, k - m + 1, se + 0.5, sa - se + 0.5, (0.025, 0.975))
    assert lo == pytest.approx(ex[0], rel=2e-4)
    assert hi == pytest.approx(ex[1], rel=2e-4)


def test_acceptance_draws():
    seed = 0x5EED0021
    u = np.array([S.acceptance_uniform(seed, i) for i in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert sst.kstest(u, "uniform").pvalue > 1e-3
    # a stream of its own: not the shot's fault-draw uniform
    assert S.acceptance_uniform(seed, 3) != osamp.SplitMix64(seed, 3).uniform01()
    assert S.acceptance_uniform(seed, 3) == osamp.SplitMix64(seed ^ S.ACCEPT_KEY, 3).uniform01()
    w = np.array([0, 1, 1, 2, 3, 5] * 500)
    pa = np.tile([1.0, 0.0, 0.5, 1.0, 0.25, 1.0], 500)
    fail = np.tile([0, 0, 1, 1, 0, 1], 500)
    n, k, m = S.count_bins(seed, 100, w, pa, fail, 4)
    assert list(n) == [500, 1000, 500, 1000]            # weight 5 joins the last bin
    assert k[0] == 500 and k[2] == 500                  # P_acc = 1 always counts
    assert m[0] == 0 and m[2] == 500
    assert 200 < k[1] < 300                             # 500 x Bernoulli(1/2)
    assert m[1] == k[1]                                 # every accepted one fails
    assert m[3] == 500
    assert 500 + 60 < k[3] < 500 + 190                  # 500 + 500 x Bernoulli(1/4)
