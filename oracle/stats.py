"""Likelihood statistics of the subset-sampling estimator, oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written from the
paper's appendices "Error analysis of the subset-sampling estimator" and
"Credible intervals for rate ratios":

* per-bin counts: n_w shots, k_w accepted, m_w accepted and wrong.  A shot's
  simulation gives the probability P_acc of its accepted branch and whether
  that branch is a logical failure; the paper's count version of the shot
  is one Bernoulli(P_acc) draw, taken here with a counter-based uniform of
  its own (``acceptance_uniform``);
* the per-bin log-likelihood of Eq. (loglik-split): a binomial in p_acc over
  n_w trials plus a binomial in p_le over k_w trials (0 log 0 = 0);
* the profile likelihood of Eq. (profile) for the two reported functionals,
  p_acc = sum_w Bin_w p_acc^(w) and p_le = sum_w Bin_w p_acc^(w) p_le^(w) /
  sum_w Bin_w p_acc^(w), over the sampled bins (n_w > 0), with p_le^(w) = 0
  imposed for w < d_e; the constrained maximum is taken by a general
  optimiser (scipy SLSQP, best of several starts) over all bin rates;
* likelihood-ratio intervals at R = 100: endpoints by bisection on the
  profile; the truncation bound B is added to the upper endpoint only
  (Appendix "Systematics");
* the 95 % central credible interval of a ratio T/S: T's posterior is the
  normalised profile likelihood of p_le with a prior flat in log(theta) on
  a log-spaced grid extended until the profile is 18 log-units below its
  maximum; S ~ Beta(n_err + 1/2, n_acc - n_err + 1/2) (Jeffreys); the density
  of log T - log S by discrete convolution on a shared lattice.

Lattice and percentile rule (the paper fixes neither): natural-log lattice
x_j = j h; densities are sampled at lattice points; the CDF of the lattice
distribution is read at cell edges x_j + h/2 and a percentile is found by
linear interpolation between consecutive edges.
"""
from __future__ import annotations

import math
import warnings

import numpy as np
from scipy import optimize
from scipy import stats as sst

from .estimators import binom_pmf
from .sampler import SplitMix64

# key of the acceptance stream: the shot's own (seed, shot) generator with
# the seed XOR'ed by this constant (the first 64 fraction bits of pi)
ACCEPT_KEY = 0x243F6A8885A308D3

P_ACC, P_LE = 0, 1


def acceptance_uniform(seed: int, shot: int) -> float:
    """Uniform in [0, 1) deciding whether a shot counts as accepted."""
    return SplitMix64(seed ^ ACCEPT_KEY, shot).uniform01()


def count_bins(seed: int, first_shot: int, weights, p_acc, fail, n_bins: int):
    """(n_w, k_w, m_w) per weight bin (weights >= n_bins - 1 share the last):
    shot i counts as accepted iff acceptance_uniform(seed, first_shot + i) <
    P_acc_i, and as wrong iff accepted and its branch fails."""
    n = np.zeros(n_bins)
    k = np.zeros(n_bins)
    m = np.zeros(n_bins)
    for i, (w, pa, f) in enumerate(zip(weights, p_acc, fail)):
        b = min(int(w), n_bins - 1)
        n[b] += 1
        if acceptance_uniform(seed, first_shot + i) < pa:
            k[b] += 1
            if f:
                m[b] += 1
    return n, k, m


def _xlogy(x, y):
    return 0.0 if x == 0 else x * math.log(y)


def loglik_bin(n, k, m, a, e) -> float:
    """Eq. (loglik-split): acceptance over n trials plus failure over the k
    accepted (the combinatorial prefactor dropped)."""
    return (_xlogy(k, a) + _xlogy(n - k, 1.0 - a)
            + _xlogy(m, e) + _xlogy(k - m, 1.0 - e))


def loglik_multinomial(n, k, m, a, e) -> float:
    """The same bin as the multinomial of its three exclusive outcomes
    (rejected, accepted and correct, accepted and wrong)."""
    return (_xlogy(n - k, 1.0 - a) + _xlogy(k - m, a * (1.0 - e))
            + _xlogy(m, a * e))


class Problem:
    """The sampled bins of one data set at one physical error rate."""

    def __init__(self, n, k, m, M: int, p: float, d_e: int = 0):
        n, k, m = (np.asarray(x, dtype=float) for x in (n, k, m))
        nb = len(n)
        self.B = sum(binom_pmf(M, w, p) for w in range(nb, M + 1))
        keep = [w for w in range(nb) if n[w] > 0]
        self.w = keep
        self.n, self.k, self.m = n[keep], k[keep], m[keep]
        self.b = np.array([binom_pmf(M, w, p) for w in keep])
        self.fixed = np.array([w < d_e for w in keep])
        if np.any(self.m[self.fixed] > 0):
            raise ValueError("a bin below d_e holds a logical failure")
        self.free = ~self.fixed
        self.nw = len(keep)
        self.nfree = int(self.free.sum())

    # parameters: a (all bins) then e (free bins)
    def unpack(self, x):
        a = x[:self.nw]
        e = np.zeros(self.nw)
        e[self.free] = x[self.nw:]
        return a, e

    def loglik(self, x) -> float:
        a, e = self.unpack(x)
        return sum(loglik_bin(self.n[i], self.k[i], self.m[i], a[i], e[i])
                   for i in range(self.nw))

    def grad(self, x):
        a, e = self.unpack(x)
        ga = np.zeros(self.nw)
        ge = np.zeros(self.nw)
        for i in range(self.nw):
            n, k, m = self.n[i], self.k[i], self.m[i]
            ga[i] = (k / a[i] if k else 0.0) - ((n - k) / (1 - a[i]) if n - k else 0.0)
            ge[i] = (m / e[i] if m else 0.0) - ((k - m) / (1 - e[i]) if k - m else 0.0)
        return np.concatenate([ga, ge[self.free]])

    def functional(self, x, which):
        a, e = self.unpack(x)
        if which == P_ACC:
            return float(self.b @ a)
        return float(self.b @ (a * e)) / float(self.b @ a)

    def mle(self):
        a = self.k / self.n
        e = np.where(self.k > 0, self.m / np.maximum(self.k, 1), 0.0)
        e[self.fixed] = 0.0
        return np.concatenate([a, e[self.free]])

    def theta_range(self, which):
        if which == P_ACC:
            return 0.0, float(self.b.sum())
        return 0.0, (1.0 if self.nfree else 0.0)


_EPS = 1e-13


def _constrained_max(pb: Problem, which: int, theta: float) -> float:
    """max of the joint log-likelihood over all bin rates subject to the
    functional equal to theta (Eq. (profile)), by SLSQP from several
    starting points; the best feasible result."""
    nv = pb.nw + pb.nfree
    bounds = [(_EPS, 1.0 - _EPS)] * nv
    if which == P_ACC:
        cons = {"type": "eq",
                "fun": lambda x: np.array([pb.b @ x[:pb.nw] - theta]),
                "jac": lambda x: np.concatenate([pb.b, np.zeros(pb.nfree)])[None, :]}
    else:
        def fun(x):
            a, e = pb.unpack(x)
            return np.array([pb.b @ (a * (e - theta))])

        def jac(x):
            a, e = pb.unpack(x)
            return np.concatenate([pb.b * (e - theta), (pb.b * a)[pb.free]])[None, :]
        cons = {"type": "eq", "fun": fun, "jac": jac}
    starts = []
    x0 = np.clip(pb.mle(), 0.02, 0.98)
    starts.append(x0)
    if which == P_ACC:
        s = np.full(pb.nw, min(max(theta / max(pb.b.sum(), 1e-300), 0.02), 0.98))
        starts.append(np.concatenate([s, x0[pb.nw:]]))
    else:
        starts.append(np.concatenate([x0[:pb.nw], np.full(pb.nfree,
                                                          min(max(theta, 0.02), 0.98))]))
    starts.append(np.full(nv, 0.5))
    best = -math.inf
    for x0 in starts:
        with warnings.catch_warnings():
            # SLSQP clips its trial steps to the bounds and says so
            warnings.simplefilter("ignore", RuntimeWarning)
            r = optimize.minimize(lambda x: -pb.loglik(x), x0, jac=lambda x: -pb.grad(x),
                                  bounds=bounds, constraints=[cons], method="SLSQP",
                                  options={"ftol": 1e-15, "maxiter": 2000})
        x = np.clip(r.x, _EPS, 1 - _EPS)
        if abs(cons["fun"](x)[0]) > 1e-9 * max(1.0, theta):
            continue
        best = max(best, pb.loglik(x))
    return best


def profile_loglik(pb: Problem, which: int, theta: float) -> float:
    """Eq. (profile): max_{f(p) = theta} l(p) - max_p l(p)."""
    lo, hi = pb.theta_range(which)
    if theta < lo or theta > hi:
        return -math.inf
    return _constrained_max(pb, which, theta) - pb.loglik(pb.mle())


def lr_interval(pb: Problem, which: int, R: float = 100.0, iters: int = 60):
    """Likelihood-ratio interval of Eq. (profile) with threshold log R,
    endpoints by bisection; returns (mle, lo, hi, hi + B)."""
    x = pb.mle()
    th = pb.functional(x, which) if (which == P_ACC or pb.b @ x[:pb.nw] > 0) else 0.0
    cut = -math.log(R)
    tlo, thi = pb.theta_range(which)

    def inside(t):
        return profile_loglik(pb, which, t) >= cut

    def edge(a, b):
        # a inside, b outside
        for _ in range(iters):
            c = 0.5 * (a + b)
            if inside(c):
                a = c
            else:
                b = c
        return 0.5 * (a + b)

    hi = thi if inside(thi) else edge(th, thi)
    lo = tlo if inside(tlo) else edge(th, tlo)
    return th, lo, hi, hi + pb.B


def _lattice_density(logf, x0, h):
    """Samples exp(logf) on the lattice j h, from the lattice point nearest
    x0 outwards in both directions until logf is 18 below its maximum."""
    j0 = int(round(x0 / h))
    vals = {j0: logf(j0 * h)}
    mx = vals[j0]
    for step in (1, -1):
        j = j0
        while True:
            j += step
            v = logf(j * h)
            vals[j] = v
            mx = max(mx, v)
            if v < mx - 18.0 and j * step > j0 * step + 2:
                break
    js = sorted(vals)
    return js[0], np.exp(np.array([vals[j] for j in js]) - mx)


def ratio_credible(pb: Problem, s_acc: int, s_err: int, level: float = 0.95,
                   h: float = 2e-3):
    """Central credible interval of T / S: T = p_le of the data set pb
    (profile posterior, prior flat in log theta), S ~ Beta(s_err + 1/2,
    s_acc - s_err + 1/2).  Returns (lo, hi)."""
    th = pb.functional(pb.mle(), P_LE)
    if not th > 0:
        raise ValueError("the profile of T needs at least one failure")

    def log_t(x):
        v = profile_loglik(pb, P_LE, math.exp(x))
        return v if v > -1e300 else -1e300

    al, be = s_err + 0.5, s_acc - s_err + 0.5

    def log_s(x):
        # density of log S: f_S(e^x) e^x
        s = math.exp(x)
        if s >= 1.0:
            return -1e300
        return float(sst.beta.logpdf(s, al, be)) + x

    jt, dt = _lattice_density(log_t, math.log(th), h)
    mode_s = (al - 0.0) / (al + be)          # mode of log S under f_S(s) s
    js, ds = _lattice_density(log_s, math.log(mode_s), h)
    # log R = x_T - x_S: g[j] = sum_i dT[i] dS[i - j]
    g = np.convolve(dt, ds[::-1])
    j_first = jt - (js + len(ds) - 1)
    c = np.cumsum(g) / g.sum()
    edges = (j_first + np.arange(len(g))) * h + 0.5 * h

    def pct(q):
        i = int(np.searchsorted(c, q))
        if i == 0:
            return math.exp(edges[0])
        f = (q - c[i - 1]) / (c[i] - c[i - 1])
        return math.exp(edges[i - 1] + f * (edges[i] - edges[i - 1]))

    a = 0.5 * (1.0 - level)
    return pct(a), pct(1.0 - a)
