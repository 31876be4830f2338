"""Subset-sampling estimators (Section 4.1; Appendix "Error analysis").

* Bin_w(p) = C(M, w) p^w (1-p)^(M-w)                      (Section 4.1)
* p_acc = sum_w Bin_w(p) p_acc^(w),
  p_acc p_le = sum_w Bin_w(p) p_acc^(w) p_le^(w)         Eq. (reweight)
* per-bin estimates from n_w shots: here the per-shot indicators of
  Eq. (estimators) are replaced by their conditional expectations given the
  fault configuration (P_acc and P_acc * fail), which estimate the same
  p_acc^(w) and p_acc^(w) p_le^(w);
* truncation bound B = sum_{w > w_max} Bin_w(p), added one-sided
  (Appendix "Systematics");
* standard errors of the re-weighted sums from the per-bin variances
  (independent bins);
* loss multiplier (1 - p_l)^(-M) on the expected attempts (Appendix
  "Losses").
"""
from __future__ import annotations

import math


def log_binom_pmf(M: int, w: int, p: float) -> float:
    if p <= 0.0:
        return 0.0 if w == 0 else -math.inf
    if p >= 1.0:
        return 0.0 if w == M else -math.inf
    return (math.lgamma(M + 1) - math.lgamma(w + 1) - math.lgamma(M - w + 1)
            + w * math.log(p) + (M - w) * math.log1p(-p))


def binom_pmf(M: int, w: int, p: float) -> float:
    return math.exp(log_binom_pmf(M, w, p))


def bin_sums(weights, p_acc, fail):
    """Per-bin (n_w, sum P_acc, sum P_acc*fail) from per-shot results."""
    wmax = max(weights) if len(weights) else 0
    n = [0.0] * (wmax + 1)
    a = [0.0] * (wmax + 1)
    e = [0.0] * (wmax + 1)
    for w, pa, f in zip(weights, p_acc, fail):
        n[w] += 1.0
        a[w] += pa
        e[w] += pa * (1.0 if f else 0.0)
    return n, a, e


def reweight(n, a, e, M: int, p: float):
    """Eq. (reweight) over the sampled bins; returns dict with p_acc,
    p_acc_le, p_le and the truncation bound B."""
    pacc = 0.0
    ple_num = 0.0
    covered = 0.0
    for w in range(len(n)):
        if n[w] <= 0:
            continue
        b = binom_pmf(M, w, p)
        covered += b
        pacc += b * a[w] / n[w]
        ple_num += b * e[w] / n[w]
    wmax = len(n) - 1
    # B is the tail sum itself (Appendix "Systematics"), not 1 - head
    B = sum(binom_pmf(M, w, p) for w in range(wmax + 1, M + 1))
    return dict(p_acc=pacc, p_acc_le=ple_num,
                p_le=(ple_num / pacc) if pacc > 0 else float("nan"), B=B)


def standard_errors(n, a, e, M: int, p: float, a2=None, e2=None):
    """Standard errors of the two lines of Eq. (reweight).  The bins are
    independent samples, bin w holding n_w shots, so the variance of
    sum_w Bin_w(p) mean_w is sum_w Bin_w(p)^2 var_w / n_w, with var_w the
    variance of one shot's value in the bin: the unbiased sample variance
    (sum of squares - sum * mean) / (n_w - 1) when the sums of squares are
    given and n_w >= 2, else the Bhatia-Davis bound mean (1 - mean) of a
    variable in [0, 1].  Returns (sem of p_acc, sem of p_acc p_le)."""
    def var(w, s, s2):
        mu = s[w] / n[w]
        if s2 is not None and n[w] >= 2:
            return max(0.0, (s2[w] - s[w] * mu) / (n[w] - 1))
        return max(0.0, mu * (1.0 - mu))

    va = ve = 0.0
    for w in range(len(n)):
        if n[w] <= 0:
            continue
        b = binom_pmf(M, w, p)
        va += b * b * var(w, a, a2) / n[w]
        ve += b * b * var(w, e, e2) / n[w]
    return math.sqrt(va), math.sqrt(ve)


def loss_multiplier(M: int, p_loss: float) -> float:
    """Multiplicative factor on the expected number of attempts when each
    of the M channels carries an independent loss of probability p_loss."""
    return (1.0 - p_loss) ** (-M)
