"""Skart stopping rule for one recorded output sequence (TEST INFRASTRUCTURE ONLY).

Parity unpinned: no published Skart implementation or worked example is
available here, so the constants below are this project's reading of the
published procedure; its components (skewness, the t interval, von Neumann's
test, Willink's adjustment, the correlation factor) and its end-to-end coverage
are pinned, the exact constants are not.

The paper names the Skart method beside the two-state Markov chain approach as
the statistical procedures its authors used for steady-state analysis of large
PBNs (Section 1, previous work); it does not restate it.  Skart (Tafazzoli,
Steiger and Wilson, IIE Transactions 43(2), 2011) is a sequential batch-means
procedure: it grows the batch size until the batch means are nearly symmetric
and pass a randomness test (with spacers between them, which also fixes a
warm-up period), then forms a confidence interval on the steady-state mean whose
half-length is adjusted for the skewness (Willink, 2005) and the lag-one
correlation of the batch means, and enlarges the sample until the half-length
meets the precision asked for.

This is the plain form of the procedure used here, step by step, on a complete
sequence x_0, x_1, ... (for a PBN trajectory, x_t = [s(t+1) hits the target]).
Each step states how many observations it needs; when the sequence is shorter
the procedure stops and reports that number, so that a driver can extend the
trajectory and replay it from the start (every decision depends only on a
prefix of the sequence, so a replay on a longer sequence takes the same
decisions up to that point).

Constants (our reading of the published procedure):
  initial batch count K0 = 1280, batch size 1; skewness measured on the last
  80 % of the batch means, batch size doubled while |skewness| > 4; randomness
  test: von Neumann's ratio, two-sided, size alpha_ran = 0.20 exp(-0.184 b^2)
  after b failures, spacers d = 0 .. 10 batches; after a failure at every
  spacer the batch size grows by sqrt(2) (ceiling) and the batch count shrinks
  to ceil(0.9 k) (not below 30); warm-up = d m observations; at most 1024
  batches in the interval; precision: an absolute half-length r.
Readings where the description leaves a choice: the randomness test uses every
(d+1)-th batch mean starting with batch d (0-based), the interval rebatches the
post-warm-up observations into min(k - d, 1024) batches, the correlation factor
is A = max(1, (1 + phi) / (1 - phi)) with phi clipped below 0.99, the
half-length is the larger of the two sides of the (asymmetric) interval, and a
sequence whose batch means are all equal asks for twice as many observations.
Every mean of batch means is the total of the observations it covers divided
by their number, so that equal batch means give deviations of exactly zero.
"""
import math

import numpy as np
from scipy import stats as _st

K0 = 1280
KMAX = 1024
KMIN = 30
SKEW_LIMIT = 4.0
ALPHA_RAN = 0.20
D_MAX = 10


def batch_sums(x, start, k, m):
    """Sums of k consecutive batches of m observations from x[start:] (exact
    integers for 0/1 observations)."""
    seg = np.asarray(x[start:start + k * m], dtype=np.float64)
    return seg.reshape(k, m).sum(axis=1)


def _mean(y, mean):
    return float(np.mean(y)) if mean is None else float(mean)


def _constant(y):
    return y.size == 0 or float(np.max(y)) == float(np.min(y))


def skewness(y, mean=None):
    """Adjusted Fisher-Pearson sample skewness; 0 for a constant sample."""
    y = np.asarray(y, dtype=np.float64)
    k = y.size
    if k < 3 or _constant(y):
        return 0.0
    dev = y - _mean(y, mean)
    m2 = float(np.sum(dev ** 2)) / k
    g1 = (float(np.sum(dev ** 3)) / k) / m2 ** 1.5
    return g1 * math.sqrt(k * (k - 1.0)) / (k - 2.0)


def von_neumann(y, mean=None):
    """von Neumann's ratio statistic C = 1 - sum (y_j - y_j+1)^2 / (2 sum (y_j - ybar)^2)
    and its null standard deviation sqrt((k - 2) / (k^2 - 1)); C = 0 for a
    constant sample."""
    y = np.asarray(y, dtype=np.float64)
    k = y.size
    sd = math.sqrt((k - 2.0) / (k * k - 1.0))
    if _constant(y):
        return 0.0, sd
    ss = float(np.sum((y - _mean(y, mean)) ** 2))
    return 1.0 - float(np.sum(np.diff(y) ** 2)) / (2.0 * ss), sd


def randomness_passes(y, alpha, mean=None):
    if len(y) < 3:
        return False
    c, sd = von_neumann(y, mean)
    return abs(c) <= float(_st.norm.ppf(1.0 - alpha / 2.0)) * sd


def lag1(y, mean=None):
    y = np.asarray(y, dtype=np.float64)
    if _constant(y):
        return 0.0
    dev = y - _mean(y, mean)
    return float(np.sum(dev[:-1] * dev[1:])) / float(np.sum(dev ** 2))


def willink_g(zeta, beta):
    """Willink's skewness-adjusted quantile: the g that solves
    zeta = g + beta + 2 beta g^2 + (4/3) beta^2 g^3 (g = zeta when beta = 0)."""
    if beta == 0.0:
        return zeta
    u = 6.0 * beta * (zeta - beta)
    # (1 + u)^(1/3) - 1 without cancellation when u is small
    root = math.expm1(math.log1p(u) / 3.0) if u > -1.0 else float(np.cbrt(1.0 + u)) - 1.0
    return root / (2.0 * beta)


def interval(y, conf, mean=None):
    """Skewness- and correlation-adjusted batch-means interval from batch means y."""
    y = np.asarray(y, dtype=np.float64)
    k = y.size
    mean = _mean(y, mean)
    var = 0.0 if _constant(y) else float(np.sum((y - mean) ** 2)) / (k - 1)
    c = skewness(y, mean)
    phi = min(lag1(y, mean), 0.99)
    a = max(1.0, (1.0 + phi) / (1.0 - phi))
    beta = c / (6.0 * math.sqrt(k))
    se = math.sqrt(a * var / k)
    tq = float(_st.t.ppf(0.5 + conf / 2.0, k - 1))
    lo = mean - willink_g(tq, beta) * se
    hi = mean - willink_g(-tq, beta) * se
    return {"mean": mean, "lower": lo, "upper": hi, "half_width": max(mean - lo, hi - mean),
            "skewness": c, "lag1": phi, "ar_factor": a, "var": var}


def skart(x, r, conf=0.95):
    """Run the procedure on the sequence x with absolute precision r.

    Returns a dict: done (precision met), n_required (observations needed next;
    the length used when done), and the state of the last step reached: m, k,
    d (spacer batches), b (randomness-test failures), warmup = d m, k_ci and
    m_ci (interval batches) and, once an interval was formed, p_hat, lower,
    upper, half_width, skewness, lag1, ar_factor."""
    x = np.asarray(x, dtype=np.float64)
    n_have = x.size
    st = {"done": False, "m": 1, "k": K0, "d": 0, "b": 0, "warmup": 0, "k_ci": 0, "m_ci": 0,
          "p_hat": float("nan"), "lower": float("nan"), "upper": float("nan"),
          "half_width": float("nan"), "skewness": float("nan"), "lag1": float("nan"),
          "ar_factor": float("nan")}

    def need(n):
        st["n_required"] = int(n)
        return st

    # batch size until the batch means are nearly symmetric
    m, k = 1, K0
    while True:
        if k * m > n_have:
            return need(k * m)
        sums = batch_sums(x, 0, k, m)
        tail = sums[k - int(0.8 * k):]
        if abs(skewness(tail / m, tail.sum() / (tail.size * m))) <= SKEW_LIMIT:
            break
        m *= 2
        st["m"] = m
    # randomness test of spaced batch means; the spacer fixes the warm-up
    b = 0
    while True:
        st["m"], st["k"], st["b"] = m, k, b
        if k * m > n_have:
            return need(k * m)
        sums = batch_sums(x, 0, k, m)
        alpha = ALPHA_RAN * math.exp(-0.184 * b * b)
        d = None
        for dd in range(D_MAX + 1):
            sp = sums[dd::dd + 1]          # every (d+1)-th batch, d spacer batches before each
            if randomness_passes(sp / m, alpha, sp.sum() / (sp.size * m)):
                d = dd
                break
        if d is not None:
            break
        b += 1
        m = int(math.ceil(math.sqrt(2.0) * m))
        k = max(int(math.ceil(0.9 * k)), KMIN)
    w = d * m
    st["d"], st["warmup"] = d, w
    # interval on the post-warm-up observations, enlarged until precise enough
    kc = min(k - d, KMAX)
    mc = (k * m - w) // kc
    while True:
        st["k_ci"], st["m_ci"] = kc, mc
        n = w + kc * mc
        if n > n_have:
            return need(n)
        sums = batch_sums(x, w, kc, mc)
        ci = interval(sums / mc, conf, sums.sum() / (kc * mc))
        st.update(p_hat=ci["mean"], lower=ci["lower"], upper=ci["upper"], half_width=ci["half_width"],
                  skewness=ci["skewness"], lag1=ci["lag1"], ar_factor=ci["ar_factor"])
        if ci["var"] > 0.0 and ci["half_width"] <= r:
            st["done"] = True
            return need(n)
        f = (ci["half_width"] / r) ** 2 if ci["var"] > 0.0 else 2.0
        grow = f * kc
        mc = int(math.ceil(mc * max(1.0, grow / KMAX)))
        kc = min(int(math.ceil(grow)), KMAX)
