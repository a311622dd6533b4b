"""Steady-state estimators used with simulated trajectories.

The paper estimates steady-state probabilities with the two-state Markov chain
approach of Raftery and Lewis (cited in Sections 1 and 4.2 but not restated).
Here, from their published definitions:

* trajectory_mean_interval: p_hat = sum hits / (N T); half-width from the
  Student t quantile and the spread of the N per-trajectory means (N >= 2).
* batch_means_interval: one trajectory cut into B contiguous batches.
* two_state: for the hit indicator z_t, alpha = P(0 -> 1), beta = P(1 -> 0)
  estimated from transition counts; the required sample size
  N = alpha beta (2 - alpha - beta) / (alpha + beta)^3 * (Phi^-1((1+conf)/2) / r)^2
  and the burn-in m* = log(eps (alpha + beta) / max(alpha, beta)) / log|1 - alpha - beta|.
"""
import math

import numpy as np
from scipy import stats as _st


def trajectory_mean_interval(hits, T, conf=0.95):
    hits = np.asarray(hits, dtype=np.float64)
    N = hits.size
    means = hits / T
    p_hat = float(means.mean())
    if N < 2:
        return p_hat, float("nan")
    sd = float(means.std(ddof=1))
    tq = float(_st.t.ppf(0.5 + conf / 2.0, N - 1))
    return p_hat, tq * sd / math.sqrt(N)


def batch_means_interval(batch_hits, batch_len, conf=0.95):
    b = np.asarray(batch_hits, dtype=np.float64) / batch_len
    B = b.size
    p_hat = float(b.mean())
    tq = float(_st.t.ppf(0.5 + conf / 2.0, B - 1))
    return p_hat, tq * float(b.std(ddof=1)) / math.sqrt(B)


def two_state(n01, n10, n0, n1, r, conf=0.95, eps=1e-3):
    """alpha, beta from transition counts out of states 0 and 1; returns
    (alpha, beta, required sample size, burn-in)."""
    alpha = n01 / n0 if n0 else 0.0
    beta = n10 / n1 if n1 else 0.0
    if alpha + beta == 0.0:
        return alpha, beta, float("inf"), float("inf")
    z = float(_st.norm.ppf(0.5 + conf / 2.0))
    nreq = alpha * beta * (2.0 - alpha - beta) / (alpha + beta) ** 3 * (z / r) ** 2
    lam = abs(1.0 - alpha - beta)
    if lam == 0.0:
        burn = 1.0
    else:
        burn = math.log(eps * (alpha + beta) / max(alpha, beta)) / math.log(lam)
    return alpha, beta, nreq, burn
