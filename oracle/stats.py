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
  and the burn-in m* = log(eps (alpha + beta) / max(alpha, beta)) / log|1 - alpha - beta|
  (m* = 1 where that logarithm is -inf or 0: alpha + beta = 1, or alpha = beta = 1).
* rl92_diagnose: the full single-chain procedure of Raftery and Lewis (1992)
  on a recorded indicator sequence: the thinning interval k is the smallest k
  for which the k-thinned sequence is better described by a first-order than
  by a second-order Markov chain (BIC of the likelihood-ratio statistic G^2,
  two degrees of freedom); alpha, beta come from the k-thinned sequence, and
  burn-in and sample size are m* k and N* k original steps.
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
    if lam == 0.0 or lam == 1.0:
        # log(lam) is -inf or 0: lam = 0 is an independent sequence, stationary
        # after one step; lam = 1 with alpha + beta > 0 means alpha = beta = 1,
        # a deterministic alternation whose time average needs no warm-up
        burn = 1.0
    else:
        burn = math.log(eps * (alpha + beta) / max(alpha, beta)) / math.log(lam)
    return alpha, beta, nreq, burn


def thinned(bits, k):
    """z_0, z_k, z_2k, ... of a 0/1 sequence."""
    return np.asarray(bits, dtype=np.int64)[::k]


def triple_counts(z):
    """n[i][j][l] = #{t : z_t = i, z_{t+1} = j, z_{t+2} = l}, plain loops."""
    n = [[[0, 0], [0, 0]], [[0, 0], [0, 0]]]
    for t in range(len(z) - 2):
        n[int(z[t])][int(z[t + 1])][int(z[t + 2])] += 1
    return n


def g2_second_vs_first(n):
    """Likelihood-ratio statistic of a second-order against a first-order
    Markov chain for triple counts n[i][j][l]: 2 sum n_ijl log(P(l|i,j) / P(l|j)),
    both estimated by maximum likelihood; empty cells contribute 0."""
    g2 = 0.0
    for i in range(2):
        for j in range(2):
            nij = n[i][j][0] + n[i][j][1]
            for l in range(2):
                nijl = n[i][j][l]
                if nijl == 0:
                    continue
                njl = n[0][j][l] + n[1][j][l]
                nj = n[0][j][0] + n[0][j][1] + n[1][j][0] + n[1][j][1]
                g2 += 2.0 * nijl * math.log((nijl / nij) / (njl / nj))
    return g2


def first_order_counts(z):
    """(n01, n10, n0, n1): transitions 0->1 and 1->0 and the number of steps
    leaving state 0 and state 1."""
    n01 = n10 = n0 = n1 = 0
    for t in range(len(z) - 1):
        if z[t] == 0:
            n0 += 1
            n01 += int(z[t + 1] == 1)
        else:
            n1 += 1
            n10 += int(z[t + 1] == 0)
    return n01, n10, n0, n1


def rl92_diagnose(bits, r, conf=0.95, eps=1e-3, kmax=100):
    """Raftery-Lewis single-chain diagnosis of a recorded 0/1 sequence.

    Returns a dict: k (thinning), g2 and bic at k, alpha, beta (per k-step),
    burn_in = m* k and n_required = N* k (original steps), and p_hat, the mean
    of the sequence after ceil(burn_in) steps (nan when nothing is left)."""
    bits = np.asarray(bits, dtype=np.int64)
    k, g2, bic = kmax, float("nan"), float("nan")
    for kk in range(1, kmax + 1):
        z = thinned(bits, kk)
        if len(z) < 3:
            break
        g2 = g2_second_vs_first(triple_counts(z))
        bic = g2 - 2.0 * math.log(len(z) - 2)
        if bic < 0.0:
            k = kk
            break
    z = thinned(bits, k)
    n01, n10, n0, n1 = first_order_counts(z)
    alpha, beta, nstar, mstar = two_state(n01, n10, n0, n1, r, conf, eps)
    burn = mstar * k
    left = bits[int(math.ceil(burn)):] if math.isfinite(burn) else bits[:0]
    return {"k": k, "g2": g2, "bic": bic, "alpha": alpha, "beta": beta, "burn_in": burn,
            "n_required": nstar * k, "p_hat": float(left.mean()) if left.size else float("nan")}
