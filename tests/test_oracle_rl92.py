"""Pins for the oracle's Raftery-Lewis (1992) single-chain diagnosis, the
two-state Markov chain approach the paper uses for its estimates (Section 4.2).

* G^2 (second- against first-order chain) equals the sum over the middle state
  j of scipy's log-likelihood-ratio test of independence between z_{t-1} and
  z_{t+1} given z_t = j (an independent implementation of the same statistic).
* Thinning a first-order chain by k gives a first-order chain with
  alpha_k = alpha (1 - lambda^k) / (alpha + beta), lambda = 1 - alpha - beta;
  the estimates on long seeded chains fall within a few standard errors.
* The diagnosis keeps k = 1 for first-order and iid sequences, thins a
  second-order chain, and reports infinite sizes for a constant sequence.
"""
import math

import numpy as np
import pytest
from scipy import stats as st

from oracle import stats as os_


def markov1(alpha, beta, n, seed, z0=0):
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    z = np.empty(n, dtype=np.int64)
    z[0] = z0
    for t in range(1, n):
        z[t] = (u[t] < alpha) if z[t - 1] == 0 else (u[t] >= beta)
    return z


def markov2(n, seed):
    rng = np.random.default_rng(seed)
    z = [0, 0]
    for _ in range(n - 2):
        p = 0.9 if (z[-1] == 1 and z[-2] == 1) else (0.5 if z[-1] == 1 else 0.02)
        z.append(int(rng.random() < p))
    return np.asarray(z)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_g2_equals_conditional_independence_g_tests(seed):
    z = markov2(5000, seed) if seed == 1 else markov1(0.1, 0.3, 5000, seed)
    n = os_.triple_counts(z)
    want = 0.0
    for j in range(2):
        table = np.array([[n[0][j][0], n[0][j][1]], [n[1][j][0], n[1][j][1]]], dtype=float)
        if (table.sum(axis=0) == 0).any() or (table.sum(axis=1) == 0).any():
            continue
        want += st.chi2_contingency(table, correction=False, lambda_="log-likelihood")[0]
    assert os_.g2_second_vs_first(n) == pytest.approx(want, rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("k", [1, 2, 5])
def test_thinned_first_order_chain_transition_probabilities(k):
    a, b = 0.05, 0.2
    z = os_.thinned(markov1(a, b, 400000, 7), k)
    n01, n10, n0, n1 = os_.first_order_counts(z)
    lam = 1 - a - b
    ak = a * (1 - lam ** k) / (a + b)
    bk = b * (1 - lam ** k) / (a + b)
    assert abs(n01 / n0 - ak) < 5 * math.sqrt(ak * (1 - ak) / n0)
    assert abs(n10 / n1 - bk) < 5 * math.sqrt(bk * (1 - bk) / n1)


def test_diagnosis_keeps_first_order_and_iid_unthinned():
    for z in (markov1(0.05, 0.2, 200000, 11), (np.random.default_rng(12).random(100000) < 0.3).astype(int)):
        d = os_.rl92_diagnose(z, 1e-3)
        assert d["k"] == 1 and d["bic"] < 0


def test_diagnosis_thins_a_second_order_chain():
    d = os_.rl92_diagnose(markov2(200000, 13), 1e-3)
    assert d["k"] > 1
    assert os_.rl92_diagnose(os_.thinned(markov2(200000, 13), d["k"]), 1e-3)["k"] == 1


def test_alternating_sequence_needs_no_thinning_and_averages_one_half():
    # a deterministic period-2 sequence: a second-order chain predicts nothing
    # a first-order one does not (G^2 = 0), alpha = beta = 1, |1 - alpha - beta|
    # = 1 (the burn-in formula's logarithm is 0), no sampling error (N* = 0),
    # and the time average of an even-length window is exactly 1/2
    z = np.arange(10001) & 1
    d = os_.rl92_diagnose(z, 1e-3)
    assert d["k"] == 1 and d["g2"] == 0.0
    assert (d["alpha"], d["beta"]) == (1.0, 1.0)
    assert d["n_required"] == 0.0 and d["burn_in"] == 1.0
    assert d["p_hat"] == 0.5


def test_diagnosis_sizes_scale_with_k_and_constant_sequences_are_infinite():
    z = markov1(0.05, 0.2, 100000, 14)
    d = os_.rl92_diagnose(z, 1e-3)
    a, b, nreq, burn = os_.two_state(*os_.first_order_counts(z), 1e-3)
    assert d["n_required"] == pytest.approx(nreq) and d["burn_in"] == pytest.approx(burn)
    c = os_.rl92_diagnose(np.zeros(1000, dtype=int), 1e-3)
    assert math.isinf(c["n_required"]) and math.isinf(c["burn_in"]) and math.isnan(c["p_hat"])
