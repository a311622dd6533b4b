"""Pins for the oracle's Skart stopping rule (the second steady-state procedure
the paper's authors name beside the two-state Markov chain approach, Section 1).

* Components against independent implementations or closed forms: the sample
  skewness equals scipy's bias-corrected skewness; for a symmetric sample with
  no positive lag-one correlation the interval is scipy's Student t interval;
  von Neumann's ratio tracks the lag-one correlation of long AR(1) sequences
  and its two-sided test has the asked size on iid normal samples.
* Willink's adjustment: the identity at zero skewness, and on right-skewed
  samples it balances the two tails that the t interval leaves unequal.
* The correlation factor: on AR(1) batch means (phi = 0.5) it averages
  (1 + phi) / (1 - phi) = 3 and brings the coverage back to the nominal 95 %.
* The batch-size rule: on iid Bernoulli data the batch size is the first power
  of two whose last 80 % of batch means have skewness at most 4.
* End to end: on two-state Markov chains and biased AR(1) sequences with known
  means, every finished run meets the precision and the 95 % intervals cover
  the mean at least 34 times in 40 seeds; replays on longer sequences take the
  same decisions; a constant sequence never finishes.
"""
import math

import numpy as np
import pytest
from scipy import stats as st

from oracle import skart as sk


def two_state_chain(alpha, beta, n, seed):
    """0/1 chain with P(0 -> 1) = alpha, P(1 -> 0) = beta, started in its
    stationary law: alternating runs of geometric lengths."""
    rng = np.random.default_rng(seed)
    pi1 = alpha / (alpha + beta)
    first = int(rng.random() < pi1)
    runs = []
    total = 0
    while total < n:
        # runs alternate between the two states: a run in state s lasts a
        # geometric number of steps with leaving probability beta (s = 1) or alpha
        pair = np.stack([rng.geometric(alpha, size=2048), rng.geometric(beta, size=2048)], axis=1)
        ln = (pair if first == 0 else pair[:, ::-1]).reshape(-1)
        runs.append(ln)
        total += int(ln.sum())
    lens = np.concatenate(runs)
    vals = (np.arange(lens.size) + first) % 2
    return np.repeat(vals, lens)[:n].astype(np.float64), pi1


def ar1(phi, n, seed, x0=0.0, mu=0.0):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(n)
    y = np.empty(n)
    p = x0 - mu
    for t in range(n):
        p = phi * p + e[t]
        y[t] = p
    return y + mu


def test_skewness_matches_scipy():
    rng = np.random.default_rng(5)
    for size in (3, 10, 1024):
        y = rng.exponential(size=size)
        assert sk.skewness(y) == pytest.approx(float(st.skew(y, bias=False)), rel=1e-12, abs=1e-12)
    assert sk.skewness(np.ones(50)) == 0.0


def test_symmetric_uncorrelated_interval_is_the_t_interval():
    rng = np.random.default_rng(6)
    half = rng.standard_normal(50)
    y = np.empty(100)
    y[0::2], y[1::2] = 3.0 + half, 3.0 - half          # zero skewness, negative lag-one correlation
    ci = sk.interval(y, 0.95)
    assert abs(ci["skewness"]) < 1e-12 and ci["ar_factor"] == 1.0
    lo, hi = st.t.interval(0.95, y.size - 1, loc=y.mean(), scale=st.sem(y))
    assert ci["lower"] == pytest.approx(lo, rel=1e-12) and ci["upper"] == pytest.approx(hi, rel=1e-12)


def test_von_neumann_ratio_tracks_lag_one_correlation():
    for phi in (0.5, -0.4, 0.0):
        c, sd = sk.von_neumann(ar1(phi, 40000, 7))
        assert c == pytest.approx(phi, abs=0.03)
        assert sd == pytest.approx(math.sqrt(39998 / (40000.0 ** 2 - 1)))


def test_von_neumann_test_has_its_size_on_iid_samples():
    rng = np.random.default_rng(8)
    for alpha in (0.2, 0.05):
        rej = sum(not sk.randomness_passes(rng.standard_normal(200), alpha) for _ in range(4000))
        assert abs(rej / 4000 - alpha) < 4 * math.sqrt(alpha * (1 - alpha) / 4000) + 0.01
    # and rejects positively correlated batch means
    rej = sum(not sk.randomness_passes(ar1(0.5, 200, 100 + s), 0.2) for s in range(200))
    assert rej > 190


def test_willink_adjustment():
    assert sk.willink_g(1.96, 0.0) == 1.96
    assert sk.willink_g(1.96, 1e-9) == pytest.approx(1.96, rel=1e-6)
    # right-skewed iid samples: the t interval misses above more often than
    # below; the adjusted interval evens the tails out
    rng = np.random.default_rng(9)
    k, reps = 20, 20000
    y = rng.exponential(size=(reps, k))
    miss_t = np.zeros(2)
    miss_w = np.zeros(2)
    tq = st.t.ppf(0.975, k - 1)
    for row in y:
        m, s = row.mean(), row.std(ddof=1) / math.sqrt(k)
        miss_t += (1.0 > m + tq * s, 1.0 < m - tq * s)
        beta = sk.skewness(row) / (6 * math.sqrt(k))
        lo, hi = m - sk.willink_g(tq, beta) * s, m - sk.willink_g(-tq, beta) * s
        miss_w += (1.0 > hi, 1.0 < lo)
    gap_t = abs(miss_t[0] - miss_t[1]) / reps
    gap_w = abs(miss_w[0] - miss_w[1]) / reps
    assert gap_t > 0.03 and gap_w < gap_t / 2
    # so the procedure's interval of right-skewed batch means reaches further up than down
    ci = sk.interval(rng.exponential(size=200), 0.95)
    assert ci["skewness"] > 0.5 and ci["upper"] - ci["mean"] > 1.05 * (ci["mean"] - ci["lower"])


def test_batch_size_rule_on_bernoulli_data():
    rng = np.random.default_rng(10)
    p = 0.002
    x = (rng.random(1280 * 512) < p).astype(np.float64)
    res = sk.skart(x, 1e-9)
    m = 1
    while abs(st.skew(x[:1280 * m].reshape(1280, m).mean(axis=1)[256:], bias=False)) > 4:
        m *= 2
    # the randomness test may raise m further, never lower it
    assert res["m"] >= m
    first = sk.skart(x[:1280 * m - 1], 1e-9)
    assert not first["done"] and first["n_required"] == 1280 * m


@pytest.mark.parametrize("alpha,beta,r", [(0.01, 0.05, 0.01), (0.002, 0.02, 0.01), (0.2, 0.3, 0.01)])
def test_two_state_chains_coverage(alpha, beta, r):
    covered = 0
    for seed in range(40):
        n = 1 << 17
        while True:
            x, pi1 = two_state_chain(alpha, beta, n, 1000 * seed + 17)
            res = sk.skart(x, r)
            if res["done"]:
                break
            assert res["n_required"] > n
            n = max(res["n_required"], 2 * n)
        assert res["half_width"] <= r
        covered += res["lower"] <= pi1 <= res["upper"]
    assert covered >= 34


def test_biased_ar1_coverage_and_warmup():
    covered, warm = 0, 0
    for seed in range(40):
        x = ar1(0.9, 600000, 500 + seed, x0=40.0, mu=2.0)
        res = sk.skart(x, 0.08)
        assert res["done"] and res["half_width"] <= 0.08
        covered += res["lower"] <= 2.0 <= res["upper"]
        warm += res["warmup"] > 0
    assert covered >= 34 and warm >= 30


def test_replay_on_a_longer_sequence_takes_the_same_decisions():
    x, _ = two_state_chain(0.01, 0.05, 1 << 21, 77)
    full = sk.skart(x, 0.01)
    assert full["done"]
    again = sk.skart(x[:full["n_required"]], 0.01)
    assert again == full
    short = sk.skart(x[:full["n_required"] - 1], 0.01)
    assert not short["done"] and short["n_required"] == full["n_required"]
    assert (short["m"], short["k"], short["d"], short["b"]) == (full["m"], full["k"], full["d"], full["b"])


def test_constant_sequence_never_finishes():
    res = sk.skart(np.zeros(1 << 16), 0.01)
    assert not res["done"] and res["n_required"] > (1 << 16)
    res = sk.skart(np.ones(1 << 20), 0.5)
    assert not res["done"] and res["n_required"] > (1 << 20)


def test_correlation_factor_restores_coverage():
    # batch means that are themselves AR(1) with phi = 0.5: the variance of their
    # mean is (1 + phi) / (1 - phi) = 3 times the iid figure
    rng = np.random.default_rng(11)
    covered, factors = 0, []
    for rep in range(1000):
        y = ar1(0.5, 400, int(rng.integers(1 << 30)))
        ci = sk.interval(y, 0.95)
        covered += ci["lower"] <= 0.0 <= ci["upper"]
        factors.append(ci["ar_factor"])
    assert np.mean(factors) == pytest.approx(3.0, rel=0.1)
    assert covered >= 920
