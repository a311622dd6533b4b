"""Pins for the CPU oracle: each check ties it to something other than itself.

* Philox4x32-10 against PyTorch's independent header implementation.
* Quantisation against exact rational arithmetic.
* The perturbation skip chain against the Bernoulli(p) law of Eq. 1 (exact
  enumeration of the chain's law, then a large-sample test of the oracle code).
* Initial-state draws: every bit position is used once and is fair.
* Transition semantics against closed forms of Eq. 1 and against the exact
  steady state of the 2^n chain (power method / linear solve).
"""
import math
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats as st

import pbn_synth as ps
from oracle import contract, exact
from oracle import simulate as sim
from oracle.philox import philox4x32

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- Philox ----

@pytest.fixture(scope="module")
def torch_philox(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    exe = str(tmp_path_factory.mktemp("philox") / "ref")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", inc,
                    os.path.join(HERE, "torch_philox_ref.cpp"), "-o", exe], check=True)
    return exe


def test_philox_matches_torch_header(torch_philox):
    rng = np.random.default_rng(7)
    rows = [(0, 0, 0, 0, 0), ((1 << 64) - 1, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF)]
    for _ in range(300):
        rows.append((int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2)),
                     *[int(x) for x in rng.integers(0, 1 << 32, size=4)]))
    text = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([torch_philox], input=text, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for r, line in zip(rows, out):
        seed, c0, c1, c2, c3 = r
        got = [int(x) for x in philox4x32(c0, c1, c2, c3, seed & 0xFFFFFFFF, seed >> 32)]
        assert got == [int(x) for x in line.split()], r


def test_philox_outputs_are_uniform():
    w = philox4x32(np.arange(200000), 3, 1, 2, 11, 12)
    for word in w:
        bits = np.unpackbits(word.astype(np.uint32).view(np.uint8))
        assert abs(bits.mean() - 0.5) < 0.002


# ----------------------------------------------------------- Quantisation ---

@pytest.mark.parametrize("p", [0.01, 1e-3, 1e-4, 0.3, 0.5])
def test_perturbation_table_is_the_no_flip_probability(p):
    n = 3000
    Q = contract.perturbation_table(n, p)
    assert Q[0] == 1 << 64
    assert all(Q[h] >= Q[h + 1] for h in range(n))
    for h in (1, 2, 10, 100, n):
        exact_v = Fraction(1 - Fraction(p)) ** h if h < 200 else None
        ideal = (1 - p) ** h
        # h rounded products plus the floor to a multiple of 2^-64
        assert abs(Q[h] / 2.0 ** 64 - ideal) <= ideal * (h + 2) * 2.0 ** -52 + 2.0 ** -64
        if exact_v is not None:
            assert abs(Fraction(Q[h], 1 << 64) - exact_v) <= (exact_v * Fraction(h + 2, 1 << 52)
                                                              + Fraction(1, 1 << 64))


def test_selection_thresholds_round_partial_sums():
    rng = np.random.default_rng(3)
    for _ in range(2000):
        l = int(rng.integers(2, 6))
        probs = rng.dirichlet(np.ones(l))
        cum = contract.selection_thresholds(probs)
        assert len(cum) == l - 1
        assert all(a <= b for a, b in zip(cum, cum[1:]))
        acc = Fraction(0)
        for m in range(l - 1):
            acc += Fraction(float(probs[m]))
            # within half a unit plus the double-sum rounding of the partial sum
            assert abs(Fraction(cum[m]) - acc * (1 << 32)) <= Fraction(1, 2) + (m + 1) * Fraction(1 << 32, 1 << 52)
    # 1e-12 is 0.0043 of one 2^-32 unit: to the nearest unit, zero words select it
    assert contract.selection_thresholds([1.0 - 1e-12, 1e-12]) == [1 << 32]
    assert contract.selection_thresholds([0.5, 0.5]) == [1 << 31]
    assert contract.selection_thresholds([0.0, 1.0]) == [0]


def test_zero_selection_probability_never_fires():
    # Section 2.1: predictor j is chosen with probability c_j, so c_j = 0 means
    # never.  A predictor is reached by the 32-bit words u >= CUM[j-1] below
    # CUM[j]; after a partial sum of exactly 1 the threshold must exceed every
    # 32-bit word (the largest is 2^32 - 1), wherever the zeros sit.
    top = (1 << 32) - 1
    assert contract.selection_thresholds([0.5, 0.5, 0.0]) == [1 << 31, 1 << 32]
    assert contract.selection_thresholds([0.25, 0.75, 0.0, 0.0]) == [1 << 30, 1 << 32, 1 << 32]
    assert contract.selection_thresholds([1.0, 0.0]) == [1 << 32]
    for probs in ([0.5, 0.5, 0.0], [1.0, 0.0, 0.0, 0.0], [0.3, 0.7, 0.0], [0.125, 0.375, 0.5, 0.0]):
        cum = contract.selection_thresholds(probs)
        assert cum[-1] > top                       # no word selects the last predictor
    # a zero in the middle: equal thresholds leave no word between them
    cum = contract.selection_thresholds([0.5, 0.0, 0.5])
    assert cum == [1 << 31, 1 << 31]


# ---------------------------------------------------- Perturbation chain ---

def chain_law(n, p):
    """Exact law of gamma under the skip chain, from Q alone (enumeration)."""
    Q = contract.perturbation_table(n, p)
    law = {}
    for pat in range(1 << n):
        prob = Fraction(1)
        j0 = 0
        ones = [i for i in range(n) if (pat >> i) & 1]
        for i in ones:
            c = i - j0                       # C = c exactly: Q[c] > u >= Q[c+1]
            prob *= Fraction(Q[c] - Q[c + 1], 1 << 64)
            j0 = i + 1
        if j0 < n:                           # final draw must stop: u < Q[n - j0]
            prob *= Fraction(Q[n - j0], 1 << 64)
        law[pat] = prob
    return law


@pytest.mark.parametrize("n,p", [(1, 0.3), (5, 0.2), (8, 0.01), (6, 0.5)])
def test_chain_law_is_iid_bernoulli(n, p):
    law = chain_law(n, p)
    assert abs(float(sum(law.values())) - 1.0) < 1e-15
    for pat, prob in law.items():
        k = bin(pat).count("1")
        ideal = p ** k * (1 - p) ** (n - k)
        assert abs(float(prob) - ideal) <= 1e-13 * max(ideal, 1e-300) + 1e-300 + n * 2.0 ** -52 * ideal


def test_oracle_chain_matches_law_by_sampling():
    n, p = 6, 0.3
    net = ps.assemble(n, p, [[(1.0, [i], [0, 1])] for i in range(n)])
    nw = sim.Network(net)
    N = 200000
    law = chain_law(n, p)
    counts = np.zeros(1 << n)
    for t in range(2):
        g = sim.perturbation(nw, 99, np.arange(N), t)
        pats = (g.astype(np.int64) << np.arange(n)).sum(axis=1)
        counts += np.bincount(pats, minlength=1 << n)
    expected = np.array([float(law[k]) for k in range(1 << n)]) * counts.sum()
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < st.chi2.ppf(0.9999, (1 << n) - 1)
    # per-node marginal p and no positional bias
    g = sim.perturbation(nw, 5, np.arange(N), 0)
    marg = g.mean(axis=0)
    assert np.all(np.abs(marg - p) < 4 * math.sqrt(p * (1 - p) / N))


def test_oracle_chain_large_network_marginals():
    n, p = 2000, 1e-3
    net = ps.assemble(n, p, [[(1.0, [i], [0, 1])] for i in range(n)])
    nw = sim.Network(net)
    N = 20000
    g = sim.perturbation(nw, 17, np.arange(N), 3)
    none = 1 - g.any(axis=1).mean()
    assert abs(none - (1 - p) ** n) < 4 * math.sqrt(0.14 * 0.86 / N)
    assert abs(g.sum() / (N * n) - p) < 4 * math.sqrt(p / (N * n))
    # first and second half of the nodes flip equally often
    a, b = g[:, : n // 2].sum(), g[:, n // 2:].sum()
    assert abs(a - b) < 4 * math.sqrt(a + b)


# -------------------------------------------------------- Initial state ---

def test_initial_state_bits_are_fair_and_distinct():
    net = ps.assemble(300, 0.1, [[(1.0, [0], [0, 1])]] * 300)
    s = contract.initial_state(net, 5, np.arange(4000))
    assert abs(s.mean() - 0.5) < 0.005
    # no two node columns share the same draw
    cols = {s[:, i].tobytes() for i in range(300)}
    assert len(cols) == 300


# -------------------------------------------------- Transition semantics ---

def one_node(p, tt):
    return ps.assemble(1, p, [[(1.0, [0], tt)]])


def test_closed_form_constant_one():
    p = 0.05
    net = ps.assemble(1, p, [[(1.0, [0], [1, 1])]])
    pi = exact.steady_state(net)
    assert abs(pi[1] - 1 / (1 + p)) < 1e-12


def test_closed_form_negation():
    pi = exact.steady_state(one_node(0.2, [1, 0]))
    assert abs(pi[1] - 0.5) < 1e-12


def test_closed_form_identity_is_uniform():
    n = 5
    net = ps.assemble(n, 0.03, [[(1.0, [i], [0, 1])] for i in range(n)])
    pi = exact.steady_state(net)
    assert np.allclose(pi, 1 / 32, atol=1e-12)


def test_exact_matrix_rows_are_stochastic_and_mix_selection():
    # node 0 copies node 1 with prob 0.25, negates it with prob 0.75
    net = ps.assemble(2, 0.1, [[(0.25, [1], [0, 1]), (0.75, [1], [1, 0])],
                               [(1.0, [1], [0, 1])]])
    P = exact.transition_matrix(net)
    assert np.allclose(P.sum(axis=1), 1.0)
    # from state 0b10 (node1 = 1, node0 = 0), no perturbation (0.81):
    # node1 stays 1, node0 = 1 w.p. 0.25 -> state 0b11 gets 0.81 * 0.25 + 0.09 (flip node 0)
    assert abs(P[0b10, 0b11] - (0.81 * 0.25 + 0.1 * 0.9)) < 1e-15
    assert abs(P[0b10, 0b10] - 0.81 * 0.75) < 1e-15


def oracle_estimate(net, targets, seed, N, T):
    r = sim.run(net, seed, np.arange(N), T, targets=targets)
    return r["hits"] / T


@pytest.mark.parametrize("n,seed,p", [(3, 11, 0.1), (6, 12, 0.05), (8, 13, 0.02)])
def test_oracle_matches_power_method(n, seed, p):
    net = ps.random_pbn(n, p, seed, nfn=lambda r: int(r.integers(1, 4)),
                        nparents=lambda r: int(r.integers(1, 4)))
    targets = [[(0, 1)], [(1, 0), (2, 1)]]
    pi = exact.steady_state(net)
    means = oracle_estimate(net, targets, 4, 400, 1500)
    for q, tg in enumerate(targets):
        want = exact.target_probability(pi, tg)
        got = means[q].mean()
        hw = 3.29 * means[q].std(ddof=1) / math.sqrt(means.shape[1]) + 2e-3
        assert abs(got - want) < hw, (tg, got, want, hw)


def test_perturbed_step_applies_no_function():
    # every node is constant 0, so without perturbation the state would be 0.
    n = 4
    net = ps.assemble(n, 0.4, [[(1.0, [0], [0, 0])] for _ in range(n)])
    nw = sim.Network(net)
    traj = np.arange(5000)
    s = np.ones((traj.size, n), dtype=np.uint8)
    nxt, pert = sim.step(nw, 3, traj, 0, s)
    gamma = sim.perturbation(nw, 3, traj, 0)
    assert np.array_equal(nxt[pert], 1 - gamma[pert].astype(np.uint8))
    assert not nxt[~pert].any()
