"""Pins for the alias-sampling oracle (Sections 2.2, 3.2; Algorithm 2; Theorem 1).

* Vose's tables encode their target distributions (random distributions,
  degenerate ones, the 2^k perturbation patterns).
* Algorithm 2's group sizes on worked values.
* Theorem 1 by exact enumeration: masking the last group's pattern to its k'
  nodes leaves every node's flip probability at p, and the flips independent.
"""
import itertools

import numpy as np
import pytest

from oracle import alias


@pytest.mark.parametrize("seed", range(5))
def test_vose_encodes_the_distribution(seed):
    rng = np.random.default_rng(seed)
    L = int(rng.integers(1, 40))
    probs = rng.dirichlet(np.ones(L) * 0.5)
    keep, al = alias.vose(probs)
    assert all(0.0 <= k <= 1.0 for k in keep) and all(0 <= a < L for a in al)
    assert np.allclose(alias.encoded(keep, al), probs, atol=1e-12)


def test_vose_degenerate_and_uniform():
    assert alias.encoded(*alias.vose([1.0])) == [1.0]
    assert np.allclose(alias.encoded(*alias.vose([0.0, 1.0, 0.0])), [0, 1, 0])
    keep, al = alias.vose([0.25] * 4)
    assert keep == [1.0] * 4 and al == [0, 1, 2, 3]


def test_pattern_table_encodes_independent_flips():
    k, p = 6, 0.03
    dist = alias.pattern_probs(k, p)
    assert sum(dist) == pytest.approx(1.0)
    enc = alias.encoded(*alias.vose(dist))
    assert np.allclose(enc, dist, atol=1e-14)
    # each node flips with probability p, pairs independently
    for b in range(k):
        assert sum(q for c, q in enumerate(enc) if (c >> b) & 1) == pytest.approx(p)
    assert sum(q for c, q in enumerate(enc) if c & 0b11 == 0b11) == pytest.approx(p * p)


@pytest.mark.parametrize("n,want", [(100, (7, 15, 10)), (16, (1, 16, 16)), (17, (2, 9, 8)), (2000, (125, 16, 16)),
                                    (85, (6, 15, 10)), (1, (1, 1, 1))])
def test_group_params_worked_values(n, want):
    g, k, kp = alias.group_params(n, 16)
    assert (g, k, kp) == want
    assert k * (g - 1) + kp == n and 1 <= kp <= k <= 16


@pytest.mark.parametrize("k,kp", [(4, 1), (5, 3), (8, 8)])
def test_theorem_1_masked_last_group(k, kp):
    p = 0.1
    dist = alias.pattern_probs(k, p)
    marg = alias.masked_marginals(dist, kp)
    assert np.allclose(marg, [p] * kp)
    # the masked pattern of the k' nodes has exactly the k'-node pattern law
    mask = (1 << kp) - 1
    law = [0.0] * (1 << kp)
    for c, q in enumerate(dist):
        law[c & mask] += q
    assert np.allclose(law, alias.pattern_probs(kp, p))


def _brute_law(thr, al, L, bits, column_bits=None):
    """Law of a quantised table by enumerating every draw of a `bits`-bit word."""
    top = 1 << bits
    w = [0] * L
    if column_bits is not None:
        for col in range(L):
            for coin in range(top):
                w[col if coin < thr[col] else al[col]] += top >> column_bits
        return w
    for W in range(top):
        prod = W * L
        col, lo = prod >> bits, prod & (top - 1)
        w[col if lo < thr[col] else al[col]] += 1
    return w


@pytest.mark.parametrize("L,seed", [(3, 0), (5, 1), (7, 2), (12, 3), (16, 4)])
def test_quantised_law_matches_enumeration(L, seed, monkeypatch):
    # the closed-form counts of a one-word draw (column = high part of W * L,
    # coin = low part) checked by enumerating all 2^12 words of a 12-bit draw
    rng = np.random.default_rng(seed)
    bits = 12
    thr = [int(x) for x in rng.integers(0, 1 << bits, size=L)]
    al = [int(x) for x in rng.integers(0, L, size=L)]
    monkeypatch.setattr(alias, "TWO32", 1 << bits)
    assert alias.quantised_law(thr, al, L) == _brute_law(thr, al, L, bits)
    if L & (L - 1) == 0:
        kb = L.bit_length() - 1
        got = alias.quantised_law(thr, al, L, column_bits=kb)
        assert [x >> (32 - bits) for x in got] == _brute_law(thr, al, L, bits, kb)


@pytest.mark.parametrize("probs", [[0.5, 0.25, 0.25], [0.1, 0.2, 0.3, 0.4], [1e-9, 1 - 1e-9], [1.0]])
def test_quantised_tables_stay_within_one_word_of_the_target(probs):
    thr, al = alias.alias_table(probs)
    L = len(probs)
    law = alias.quantised_law(thr, al, L)
    assert sum(law) == 1 << 32
    # each column moves at most one word's weight of mass, plus the uneven
    # column sizes of a one-word draw
    for q, w in zip(probs, law):
        assert abs(w - q * 2 ** 32) <= 2 * L + 1


def test_pattern_table_quantised_law_and_theorem_1():
    k, kp, p = 10, 7, 1e-2
    probs = alias.pattern_probs(k, p)
    thr, al = alias.alias_table(probs)
    law = alias.quantised_law(thr, al, 1 << k, column_bits=k)
    assert sum(law) == 1 << 64
    dist = [w / 2.0 ** 64 for w in law]
    assert max(abs(a - b) for a, b in zip(dist, probs)) < 2 ** -31
    for m in alias.masked_marginals(dist, kp):
        assert m == pytest.approx(p, abs=2 ** -20)


def test_pattern_probs_are_the_product_form():
    k, p = 5, 0.3
    for c, q in enumerate(alias.pattern_probs(k, p)):
        m = bin(c).count("1")
        assert q == pytest.approx(p ** m * (1 - p) ** (k - m), rel=1e-15)


@pytest.mark.parametrize("l", [0, 1, 3, 40])
def test_leaf_threshold_gives_one_minus_t(l):
    p = 0.01
    t = alias.leaf_product(p, l)
    assert t == pytest.approx((1 - p) ** l, rel=1e-14)
    thr = alias.leaf_threshold(t, l)
    prob = ((1 << 32) - 1 - thr) / 2.0 ** 32       # P(W > thr)
    if l == 0:
        assert prob == 0.0
    else:
        assert abs(prob - (1 - t)) <= 2 ** -32


def test_combined_probs_first_member_most_significant():
    import pbn_synth as ps
    net = ps.random_pbn(6, 0.05, 9, nfn=lambda r: int(r.integers(2, 4)), nparents=lambda r: 2)
    fo, sp = net["fn_off"], net["sel_prob"]
    a, b = 1, 4
    la, lb = int(fo[a + 1] - fo[a]), int(fo[b + 1] - fo[b])
    got = alias.combined_probs(net, [a, b])
    for ja in range(la):
        for jb in range(lb):
            assert got[ja * lb + jb] == pytest.approx(sp[fo[a] + ja] * sp[fo[b] + jb], rel=1e-15)
    assert sum(got) == pytest.approx(1.0)


def _small_net(seed=31):
    import pbn_synth as ps
    return ps.random_pbn(7, 0.07, seed, nfn=lambda r: int(r.integers(1, 4)), nparents=lambda r: int(r.integers(1, 4)),
                         leaf_frac=0.3)


def _chi2_ok(counts, expected, alpha=1e-6):
    from scipy.stats import chi2
    counts, expected = np.asarray(counts, float), np.asarray(expected, float)
    big = expected >= 5
    obs = np.append(counts[big], counts[~big].sum())
    exp = np.append(expected[big], expected[~big].sum())
    keep = exp > 0
    stat = float(((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum())
    return chi2.sf(stat, int(keep.sum()) - 1) > alpha, stat


@pytest.mark.parametrize("reduce,group,steps", [(0, 1, 1), (1, 1, 1), (1, 0, 3), (0, 0, 2)])
def test_alias_steps_follow_equation_1(reduce, group, steps):
    # from a fixed state, the law of s(steps) over many trajectories is row s0
    # of P^steps (Eq. 1), restricted to the kept nodes when leaves are removed
    from oracle import exact
    net = _small_net()
    n = int(net["n"])
    interest = [v for v in range(n) if v not in set(int(x) for x in net["designated_leaves"])]
    plan = alias.alias_plan(net, interest, reduce=reduce, group=group, theta=10 ** 6, weight_mode=0)
    if reduce:
        assert len(plan["kept"]) < n
    if group:
        assert any(len(g) > 1 for g in plan["groups"])
    N = 30000
    s0 = 0b1011001 & ((1 << n) - 1)
    state = np.array([[(s0 >> v) & 1 for v in plan["kept"]]] * N, dtype=np.uint8)
    out = alias.simulate(net, plan, 77, np.arange(N), steps, state=state)
    idx = np.zeros(N, dtype=np.int64)
    for b, v in enumerate(plan["kept"]):
        idx |= out["reduced"][:, b].astype(np.int64) << b
    P = np.linalg.matrix_power(exact.transition_matrix(net), steps)[s0]
    S = np.arange(1 << n)
    exp = np.zeros(1 << len(plan["kept"]))
    red = np.zeros(S.size, dtype=np.int64)
    for b, v in enumerate(plan["kept"]):
        red |= ((S >> v) & 1) << b
    np.add.at(exp, red, P)
    ok, stat = _chi2_ok(np.bincount(idx, minlength=exp.size), exp * N)
    assert ok, stat


def test_alias_plan_parameters():
    net = _small_net()
    n = int(net["n"])
    leaves = set(int(x) for x in net["designated_leaves"])
    plan = alias.alias_plan(net, [v for v in range(n) if v not in leaves], reduce=1, group=0)
    nk = len(plan["kept"])
    assert (plan["g"], plan["k"], plan["kp"]) == alias.group_params(nk)
    assert plan["leaf_t"] == pytest.approx((1 - net["p"]) ** (n - nk))
    nfn = np.diff(net["fn_off"])
    assert [g[0] for g in plan["groups"]] == [v for v in plan["kept"] if nfn[v] >= 2]
    assert plan["n_jobs"] == (2 + 2 * plan["g"] + len(plan["groups"]) + 3) // 4


def test_group_perturbation_flips_each_node_with_p():
    # identity network: s(t+1) = s(t) unless perturbed, so s(1) ^ s(0) is the
    # perturbation vector; with n = 40 Algorithm 2 uses g = 3 groups of
    # k = 14 and a masked last group of k' = 12 (Theorem 1)
    import pbn_synth as ps
    from scipy.stats import binom
    n, p, N = 40, 0.05, 20000
    net = ps.assemble(n, p, [[(1.0, [i], np.array([0, 1]))] for i in range(n)])
    plan = alias.alias_plan(net, list(range(n)), reduce=0, group=0)
    assert (plan["g"], plan["k"], plan["kp"]) == (3, 14, 12) and plan["groups"] == []
    s0 = initial = np.zeros((N, n), dtype=np.uint8)
    out = alias.simulate(net, plan, 5, np.arange(N), 1, state=initial)
    flips = out["reduced"] ^ s0
    freq = flips.mean(axis=0)
    sigma = np.sqrt(p * (1 - p) / N)
    assert np.all(np.abs(freq - p) < 5 * sigma), freq
    ok, stat = _chi2_ok(np.bincount(flips.sum(axis=1), minlength=n + 1), binom.pmf(np.arange(n + 1), n, p) * N)
    assert ok, stat
    both = (flips[:, 0] & flips[:, 39]).mean()         # nodes of the first and the last group
    assert abs(both - p * p) < 5 * np.sqrt(p * p / N)
