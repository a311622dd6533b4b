"""Pins for the oracle's structure analysis (Section 3).

* Definition 1 on hand-built graphs whose leaf sets are worked out by hand.
* The cone-of-influence reduction: hand-built graphs, and on random graphs a
  brute-force reachability check of every node, closure of the kept set under
  parents, and that it contains Definition 1's leaves.
* Equation 2 / Theorem 2: the bound never exceeds the true minimum number of
  groups found by brute force over all set partitions of small item lists.
* Algorithm 3 on a hand-traced example; Algorithm 4 meets its bound.
* Combined functions: selection probabilities of the combined functions sum to
  one (Section 3.3), a one-node group reproduces the node's truth tables, and
  each output bit depends only on its own member's chosen function.
"""
import itertools

import numpy as np
import pytest

import pbn_synth as ps
from oracle import structure as so


def graph(n, edges, self_loops=()):
    """Single-predictor network where node v reads the listed parents."""
    par = {v: [] for v in range(n)}
    for a, b in edges:            # a is a parent of b
        par[b].append(a)
    for v in self_loops:
        par[v].append(v)
    fns = []
    for v in range(n):
        k = len(par[v])
        fns.append([(1.0, par[v], [0] * (1 << k))])
    return ps.assemble(n, 0.1, fns)


def test_leaf_chain_collapses_to_interest():
    net = graph(4, [(0, 1), (1, 2), (2, 3)])
    assert so.leaf_nodes(net, [0]) == {1, 2, 3}
    assert so.leaf_nodes(net, [2]) == {3}
    assert so.leaf_nodes(net, [3]) == set()


def test_leaf_self_loop_and_cycle_are_kept():
    net = graph(5, [(0, 1), (1, 0), (0, 2), (3, 4)], self_loops=[3])
    # 2 and 4 are sinks; 0-1 is a cycle; 3 reads itself
    assert so.leaf_nodes(net, []) == {2, 4}


def test_cone_removes_unreachable_cycles_and_self_loops():
    # 0 -> 1 -> 2 (interest); 0 -> 3 <-> 4 (a cycle nobody reads); 5 reads itself
    # and 0; 6 is a sink
    net = graph(7, [(0, 1), (1, 2), (0, 3), (3, 4), (4, 3), (5, 6), (0, 5)], self_loops=[5])
    assert so.cone_removed(net, [2]) == {3, 4, 5, 6}
    assert so.leaf_nodes(net, [2]) == {6}               # Definition 1 keeps the cycle and the self-loop
    assert so.cone_removed(net, [4]) == {1, 2, 5, 6}    # 0 reaches 4 through 3
    assert so.cone_removed(net, [2, 6]) == {3, 4}
    assert so.cone_removed(net, []) == set(range(7))


def _reaches(net, v, targets):
    ch = so.children(net)
    seen, stack = {v}, [v]
    while stack:
        u = stack.pop()
        if u in targets:
            return True
        for c in ch[u]:
            if c not in seen:
                seen.add(c)
                stack.append(c)
    return False


@pytest.mark.parametrize("seed", range(6))
def test_cone_is_the_complement_of_the_ancestors(seed):
    rng = np.random.default_rng(seed)
    n = 24
    fns = []
    for v in range(n):
        k = int(rng.integers(0, 3))
        fns.append([(1.0, list(rng.choice(n, size=k, replace=False)), [0] * (1 << k))])
    net = ps.assemble(n, 0.1, fns)
    interest = sorted(rng.choice(n, size=2, replace=False).tolist())
    removed = so.cone_removed(net, interest)
    for v in range(n):                                   # brute force, node by node
        assert (v in removed) == (not _reaches(net, v, set(interest)))
    kept = set(range(n)) - removed
    for v in kept:                                       # closed under parents
        for f in range(int(net["fn_off"][v]), int(net["fn_off"][v + 1])):
            assert set(int(u) for u in net["parents"][net["par_off"][f]:net["par_off"][f + 1]]) <= kept
    assert so.leaf_nodes(net, interest) <= removed


def test_leaf_interest_sink_is_kept():
    net = graph(3, [(0, 1), (0, 2)])
    assert so.leaf_nodes(net, [2]) == {1}
    assert so.leaf_nodes(net, []) == {0, 1, 2}


def set_partitions(items):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in set_partitions(rest):
        for k in range(len(part)):
            yield part[:k] + [[first] + part[k]] + part[k + 1:]
        yield [[first]] + part


def true_min_groups(weights, theta):
    best = None
    for part in set_partitions(list(range(len(weights)))):
        total = sum(int(np.prod([weights[i] for i in g])) for g in part)
        if total <= theta and (best is None or len(part) < best):
            best = len(part)
    return best


@pytest.mark.parametrize("seed", range(40))
def test_eq2_is_a_lower_bound(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 7))
    w = [int(x) for x in rng.integers(2, 6, size=k)]
    theta = int(rng.integers(2, 200))
    mhat = so.eq2_lower_bound(w, theta)
    m_true = true_min_groups(w, theta)
    if m_true is not None:
        assert mhat is not None and mhat <= m_true
    if mhat is not None:
        # by definition m-hat satisfies Eq. 2 and m-hat - 1 does not
        W = int(np.prod(w))
        assert W * mhat ** mhat <= theta ** mhat
        if mhat > 1:
            assert W * (mhat - 1) ** (mhat - 1) > theta ** (mhat - 1)


def test_eq2_worked_values():
    # four nodes with 2 predictors each: W = 16.  theta = 8: m = 2 gives 2*4 = 8.
    assert so.eq2_lower_bound([2, 2, 2, 2], 8) == 2
    # min over m of m * 16^(1/m) is about 7.54 (m = 3): theta = 7 admits no m
    assert so.eq2_lower_bound([2, 2, 2, 2], 7) is None
    # eight nodes: W = 256; m = 4 gives 4 * 4 = 16, m = 3 gives 19.05
    assert so.eq2_lower_bound([2] * 8, 16) == 4
    assert so.eq2_lower_bound([2] * 8, 15) is None
    assert so.eq2_lower_bound([2, 2, 2, 2], 16) == 1


def test_find_partitions_hand_trace():
    items = [(10, 3), (11, 2), (12, 4), (13, 2), (14, 3)]
    # sorted: 12(4) 10(3) 14(3) 11(2) 13(2); groups start empty (weight 0)
    # 12 -> g0 [4]; 10 -> g1 [3]; 14 -> g1? no: g1=3 < g0=4 -> g1 [9];
    # 11 -> g0 [8]; 13 -> g0 (8 < 9) [16]
    assert so.find_partitions(items, 2) == [[12, 11, 13], [10, 14]]


def test_partition_multi_meets_theta_or_stops_at_singletons():
    rng = np.random.default_rng(2)
    for _ in range(50):
        k = int(rng.integers(1, 12))
        items = [(i, int(rng.integers(2, 5))) for i in range(k)]
        theta = int(rng.integers(4, 300))
        groups = so.partition_multi(items, theta)
        assert sorted(v for g in groups for v in g) == list(range(k))
        w = dict(items)
        total = sum(int(np.prod([w[v] for v in g])) for g in groups)
        assert total <= theta or len(groups) == k
        mhat = so.eq2_lower_bound([x for _, x in items], theta)
        if mhat is not None:
            assert len(groups) >= min(mhat, k)


def test_partition_multi_stops_when_the_sum_equals_theta():
    # Section 3.3's problem bounds the sum of group weights by theta (<=).
    # Four nodes of weight 2, theta = 8: Eq. 2 gives m = 2 (2 * 16^(1/2) = 8);
    # Algorithm 3 with m = 2 puts nodes 0, 2 in group 0 and 1, 3 in group 1
    # (ties go to the lower group), weights 4 + 4 = 8 <= 8, so Algorithm 4
    # stops there.  The literal strict test (8 < 8 fails at every m) would
    # end at four singletons.
    items = [(0, 2), (1, 2), (2, 2), (3, 2)]
    assert so.partition_multi(items, 8) == [[0, 2], [1, 3]]
    # one less than the sum: infeasible at every m, one group per item
    assert so.partition_multi(items, 7) == [[0], [1], [2], [3]]


def test_partition_multi_returns_the_first_feasible_m():
    # weights 3, 3, 2, 2, 2 (nodes 0..4), theta = 17.  Eq. 2: W = 72;
    # m = 1: 72 > 17; m = 2: 72 * 2^2 = 288 <= 17^2 = 289, so Algorithm 4 starts
    # at m = 2.  Algorithm 3, m = 2: 0 -> g0 (3), 1 -> g1 (3), 2 -> g0 (tie, 6),
    # 3 -> g1 (6), 4 -> g0 (tie, 12): 12 + 6 = 18 > 17, so m grows to 3:
    # 0 -> g0 (3), 1 -> g1 (3), 2 -> g2 (2), 3 -> g2 (4), 4 -> g0 (tie of 3 and
    # 3, 6): 6 + 3 + 4 = 13 <= 17.  m = 4 would also fit (3 + 3 + 4 + 2 = 12),
    # so returning anything but the first feasible m shows here.
    items = [(0, 3), (1, 3), (2, 2), (3, 2), (4, 2)]
    assert so.eq2_lower_bound([w for _, w in items], 17) == 2
    assert so.partition_multi(items, 17) == [[0, 4], [1], [2, 3]]


def test_group_single_ties_go_to_the_smaller_union_then_the_lower_index():
    # max_bits = 3.  Node 10 opens g0 = {1, 2}; node 11 ({3, 4}) would make g0's
    # union 4 bits, so it opens g1.  Node 12 ({5}) shares no parent with either
    # and both unions would be 3 bits: the lower index, g0, takes it.
    parents = {10: [1, 2], 11: [3, 4], 12: [5]}
    assert so.group_single([10, 11, 12], parents, max_nodes=4, max_bits=3) == [[10, 12], [11]]
    # max_bits = 4.  g0 = {1, 2, 3}; node 11 ({4, 5}) would give 5 bits: g1.
    # Node 12 ({6}) shares nothing with either; g0 would grow to 4 bits, g1 to
    # 3: the smaller union wins over the lower index.
    parents = {10: [1, 2, 3], 11: [4, 5], 12: [6]}
    assert so.group_single([10, 11, 12], parents, max_nodes=4, max_bits=4) == [[10], [11, 12]]
    # max_bits = 5.  g0 = {1, 2, 3, 4}; node 11 ({5, 6}) would give 6 bits: g1.
    # Node 12 ({1, 7}) shares parent 1 with g0 (union 5 bits) and nothing with
    # g1 (union 4 bits): shared parents come before the union size.
    parents = {10: [1, 2, 3, 4], 11: [5, 6], 12: [1, 7]}
    assert so.group_single([10, 11, 12], parents, max_nodes=4, max_bits=5) == [[10, 12], [11]]


def test_group_single_respects_caps_and_prefers_shared_parents():
    parents = {0: [5, 6], 1: [7, 8], 2: [5, 6, 9], 3: [7], 4: [1, 2, 3, 4]}
    groups = so.group_single([0, 1, 2, 3, 4], parents, max_nodes=2, max_bits=3)
    assert groups[0] == [0, 2]          # shares {5, 6}
    assert groups[1] == [1, 3]          # shares {7}
    assert groups[2] == [4]             # union cap
    for g in groups:
        assert len(g) <= 2
        assert len(set().union(*[parents[v] for v in g])) <= 3 or len(g) == 1


def test_combined_table_probabilities_and_members():
    net = ps.random_pbn(6, 0.1, 5, nfn=lambda r: int(r.integers(1, 4)),
                        nparents=lambda r: int(r.integers(1, 4)))
    members = [1, 3, 4]
    union, table = so.combined_table(net, members)
    fns = [so.node_functions(net, v) for v in members]
    probs = [net["sel_prob"][net["fn_off"][v]:net["fn_off"][v + 1]] for v in members]
    total = sum(np.prod(c) for c in itertools.product(*probs))
    assert abs(total - 1.0) < 1e-12
    radix = [len(f) for f in fns]
    assert table.shape == (int(np.prod(radix)), 1 << len(union))
    rng = np.random.default_rng(0)
    for _ in range(200):
        digits = [int(rng.integers(0, r)) for r in radix]
        c = 0
        for d, r in zip(digits, radix):
            c = c * r + d
        x = int(rng.integers(0, 1 << len(union)))
        vals = {p: (x >> b) & 1 for b, p in enumerate(union)}
        for k, (fl, j) in enumerate(zip(fns, digits)):
            pa, bits = fl[j]
            idx = sum(vals[p] << b for b, p in enumerate(pa))
            assert (int(table[c, x]) >> k) & 1 == bits[idx]


def test_combined_table_of_one_node_is_its_truth_tables():
    net = ps.assemble(3, 0.1, [[(0.5, [2, 0], [0, 1, 1, 0]), (0.5, [1], [1, 0])],
                               [(1.0, [0], [0, 1])], [(1.0, [1], [1, 1])]])
    union, table = so.combined_table(net, [0])
    assert union == [0, 1, 2]
    for x in range(8):
        s0, s1, s2 = x & 1, (x >> 1) & 1, (x >> 2) & 1
        assert table[0, x] == [0, 1, 1, 0][s2 | (s0 << 1)]
        assert table[1, x] == [1, 0][s1]
