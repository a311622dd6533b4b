"""Structure analysis of Section 3: leaf nodes, node grouping, combined functions.

Plain Python (sets, lists, big integers) written from the text:

* leaf_nodes        Definition 1 (Section 3.1), iterated removal of sinks
* cone_removed      the stronger reduction the same section's argument allows:
                    every node from which no node of interest can be reached
* eq2_lower_bound   Equation 2 and Theorem 2 (Section 3.3)
* find_partitions   the greedy multi-way partition of Algorithm 3
* partition_multi   Algorithm 4 on the multi-predictor nodes
* group_single      grouping of single-predictor nodes by shared parents (Sec. 3.3)
* combined_table    combined predictor functions of a group (Section 3.3)

Readings where the text is silent (also listed in the design notes):
* a self-edge makes a node its own child, so self-looped nodes are never leaves;
* Algorithm 4 stops at the first m whose partition weight sum is <= theta (the
  problem statement's bound) and never goes beyond one group per item;
* Algorithm 3 sorts by weight descending with node id ascending as tie-break,
  gives an empty group weight 0, and breaks ties by the lowest group index;
* products saturate at 2^62 so that both implementations stay in exact integers;
* single-predictor nodes are processed in node-id order and join the group
  sharing the most parents among those that stay within the node and parent
  caps; ties go to the smaller resulting parent union, then the lower index;
  a new group is opened when none fits;
* combined function index: the first member is the most significant digit
  (the enumeration f_1^a f_1^b, f_1^a f_2^b, ... of Section 3.3), and the
  first member's output is the least significant bit of the table entry.
"""
import math

import numpy as np

SATURATE = 1 << 62


def children(net):
    """children[v] = set of nodes having v as a parent in any predictor function."""
    n = int(net["n"])
    ch = [set() for _ in range(n)]
    fn_off, par_off, parents = net["fn_off"], net["par_off"], net["parents"]
    for i in range(n):
        for f in range(int(fn_off[i]), int(fn_off[i + 1])):
            for v in parents[par_off[f]:par_off[f + 1]]:
                ch[int(v)].add(i)
    return ch


def leaf_nodes(net, interest):
    """Set of leaf nodes (Definition 1): not of interest, no children left after
    iteratively removing leaf children."""
    n = int(net["n"])
    ch = children(net)
    interest = set(int(x) for x in interest)
    removed = set()
    changed = True
    while changed:
        changed = False
        for v in range(n):
            if v in removed or v in interest:
                continue
            if not (ch[v] - removed):
                removed.add(v)
                changed = True
    return removed


def cone_removed(net, interest):
    """Set of nodes from which no node of interest is reachable along
    parent -> child edges (the complement of the interest nodes' ancestors).

    Section 3.1 removes leaves because nothing of interest depends on them; the
    same argument removes every node outside the ancestor set of the nodes of
    interest, cycles included.  The ancestor set is closed under taking
    parents, so the kept nodes evolve exactly as in the full network.
    """
    n = int(net["n"])
    ch = children(net)
    parents = [set() for _ in range(n)]
    for v in range(n):
        for c in ch[v]:
            parents[c].add(v)
    keep = set(int(x) for x in interest)
    frontier = list(keep)
    while frontier:
        v = frontier.pop()
        for u in parents[v]:
            if u not in keep:
                keep.add(u)
                frontier.append(u)
    return set(range(n)) - keep


def sat_mul(a, b):
    return min(SATURATE, a * b)


def sat_prod(ws):
    out = 1
    for w in ws:
        out = sat_mul(out, w)
    return out


def eq2_lower_bound(weights, theta):
    """Smallest m >= 1 with m * (prod w)^(1/m) <= theta, i.e. prod w * m^m <= theta^m.

    Exact integer test.  Returns None when no m satisfies it (the left side is
    minimised near m = ln(prod w) and grows without bound afterwards).
    """
    W = 1
    for w in weights:
        W *= int(w)
    if not weights:
        return 0
    m = 1
    while True:
        if W * m ** m <= theta ** m:
            return m
        # ln m + ln(W)/m increases for m > ln W: past that point a failure is final
        if m >= math.log(W) + 1:
            return None
        m += 1


def find_partitions(items, m):
    """Algorithm 3.  items: list of (node, weight).  Returns m lists of nodes."""
    order = sorted(items, key=lambda it: (-it[1], it[0]))
    groups = [[] for _ in range(m)]
    prods = [0] * m                  # weight of an empty group is 0
    for node, w in order:
        best = min(range(m), key=lambda g: (prods[g], g))
        groups[best].append(node)
        prods[best] = w if not groups[best][:-1] else sat_mul(prods[best], w)
    return groups


def partition_multi(items, theta):
    """Algorithm 4 on the multi-predictor nodes: start at the Eq. 2 bound and add
    groups until the sum of group weights is <= theta (at most one group per item)."""
    if not items:
        return []
    weight = dict(items)
    if sum(w for _, w in items) > theta:
        # weights are >= 2, so a * b >= a + b: merging never lowers the sum and
        # no m below one group per item can meet theta
        return find_partitions(items, len(items))
    m0 = eq2_lower_bound([w for _, w in items], theta)
    m = len(items) if m0 is None else min(max(1, m0), len(items))
    while True:
        groups = find_partitions(items, m)
        total = 0
        for g in groups:
            total = min(SATURATE, total + sat_prod(weight[v] for v in g))
        if total <= theta or m >= len(items):
            return groups
        m += 1


def group_single(nodes, parent_sets, max_nodes, max_bits):
    """Single-predictor grouping by shared parents.  Returns a list of node lists."""
    groups, unions = [], []
    for v in nodes:
        pv = set(parent_sets[v])
        best, key = None, None
        for g, members in enumerate(groups):
            if len(members) >= max_nodes:
                continue
            u = unions[g] | pv
            if len(u) > max_bits:
                continue
            k = (-len(unions[g] & pv), len(u), g)
            if key is None or k < key:
                best, key = g, k
        if best is None:
            groups.append([v])
            unions.append(set(pv))
        else:
            groups[best].append(v)
            unions[best] |= pv
    return groups


def node_functions(net, i):
    """[(parents list, truth-table bits list)] of node i."""
    out = []
    for f in range(int(net["fn_off"][i]), int(net["fn_off"][i + 1])):
        pa = [int(x) for x in net["parents"][net["par_off"][f]:net["par_off"][f + 1]]]
        words = net["tt"][net["tt_off"][f]:net["tt_off"][f + 1]]
        bits = [(int(words[j // 64]) >> (j % 64)) & 1 for j in range(1 << len(pa))]
        out.append((pa, bits))
    return out


def combined_table(net, members):
    """Combined predictor functions of a group (Section 3.3).

    Returns (union parents in ascending node id, table) with
    table[c][x] = sum_k f^(members[k])_{j_k}(x) << k, where x indexes the union
    parents (bit b = value of union[b]) and the combined index c enumerates the
    member choices with the first member most significant.
    """
    fns = [node_functions(net, v) for v in members]
    union = sorted(set(p for fl in fns for pa, _ in fl for p in pa))
    pos = {p: b for b, p in enumerate(union)}
    radix = [len(fl) for fl in fns]
    ncomb = 1
    for r in radix:
        ncomb *= r
    table = np.zeros((ncomb, 1 << len(union)), dtype=np.int64)
    for c in range(ncomb):
        digits, rest = [], c
        for r in reversed(radix):
            digits.append(rest % r)
            rest //= r
        digits.reverse()
        for x in range(1 << len(union)):
            out = 0
            for k, (fl, j) in enumerate(zip(fns, digits)):
                pa, bits = fl[j]
                idx = 0
                for b, par in enumerate(pa):
                    idx |= ((x >> pos[par]) & 1) << b
                out |= bits[idx] << k
            table[c, x] = out
    return union, table
