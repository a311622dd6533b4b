"""Alias sampling of Sections 2.2 and 3.2-3.4 (Walker's method, built with
Vose's construction), Algorithm 1's leaf draw, Algorithm 2's group
perturbation with Theorem 1's mask, and Algorithm 5's per-group selection of
combined predictor functions.

Test infrastructure (see oracle/__init__.py).  The library's alias sampling
mode is checked bit for bit against `simulate` below, which follows this
written draw contract (an independent implementation of the same definition,
like the Philox generator):

* Step t of trajectory r reads words W[4c + e] = output e of
  Philox(r, t, c, ALIAS = 4), c = 0, 1, ...
* W[0]: Algorithm 1.  With t_leaf = (1 - p)^l for the l removed nodes
  (a left-to-right product of l factors 1 - p from 1.0), a leaf is perturbed
  when W[0] > leaf_threshold(t_leaf) = ceil(t_leaf 2^32) - 1 (never when
  l = 0).  W[1] is not used.
* W[2 + 2q], W[3 + 2q]: Algorithm 2's draw for perturbation group q of the
  g = ceil(n' / 16) groups (k = ceil(n' / g) nodes each, k' in the last,
  kept nodes in ascending original id): column = the top k bits of the first
  word, kept when the second word is below the column's threshold, else its
  alias; the last group's pattern is ANDed with the mask of its k' low bits.
  Bit b of group q's pattern flips kept node q k + b.
* W[2 + 2g + s]: selecting group s (groups holding a multi-predictor node,
  numbered by their smallest node id) draws its combined index from its
  table of L columns: column = high word of W * L, kept when the low word is
  below the column's threshold, else its alias.
* Tables: Vose's construction in IEEE double (below), thresholds
  floor(keep 2^32), at most 2^32 - 1.  Pattern c of k nodes has probability
  the product over bits b = 0 .. k-1 of (p if bit b of c is set else 1 - p),
  multiplied left to right from 1.0; a combined index's probability is the
  product of its members' selection probabilities, first member first.

Functions
* vose(probs), encoded(keep, alias), thresholds(keep), alias_table(probs)
* group_params(n, kmax), pattern_probs(k, p), masked_marginals(dist, kp)
* leaf_product(p, l), leaf_threshold(t)
* quantised_law(thr, alias, L, column_bits) exact law of a quantised table
* alias_plan(net, interest, reduce, group, theta, weight_mode)
* simulate(net, plan, seed, traj, steps, ...)
"""
import math

import numpy as np

from . import structure
from .contract import draw, initial_state

ALIAS = 4
KMAX = 16            # Algorithm 2's k as set for the paper's experiments (Section 3.2)
TWO32 = 1 << 32


def vose(probs):
    """(keep, alias): column i is kept with probability keep[i], else it
    yields alias[i]; columns are drawn uniformly.  Stacks are Python lists in
    ascending index order, popped from the end."""
    L = len(probs)
    scaled = [float(q) * L for q in probs]
    keep = [0.0] * L
    alias = [0] * L
    small = [i for i, v in enumerate(scaled) if v < 1.0]
    large = [i for i, v in enumerate(scaled) if v >= 1.0]
    while small and large:
        s = small.pop()
        l = large.pop()
        keep[s] = scaled[s]
        alias[s] = l
        scaled[l] = scaled[l] + scaled[s] - 1.0
        if scaled[l] < 1.0:
            small.append(l)
        else:
            large.append(l)
    for i in large + small:          # what is left keeps itself (rounding leftovers)
        keep[i] = 1.0
        alias[i] = i
    return keep, alias


def encoded(keep, alias):
    L = len(keep)
    out = [0.0] * L
    for i in range(L):
        out[i] += keep[i] / L
        out[alias[i]] += (1.0 - keep[i]) / L
    return out


def thresholds(keep):
    return [min(TWO32 - 1, int(math.floor(k * 4294967296.0))) for k in keep]


def alias_table(probs):
    keep, alias = vose(probs)
    return thresholds(keep), alias


def group_params(n, kmax=KMAX):
    g = math.ceil(n / kmax)
    k = math.ceil(n / g)
    return g, k, n - k * (g - 1)


def pattern_probs(k, p):
    """Probabilities of the 2^k perturbation patterns (bit b of c: node b flips)."""
    p = float(p)
    q = 1.0 - p
    c = np.arange(1 << k, dtype=np.int64)
    v = np.ones(1 << k, dtype=np.float64)
    for b in range(k):
        v = v * np.where((c >> b) & 1, p, q)
    return [float(x) for x in v]


def masked_marginals(dist, kp):
    mask = (1 << kp) - 1
    marg = [0.0] * kp
    for c, q in enumerate(dist):
        m = c & mask
        for b in range(kp):
            if (m >> b) & 1:
                marg[b] += q
    return marg


def leaf_product(p, l):
    v = 1.0
    for _ in range(l):
        v = v * (1.0 - float(p))
    return v


def leaf_threshold(t, l):
    if l == 0:
        return TWO32 - 1
    return max(0, min(TWO32 - 1, math.ceil(t * 4294967296.0) - 1))


def quantised_law(thr, alias, L, column_bits=None):
    """Exact law (as fractions of 2^32 or 2^(32+column_bits)) of a quantised table.

    column_bits=None: one-word draw (column = high word of W * L, coin = low
    word).  column_bits=k: two-word draw (column = top k bits, coin = a full
    32-bit word).  Returns integer weights summing to the draw space size."""
    w = [0] * L
    if column_bits is not None:
        for c in range(L):
            w[c] += thr[c] << (32 - column_bits)
            w[alias[c]] += (TWO32 - thr[c]) << (32 - column_bits)
        return w
    for c in range(L):
        lo = -(-(c * TWO32) // L)                   # first W with high(W * L) = c
        hi = -(-((c + 1) * TWO32) // L)
        # W in [lo, hi): low word = W * L - c 2^32, increasing by L
        kept = min(hi, max(lo, -(-(thr[c] + c * TWO32) // L))) - lo
        w[c] += kept
        w[alias[c]] += (hi - lo) - kept
    return w


def combined_probs(net, members):
    """Probabilities of a group's combined indices (first member most significant)."""
    fo = net["fn_off"]
    radix = [int(fo[v + 1] - fo[v]) for v in members]
    L = int(np.prod(radix))
    out = []
    for c in range(L):
        digits, rest = [], c
        for r in reversed(radix):
            digits.append(rest % r)
            rest //= r
        digits.reverse()
        q = 1.0
        for v, j in zip(members, digits):
            q = q * float(net["sel_prob"][int(fo[v]) + j])
        out.append(q)
    return out


def alias_plan(net, interest, reduce=1, group=0, theta=65536, weight_mode=1, caps=None):
    """What the draws of alias sampling depend on: the kept nodes (Definition 1
    for reduce=1, the interest nodes' ancestors for reduce=2, all for 0), the
    selecting groups (Algorithm 4 over the kept multi-predictor nodes when
    grouping, else one per node) and the tables.

    caps = (max_nodes, max_bits, max_entries): a simulator's limits on a
    group's members, union parents and combined-table entries; a group of
    Algorithm 4 beyond them gives up its first (heaviest) member as a group of
    its own until it fits."""
    n = int(net["n"])
    if reduce == 1:
        removed = structure.leaf_nodes(net, interest)
    elif reduce == 2:
        removed = structure.cone_removed(net, interest)
    else:
        removed = set()
    kept = [v for v in range(n) if v not in removed]
    nfn = np.diff(net["fn_off"])
    multi = [v for v in kept if nfn[v] >= 2]
    if group:
        items = []
        for v in multi:
            par = set(p for pa, _ in structure.node_functions(net, v) for p in pa)
            w = int(nfn[v]) * (2 ** len(par) if weight_mode == 1 else 1)
            items.append((v, min(w, structure.SATURATE)))
        groups = [g for g in structure.partition_multi(items, theta) if g]
        if caps is not None:
            max_nodes, max_bits, max_entries = caps

            def fits(members):
                union = set(p for v in members for pa, _ in structure.node_functions(net, v) for p in pa)
                entries = int(np.prod([int(nfn[v]) for v in members])) << len(union)
                return len(members) <= max_nodes and len(union) <= max_bits and entries <= max_entries

            capped = []
            for members in groups:
                members = list(members)
                while len(members) > 1 and not fits(members):
                    capped.append([members[0]])
                    members = members[1:]
                capped.append(members)
            groups = capped
    else:
        groups = [[v] for v in multi]
    groups.sort(key=min)
    g, k, kp = group_params(len(kept))
    t = leaf_product(net["p"], n - len(kept))
    pthr, palias = alias_table(pattern_probs(k, net["p"]))
    tables = [alias_table(combined_probs(net, members)) for members in groups]
    nwords = 2 + 2 * g + len(groups)
    return dict(kept=kept, groups=groups, g=g, k=k, kp=kp, leaf_t=t,
                leaf_thr=leaf_threshold(t, n - len(kept)), pattern=(pthr, palias),
                tables=tables, n_jobs=(nwords + 3) // 4)


def _words(seed, traj, t, n_jobs):
    out = []
    for c in range(n_jobs):
        out.extend(draw(seed, traj, t, c, ALIAS))
    return np.stack(out, axis=1)          # (ntraj, 4 n_jobs) uint64 holding 32-bit values


def step(net, plan, fns, seed, traj, t, s):
    """One transition of Algorithm 5 on the reduced state s (ntraj, n')."""
    W = _words(seed, traj, t, plan["n_jobs"])
    g, k, kp = plan["g"], plan["k"], plan["kp"]
    pthr = np.array(plan["pattern"][0], dtype=np.uint64)
    palias = np.array(plan["pattern"][1], dtype=np.uint64)
    flips = np.zeros_like(s)
    anyc = np.zeros(s.shape[0], dtype=bool)
    for q in range(g):                       # Algorithm 2
        col = W[:, 2 + 2 * q] >> np.uint64(32 - k)
        c = np.where(W[:, 3 + 2 * q] < pthr[col], col, palias[col])
        width = kp if q == g - 1 else k
        c &= np.uint64((1 << width) - 1)
        for b in range(width):
            flips[:, q * k + b] = ((c >> np.uint64(b)) & np.uint64(1)).astype(np.uint8)
        anyc |= c != 0
    leaf = W[:, 0] > np.uint64(plan["leaf_thr"])   # Algorithm 1
    pert = anyc | leaf
    # predictor selection by group (Algorithm 5), then synchronous update
    choice = {}
    for si, members in enumerate(plan["groups"]):
        thr = np.array(plan["tables"][si][0], dtype=np.uint64)
        al = np.array(plan["tables"][si][1], dtype=np.uint64)
        radix = [len(fns[v]) for v in members]
        L = int(np.prod(radix))
        prod = W[:, 2 + 2 * g + si] * np.uint64(L)
        col = prod >> np.uint64(32)
        c = np.where((prod & np.uint64(TWO32 - 1)) < thr[col], col, al[col]).astype(np.int64)
        for kk in range(len(members) - 1, -1, -1):
            choice[members[kk]] = c % radix[kk]
            c = c // radix[kk]
    col_of = {v: i for i, v in enumerate(plan["kept"])}
    new = np.zeros_like(s)
    for i, v in enumerate(plan["kept"]):
        j = choice.get(v, np.zeros(s.shape[0], dtype=np.int64))
        val = np.zeros(s.shape[0], dtype=np.uint8)
        for jj, (pa, bits) in enumerate(fns[v]):
            sel = j == jj
            if not sel.any():
                continue
            idx = np.zeros(int(sel.sum()), dtype=np.int64)
            for b, par in enumerate(pa):
                idx |= s[sel, col_of[par]].astype(np.int64) << b
            val[sel] = np.array(bits, dtype=np.uint8)[idx]
        new[:, i] = val
    return np.where(pert[:, None], s ^ flips, new), pert


def simulate(net, plan, seed, traj, steps, *, step0=0, count_from=0, targets=(), state=None):
    """Trajectories of the reduced network under alias sampling.

    `state`: reduced state (ntraj, n') to start from, else s(0) of the
    contract restricted to the kept nodes.  Targets name original node ids
    (all kept).  Returns the final state in original node order (removed
    nodes 0) and the per-target counters as in oracle.simulate.run."""
    traj = np.asarray(traj, dtype=np.uint64)
    kept = plan["kept"]
    fns = {v: structure.node_functions(net, v) for v in kept}
    s = initial_state(net, seed, traj)[:, kept] if state is None else state.copy()
    col_of = {v: i for i, v in enumerate(kept)}

    def hit(st, tg):
        ok = np.ones(st.shape[0], dtype=bool)
        for node, val in tg:
            ok &= st[:, col_of[node]] == val
        return ok

    ntg = len(targets)
    hits = np.zeros((ntg, traj.size), dtype=np.int64)
    n01 = np.zeros((ntg, traj.size), dtype=np.int64)
    n10 = np.zeros((ntg, traj.size), dtype=np.int64)
    zprev = [hit(s, tg) for tg in targets]
    npert = np.zeros(traj.size, dtype=np.int64)
    for t in range(step0, step0 + steps):
        s, pert = step(net, plan, fns, seed, traj, t, s)
        npert += pert
        for q, tg in enumerate(targets):
            z = hit(s, tg)
            if t >= count_from:
                hits[q] += z
            if t >= count_from + 1:
                n01[q] += (~zprev[q]) & z
                n10[q] += zprev[q] & (~z)
            zprev[q] = z
    full = np.zeros((traj.size, int(net["n"])), dtype=np.uint8)
    full[:, kept] = s
    return {"state": full, "reduced": s, "hits": hits, "n01": n01, "n10": n10, "perturbed": npert}
