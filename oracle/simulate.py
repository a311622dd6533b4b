"""Plain simulation of an independent-synchronous PBN with perturbations.

This is the paper's baseline simulation (Section 2.2, "Method_old" of Section 4)
on the *unreduced, ungrouped* network, one node at a time, with the random
draws fixed by `oracle.contract`:

  1. Perturbation (Eq. 1, Section 2.1): every node flips independently with
     probability p.  If any node flips, s(t+1) = s(t) XOR gamma(t) and no
     predictor function is applied in that step.
  2. Otherwise every node selects one predictor function by its selection
     probabilities and all nodes are updated synchronously from s(t).

Vectorised over trajectories; states are uint8 arrays (ntraj, n), node i in
column i.
"""
import numpy as np

from .contract import (PERT, SEL, draw, initial_state, multi_ranks,
                       perturbation_table, selection_thresholds)


class Network:
    """Decoded view of the CSR description for per-node evaluation."""

    def __init__(self, net):
        self.net = net
        self.n = int(net["n"])
        self.p = float(net["p"])
        fn_off = net["fn_off"]
        self.functions = []        # per node: list of (parents array, truth-table bit array)
        self.thresholds = []       # per node: integer thresholds CUM[0..l-2]
        for i in range(self.n):
            fl = []
            for f in range(int(fn_off[i]), int(fn_off[i + 1])):
                pa = net["parents"][net["par_off"][f]:net["par_off"][f + 1]].astype(np.int64)
                words = net["tt"][net["tt_off"][f]:net["tt_off"][f + 1]]
                bits = np.array([(int(words[j // 64]) >> (j % 64)) & 1
                                 for j in range(1 << pa.size)], dtype=np.uint8)
                fl.append((pa, bits))
            self.functions.append(fl)
            self.thresholds.append(selection_thresholds(net["sel_prob"][fn_off[i]:fn_off[i + 1]]))
        self.rank = multi_ranks(net)
        self.Q = perturbation_table(self.n, self.p)
        self.Qarr = np.array(self.Q[1:], dtype=np.uint64)   # Q[1..n]


def perturbation(nw, seed, traj, t):
    """gamma(t) for each trajectory: bool array (ntraj, n), drawn by the skip chain."""
    n = nw.n
    traj = np.asarray(traj, dtype=np.uint64)
    gamma = np.zeros((traj.size, n), dtype=bool)
    j0 = np.zeros(traj.size, dtype=np.int64)        # next node index to examine
    live = np.ones(traj.size, dtype=bool)
    while live.any():
        idx = np.nonzero(live)[0]
        x0, x1, _, _ = draw(seed, traj[idx], t, j0[idx], PERT)
        u = (x1 << np.uint64(32)) | x0
        # C = number of leading unperturbed nodes = #{h : Q[h] > u}
        C = (nw.Qarr[None, :] > u[:, None]).sum(axis=1)
        stop = C >= n - j0[idx]
        hit = idx[~stop]
        gamma[hit, j0[hit] + C[~stop]] = True
        j0[hit] = j0[hit] + C[~stop] + 1
        live[idx[stop]] = False
        live[hit[j0[hit] >= n]] = False
    return gamma


def function_update(nw, seed, traj, t, s):
    """f(t)(s(t)) for every trajectory: selection by thresholds, then evaluation."""
    n = nw.n
    traj = np.asarray(traj, dtype=np.uint64)
    out = np.zeros_like(s)
    cache = {}
    for i in range(n):
        fl = nw.functions[i]
        if len(fl) == 1:
            choice = np.zeros(traj.size, dtype=np.int64)
        else:
            r = int(nw.rank[i])
            if (r >> 2) not in cache:
                cache[r >> 2] = draw(seed, traj, t, r >> 2, SEL)
            u = cache[r >> 2][r & 3]
            choice = np.zeros(traj.size, dtype=np.int64)
            for c in nw.thresholds[i]:
                choice += (u >= np.uint64(c)).astype(np.int64)
        val = np.zeros(traj.size, dtype=np.uint8)
        for j, (pa, bits) in enumerate(fl):
            sel = choice == j
            if not sel.any():
                continue
            index = np.zeros(int(sel.sum()), dtype=np.int64)
            for k, par in enumerate(pa):
                index |= s[sel, par].astype(np.int64) << k
            val[sel] = bits[index]
        out[:, i] = val
    return out


def step(nw, seed, traj, t, s):
    """One transition s(t) -> s(t+1) of Eq. 1.  Returns (s_next, perturbed)."""
    gamma = perturbation(nw, seed, traj, t)
    pert = gamma.any(axis=1)
    s_next = function_update(nw, seed, traj, t, s)
    s_next[pert] = s[pert] ^ gamma[pert].astype(np.uint8)
    return s_next, pert


def target_hit(s, target):
    """[s matches every (node, value) of the target] per trajectory."""
    ok = np.ones(s.shape[0], dtype=bool)
    for node, val in target:
        ok &= s[:, node] == val
    return ok


def run(net, seed, traj, steps, *, step0=0, count_from=0, targets=(), state=None,
        nw=None, record=(), indicators=False):
    """Simulate `steps` transitions starting at global step `step0`.

    Returns a dict with the final state, per-target counters per trajectory
    (hits over transitions t >= count_from, and 0->1 / 1->0 transitions of the
    hit indicator between consecutive counted samples), the number of
    perturbed steps, and the states after the transitions listed in `record`;
    with `indicators`, also "z": the indicator of the first target after every
    transition, [trajectory][step - step0].
    """
    nw = nw or Network(net)
    traj = np.asarray(traj, dtype=np.uint64)
    s = initial_state(net, seed, traj) if state is None else state.copy()
    ntg = len(targets)
    hits = np.zeros((ntg, traj.size), dtype=np.int64)
    n01 = np.zeros((ntg, traj.size), dtype=np.int64)
    n10 = np.zeros((ntg, traj.size), dtype=np.int64)
    zprev = [target_hit(s, tg) for tg in targets]
    npert = np.zeros(traj.size, dtype=np.int64)
    snaps = {}
    zs = np.zeros((traj.size, steps), dtype=np.uint8) if indicators else None
    for t in range(step0, step0 + steps):
        s, pert = step(nw, seed, traj, t, s)
        npert += pert
        for q, tg in enumerate(targets):
            z = target_hit(s, tg)
            if indicators and q == 0:
                zs[:, t - step0] = z
            if t >= count_from:
                hits[q] += z
            if t >= count_from + 1:
                n01[q] += (~zprev[q]) & z
                n10[q] += zprev[q] & (~z)
            zprev[q] = z
        if t + 1 in record:
            snaps[t + 1] = s.copy()
    out = {"state": s, "hits": hits, "n01": n01, "n10": n10, "perturbed": npert, "snapshots": snaps}
    if indicators:
        out["z"] = zs
    return out
