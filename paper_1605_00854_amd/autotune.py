"""Autotuner: picks the preparation options (reduction, grouping caps, weights)
and the launch shape (wavefronts per workgroup, trajectories per wavefront) of
the step kernel by timing short probe runs on the device.

Every candidate simulates the same trajectories bit for bit (reduction and
grouping never change a kept node), so the choice is purely a speed choice.
The GPU payoff of the paper's node grouping depends on the network: grouping
pays when it removes whole lane passes or lets several cheap nodes share one
lookup (sparse networks with many single-predictor nodes), and loses when
combined tables need more parent bits than the nodes they merge (dense,
multi-predictor networks).
"""
import time

import numpy as np

from . import api

PLAIN = dict(reduce=0, group=0)
REDUCTION = dict(reduce=1, group=0)


def candidates(quick=False, reduce=1):
    """Plan options to probe.  `reduce` is the reduction the reduced
    candidates use: 1 (Definition 1's leaves) or 2 (the cone of influence of
    the nodes of interest, which removes a superset of the leaves)."""
    out = [PLAIN, dict(reduce=reduce, group=0)]
    bits = (4, 5, 6, 8) if quick else (4, 5, 6, 8, 10, 12)
    nodes = (2, 4) if quick else (2, 3, 4)
    for b in bits:
        for g in nodes:
            out.append(dict(reduce=reduce, group=1, max_parent_bits=b, max_group_nodes=g))
    out.append(dict(reduce=reduce, group=1, weight_mode=0, theta=1 << 20, max_parent_bits=8, max_group_nodes=4))
    return out


def best_reduction(net, interest):
    """2 when the cone-of-influence reduction removes more nodes than
    Definition 1 does (a subset of the kept nodes: never more work), else 1."""
    leaf = api.Plan(net, interest=interest, reduce=1, group=0).info["n_kept"]
    cone = api.Plan(net, interest=interest, reduce=2, group=0).info["n_kept"]
    return 2 if cone < leaf else 1


_CACHE = {}


def traj_per_wave_choices(plan, ntargets):
    """Trajectories per wavefront the step kernel accepts for a plan: 1, and
    2 .. 4 for keyed plans without table slots whose K slot sets fit four lane
    passes and whose K steps' draws fit one wave; only counts that save lane
    passes are worth probing."""
    out = [1]
    info = plan.info
    if info["n_table_slots"] or info["max_union_bits"] or plan.opts.sampling:
        return out
    S, passes = info["n_slots"], info["n_passes"]
    for k in (2, 3, 4):
        packed = (k * S + 63) // 64
        if packed <= 4 and k * info["n_jobs"] <= 64 and k * ntargets <= 64 and packed < k * passes:
            out.append(k)
    return out


def best_launch(trials):
    """(waves per workgroup, trajectories per wavefront) of the fastest trial."""
    ok = [t for t in trials if "node_updates_per_s" in t]
    best = max(ok, key=lambda t: t["node_updates_per_s"])
    return best["wpb"], best.get("tpw", 1)


def _probe(torch, plan, tg, seed, ntraj, steps, wpb, plain, tpw=1):
    state = api.state_init(plan, seed, ntraj)
    counts = api.new_counts(tg.ntargets, ntraj)
    api.simulate(plan, seed, state, counts, tg, 0, min(steps, 64), plain=plain, waves_per_block=wpb,
                 traj_per_wave=tpw)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    api.simulate(plan, seed, state, counts, tg, 64, steps, plain=plain, waves_per_block=wpb, traj_per_wave=tpw)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3


def batch_waves_per_block(items, count_from=0, wpbs=(2, 4, 8), probe_steps=200, queues=None):
    """Waves per workgroup of a batched persistent launch (api.Batch items),
    timed on the batch itself: how many networks share a CU, and its vector
    L1, depends on the workgroup size, which single-network probes cannot
    see.  Returns (the fastest, trials)."""
    import torch
    trials = []
    for wpb in wpbs:
        b = api.Batch(items, count_from=count_from, waves_per_block=wpb, queues=queues or api.DEFAULT_QUEUES)
        b.init_states()
        b.set_window(0, probe_steps)
        b.launch()                                  # warm-up: caches, first touch
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        b.set_window(probe_steps, probe_steps)
        e0.record(stream)
        b.launch()
        e1.record(stream)
        e1.synchronize()
        trials.append({"wpb": wpb, "seconds": e0.elapsed_time(e1) * 1e-3})
        del b
    best = min(trials, key=lambda t: t["seconds"])
    return best["wpb"], trials


def tune(net, interest, target_sets, ntraj, seed=1, probe_steps=2000, wpbs=(2, 4, 8), quick=False,
         key=None, verbose=False):
    """Return (best plan options, best waves_per_block, list of trials).

    Trials report node-updates/s of the probe (n_original per trajectory-step).
    """
    import torch
    key = key or (id(net), ntraj, tuple(interest), probe_steps, quick)
    if key in _CACHE:
        return _CACHE[key]
    n = int(net["n"])
    trials = []
    seen = set()
    for opts in candidates(quick, best_reduction(net, interest)):
        try:
            plan = api.Plan(net, interest=interest, **opts)
        except api._lib.PbnError as e:      # a cap the network cannot meet
            trials.append({"opts": opts, "error": str(e)})
            continue
        sig = (plan.info["n_slots"], plan.info["n_table_slots"], plan.info["max_union_bits"],
               plan.info["n_kept"], plan.info["image_in_lds"], plan.info["table_bytes"])
        if sig in seen:
            continue
        seen.add(sig)
        tg = plan.targets(target_sets)
        plain = plan.info["n_table_slots"] == 0
        for tpw in traj_per_wave_choices(plan, tg.ntargets):
            for wpb in wpbs:
                dt = _probe(torch, plan, tg, seed, ntraj, probe_steps, wpb, plain, tpw)
                rate = ntraj * probe_steps * n / dt
                trials.append({"opts": opts, "wpb": wpb, "tpw": tpw, "node_updates_per_s": rate,
                               "slots": plan.info["n_slots"], "table_slots": plan.info["n_table_slots"],
                               "passes": plan.info["n_passes"]})
                if verbose:
                    print(f"[autotune] {opts} wpb={wpb} tpw={tpw} slots={plan.info['n_slots']} "
                          f"tables={plan.info['n_table_slots']} {rate:.3e}", flush=True)
    ok = [t for t in trials if "node_updates_per_s" in t]
    best = max(ok, key=lambda t: t["node_updates_per_s"])
    out = (best["opts"], best["wpb"], trials)
    _CACHE[key] = out
    return out
