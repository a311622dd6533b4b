#!/usr/bin/env python3
"""Throughput benchmark: node-updates/s of PBN simulation on one MI355X.

One benchmark step is one pass of the whole hot path over the medium workload
(C2: n = 100 nodes, 1-4 predictors of 2-5 parents, 15% designated leaves,
p = 1e-3, 4096 trajectories x 10^6 steps):
  host preparation (validation, quantisation, leaf reduction, grouping,
  combined tables, device blob) -> upload -> s(0) -> 10^6 simulation steps in
  chunked launches (perturbation chain, predictor selection, table lookups,
  hit counting) -> per-trajectory counters -> steady-state estimate.

node-updates = trajectories x (burn-in + steps) x n_original (leaves count),
so the ratio of two kernels equals the paper's time-ratio speedup.

The JSON line also reports the plain per-node kernel (Method_old analogue:
no reduction, no grouping), the reduced kernel (Method_reduction analogue),
the roofline of the dominant kernel and the CPU oracle on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import pbn_synth as ps  # noqa: E402

PEAK_ALU = 256 * 64 * 2.4e9        # int32 VALU lane-operations per second (256 CUs x 64 lanes x 2.4 GHz)
L1_PROBE_LOG2 = 14                 # 16 KiB global probe buffer: fits the vector L1 of a CU
PHILOX_SLOTS = 60                  # 10 rounds x (2 full-rate 32x32->64 multiplies + 4 two-input xors)

# HBM bytes per k_simulate launch of the C2 and C3 workloads (product plans),
# from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch) scaled by what the same counters read for a 256 MiB device copy
# (fetch x 2.0, write x 1.0).  The kernel touches HBM only at launch
# boundaries (states, counters, plan tables), so a launch of any length moves
# the same bytes.  Valid only for the kernel source it was measured on, or a
# later source whose k_simulate instances compile to the same gfx950
# instructions (their assembly compared instance by instance, labels aside)
# with the same host plan builder.
SAME_CODE_SOURCES = (
    "96b5f63677dfb4de9a7cbe99aea9c6b59f49724fce4ae7323b25bb8d01d33968",   # counters taken here
    "d0a1234e9adf49cd7c8fe3c0b6ddf868809dba4a5b8f3c73b475d4a800cd960c",   # a compile-time check added; every kernel's code unchanged
    "97ee4dcda3638f74a8698679d3dd1de24e569094665c0907c1019a20966b3538",   # register-state kernels back to their previous form; the others unchanged
    "3af68a17e4e0cf6b992298558252103a962552b83cfa04b94025f4c4e5673817",   # host fallback for chain tables beyond LDS; kernels unchanged
)
MEASURED_TRAFFIC = {
    # per launch of the product plan: FETCH_SIZE and WRITE_SIZE (KiB per
    # dispatch) of one rocprofv3 --pmc run each, and the factors a 256 MiB
    # device copy reads for them (fetch 131 088 KiB, write 262 144 KiB)
    "C2": {"kernel_source_sha256": SAME_CODE_SOURCES,
           "plan": {"group": 0, "reduce": 1},
           "fetch_kib": 233.0, "fetch_factor": 2.0, "write_kib": 176.0, "write_factor": 1.0},
    "C3": {"kernel_source_sha256": SAME_CODE_SOURCES,
           "plan": {"group": 1, "max_group_nodes": 4, "max_parent_bits": 5, "reduce": 1},
           "fetch_kib": 12132.25, "fetch_factor": 2.0, "write_kib": 22016.0, "write_factor": 1.0},
}


def measured_traffic(cfg_name, opts):
    """Scaled HBM bytes per launch, or None when not measured for this
    workload and plan or the kernel source has changed since."""
    import hashlib
    m = MEASURED_TRAFFIC.get(cfg_name)
    if m is None or dict(opts) != m["plan"]:
        return None
    src = os.path.join(ROOT, "paper_1605_00854_amd", "csrc", "device.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() not in m["kernel_source_sha256"]:
            return None
    return int(round(1024 * (m["fetch_kib"] * m["fetch_factor"] + m["write_kib"] * m["write_factor"])))


PLANS = {
    "grouped": dict(reduce=1, group=1),
    "reduction": dict(reduce=1, group=0),
    "cone": dict(reduce=2, group=0),
    "plain": dict(reduce=0, group=0),
    "alias": dict(reduce=1, group=0, sampling=1),
}


def algorithmic_ops(net, plan_info, slots_desc, n_targets, n_pairs):
    """VALU lane-operations one trajectory-step must perform (the work model).

    Every step draws the perturbation chain (1 + n p Philox calls on average)
    and compares; a step without perturbation (probability (1-p)^n) also draws
    the SEL blocks and evaluates every slot: 2 ops per parent bit gathered,
    3 per lookup/write, 4 per multi-predictor selection; hit tests cost 3 per
    target pair.
    """
    n, p = net["n"], net["p"]
    f = (1.0 - p) ** n
    B = plan_info["n_jobs"] - 1
    chain = PHILOX_SLOTS * (1 + n * p) + 2 * (1 + n * p)
    func = PHILOX_SLOTS * B + sum(2 * bits + 3 + 4 * nmulti for bits, nmulti in slots_desc)
    return chain + f * func + 3 * n_pairs + n_targets


def slot_work(net, plan):
    """(parent bits gathered, multi-predictor members) per slot of the plan."""
    slot, is_table = plan.slots()
    fn_off, par_off = net["fn_off"], net["par_off"]
    out = []
    for s in range(plan.info["n_slots"]):
        members = np.nonzero(slot == s)[0]
        nmulti = int(sum(1 for v in members if fn_off[v + 1] - fn_off[v] > 1))
        if is_table[s]:
            union = set()
            for v in members:
                for fi in range(fn_off[v], fn_off[v + 1]):
                    union.update(net["parents"][par_off[fi]:par_off[fi + 1]].tolist())
            out.append((len(union), nmulti))
        else:
            v = members[0]
            probs = net["sel_prob"][fn_off[v]:fn_off[v + 1]]
            phis = np.diff(par_off[fn_off[v]:fn_off[v + 1] + 1])
            out.append((float((probs * phis).sum()), nmulti))
    return out


def lds_work(net, plan, slots_desc):
    """LDS and image lookups one trajectory-step must make (the gather model).

    A step without perturbation gathers every slot's parent bits (one state
    byte each), writes one state byte per kept node, reads one drawn word per
    selecting slot, one combined-table entry per table slot and one 16-byte
    predictor record per multi-predictor FN slot (a one-predictor slot's
    record can stay in registers).  Returns per-trajectory-step counts:
    u8 (random byte gathers and stores), w4 (drawn words), rec16 (records) and
    tab8 (table entries), and where records and tables live ("lds" or
    "global"); for a global image, the vector-memory reads of vmem_work."""
    n, p = net["n"], net["p"]
    f = (1.0 - p) ** n
    slot, is_table = plan.slots()
    bits = bool(plan.opts.state_bits)
    gathers = sum(bits for bits, _ in slots_desc)
    n_multi_fn = sum(1 for (bits, nm), t in zip(slots_desc, is_table) if not t and nm)
    n_sel = sum(1 for (_, nm) in slots_desc if nm)
    n_tab = int(np.count_nonzero(is_table))
    return {"u8": f * (gathers + plan.info["n_kept"]), "w4": f * n_sel, "rec16": f * n_multi_fn,
            "tab8": f * n_tab, "image": "lds" if plan.info["image_in_lds"] else "global",
            "state": "bits" if bits else "bytes",
            "vmem": None if plan.info["image_in_lds"] else vmem_work(net, plan)}


# plan blob header words (pbn_plan_header, uint32 little-endian)
_H_N_PASSES, _H_IMAGE_BYTES, _H_IMAGE_OFF = 7, 12, 13
_H_FN_UNITS, _H_FN_JSHIFT, _H_FN_HOFF, _H_FN_VAR = 26, 27, 28, 39
_SLOT_TABLE, _SLOT_INLINE = 0x40000000, 0x20000000


def vmem_work(net, plan, samples=32, seed=1):
    """Vector-L1 accesses (64-byte units) one trajectory-step makes when the
    plan image stays in global memory, from the plan's own slot records and
    addresses.  Plans of more than two lane passes (streaming evaluation):
    every pass reads its 64 lanes' 16-byte slot records (16 units); table
    lanes read one table byte each, at a state-dependent offset (drawn
    uniformly here), plus union words and choice records when the slot record
    does not carry them; FN lanes and padded lanes read a choice record when
    they select, then one or two 16-byte units of the chosen predictor record
    (the choice drawn from the record's own thresholds).  Lanes of one read
    that fall in the same unit make one access.  Plans of one or two passes
    keep slot data in registers and skip the slot-record read.  Steps with a
    perturbation (1 - f of them) read only Q words, not counted.  Returns
    per-step accesses and wave-level read instructions."""
    rng = np.random.default_rng(seed)
    f = (1.0 - net["p"]) ** net["n"]
    blob = plan.blob()
    hdr = np.frombuffer(blob[:4 * 41].tobytes(), dtype="<u4").astype(np.int64)
    n_passes, img, img_bytes = int(hdr[_H_N_PASSES]), int(hdr[_H_IMAGE_OFF]), int(hdr[_H_IMAGE_BYTES])
    fn_units, fn_jshift, fn_hoff, fn_var = (int(hdr[i]) for i in (_H_FN_UNITS, _H_FN_JSHIFT, _H_FN_HOFF, _H_FN_VAR))
    image = np.frombuffer(blob[img:img + img_bytes].tobytes(), dtype=np.uint8)
    words = np.frombuffer(image[:image.size // 4 * 4].tobytes(), dtype="<u4").astype(np.int64)
    rec = words[:256 * n_passes].reshape(-1, 4)          # 64 slot records of 16 bytes per pass
    info, y, z = rec[:, 0], rec[:, 1], rec[:, 2]
    table = (info & _SLOT_TABLE) != 0
    inline = (info & _SLOT_INLINE) != 0
    nmulti = (info >> 3) & 7
    nu = (info >> 6) & 31
    two = (nu > 5) if fn_var else np.full(info.shape, fn_units == 2)
    jshift = np.where(two, 5, 4) if fn_var else np.full(info.shape, fn_jshift)
    hoff = np.where(two, 16, 0) if fn_var else np.full(info.shape, fn_hoff)
    streaming = n_passes > 2 or plan.opts.state_bits

    def units(addr):
        return len(np.unique(np.asarray(addr) // 64))

    def choose(off):
        w = words[off // 4: off // 4 + 4]
        thr = w[1:1 + max(0, int(w[0] >> 24) - 1)]
        return int(np.count_nonzero(int(rng.integers(0, 1 << 32)) >= thr))

    acc = ins = 0.0
    for p in range(n_passes):
        sl = np.arange(64 * p, 64 * p + 64)
        if streaming:
            acc += units(16 * sl)
            ins += 1
        tl, fl = sl[table[sl]], sl[~table[sl]]
        for _ in range(samples):
            a = k = 0
            if tl.size:
                c = np.zeros(tl.size, dtype=np.int64)
                wide = tl[~inline[tl]]
                if wide.size:                 # union words, then members' choice records
                    uw = int(np.max((nu[wide] + 1) // 2))
                    for q in range(uw):
                        a, k = a + units(y[wide] + 4 * q), k + 1
                    for m in range(int(np.max(nmulti[wide]))):
                        has = wide[nmulti[wide] > m]
                        a, k = a + units(z[has] + 16 * m), k + 1
                        for i, s_ in enumerate(has):
                            c[np.searchsorted(tl, s_)] += choose(int(z[s_] + 16 * m)) * \
                                ((int(rec[s_, 3]) >> (8 * m)) & 0xFF)
                x = rng.integers(0, 1 << nu[tl])
                lst = np.where(inline[tl], 0, 32)      # inline slots: no union list before the table
                a, k = a + units(y[tl] + lst + (c << nu[tl]) + x), k + 1
            if fl.size:
                j = np.zeros(fl.size, dtype=np.int64)
                sel = fl[nmulti[fl] > 0]
                if sel.size:
                    a, k = a + units(z[sel]), k + 1
                    j[nmulti[fl] > 0] = [choose(int(z[s_])) for s_ in sel]
                ua = y[fl] + (j << jshift[fl])
                a, k = a + units(ua), k + 1
                tw = two[fl]
                if tw.any():
                    a, k = a + units(ua[tw] + hoff[fl][tw]), k + 1
            acc += a / samples
            ins += k / samples
    return {"accesses": f * acc, "instructions": f * ins}


def measure_gather_rates(api, torch, plan):
    """Chip-wide lane-lookup rates of the probe kernels (lookups/s): random byte
    gathers from an LDS buffer the size of the plan's state bytes, swizzled
    4- and 16-byte reads, and random 16-byte reads of a global buffer the size
    of the plan image."""
    from paper_1605_00854_amd import _lib
    L = api.lib()
    stream = torch.cuda.current_stream()
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    blocks, iters = 2048, 2048
    per_launch = blocks * 256 * iters * 8
    # the LDS buffer gathers read: one byte per node, or 4 bytes per 32 nodes
    # for packed-bit plans (whose gathers read words)
    lds_state = plan.info["state_bytes"] // (8 if plan.opts.state_bits else 1)
    state_bytes = max(128, 1 << int(math.ceil(math.log2(max(1, lds_state)))))
    img_log2 = max(L1_PROBE_LOG2, int(math.ceil(math.log2(max(16, plan.info["image_bytes"])))))
    buf = torch.zeros(1 << img_log2, dtype=torch.uint8, device="cuda")

    def timed(fn):
        fn()                                   # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        return per_launch / (e0.elapsed_time(e1) * 1e-3)

    sp = _lib.C.c_void_p(stream.cuda_stream)
    dsink = _lib.C.c_void_p(sink.data_ptr())
    out = {}
    for name, (lg, width, pattern) in {"u8_random": (int(math.log2(state_bytes)), 1, 0),
                                       "w4_random": (int(math.log2(state_bytes)), 4, 0),
                                       "w4_swizzled": (int(math.log2(state_bytes)), 4, 1),
                                       "rec16_swizzled": (min(16, img_log2), 16, 1),
                                       "rec16_random": (min(16, img_log2), 16, 0)}.items():
        def lds_probe(lg=lg, width=width, pattern=pattern):
            api.check(L.pbn_probe_lds_gather(lg, width, pattern, iters, blocks, dsink, sp))
        out[name] = timed(lds_probe)

    # global reads: a buffer that fits the vector L1 (every read hits: the
    # ceiling), and one the size of the plan image (reads spread over all of it)
    for name, (lg, width, pattern) in {"global16_rows": (L1_PROBE_LOG2, 16, 1),
                                       "global16_random": (L1_PROBE_LOG2, 16, 0),
                                       "global1_random": (L1_PROBE_LOG2, 1, 0),
                                       "global16_image_random": (img_log2, 16, 0)}.items():
        def vmem_probe(lg=lg, width=width, pattern=pattern):
            api.check(L.pbn_probe_vmem_gather(_lib.C.c_void_p(buf.data_ptr()), lg, width, pattern, iters // 4,
                                              blocks, dsink, sp))
        out[name] = timed(vmem_probe) / 4    # a quarter of the iterations per launch
    # the random 16-byte probe in accesses (64-byte units) per second: its 64
    # lanes fall in 64 random units of the L1-resident buffer, some shared
    units_l1 = (1 << L1_PROBE_LOG2) // 64
    out["l1_accesses"] = out["global16_random"] / 64 * units_l1 * (1 - (1 - 1 / units_l1) ** 64)
    out["state_buffer_bytes"] = state_bytes
    out["l1_buffer_bytes"] = 1 << L1_PROBE_LOG2
    out["image_buffer_bytes"] = 1 << img_log2
    return out


def roofline_head(ceil, alu_achieved, traj_steps_per_s):
    """bound / achieved / peak / unit / frac of the binding resource: the VALU
    in int32 lane-operations per second, LDS or vector memory in
    trajectory-steps per second at the ceiling the probes measured."""
    b = ceil["bound"]
    if b == "alu":
        return {"bound": "alu", "achieved": alu_achieved / 1e12, "peak": PEAK_ALU / 1e12,
                "unit": "Tops/s (int32 VALU lane-ops)", "frac": alu_achieved / PEAK_ALU}
    peak = 1.0 / ceil[b]["seconds_per_traj_step"]
    return {"bound": b, "achieved": traj_steps_per_s, "peak": peak,
            "unit": f"trajectory-steps/s ({'LDS' if b == 'lds' else 'vector-memory'} gather ceiling from the probes)",
            "frac": traj_steps_per_s / peak}


def ceilings(w_ops, work, rates, traj_steps_per_s):
    """Fractions of the VALU, LDS and vector-memory ceilings the kernel reaches.
    Each resource's time per trajectory-step at its measured (or nominal VALU)
    rate; the binding resource is the one with the largest fraction."""
    t_alu = w_ops / PEAK_ALU
    gather_rate = rates["w4_random"] if work.get("state") == "bits" else rates["u8_random"]
    t_lds = (work["u8"] / gather_rate + work["w4"] / rates["w4_swizzled"]
             + (work["rec16"] / rates["rec16_swizzled"] + work["tab8"] / rates["u8_random"]
                if work["image"] == "lds" else 0.0))
    vm = work.get("vmem")
    t_vmem = vm["accesses"] / rates["l1_accesses"] if work["image"] == "global" and vm else 0.0
    out = {}
    for name, t in (("alu", t_alu), ("lds", t_lds), ("vmem", t_vmem)):
        if t > 0:
            out[name] = {"seconds_per_traj_step": t, "frac": t * traj_steps_per_s}
    out["bound"] = max((k for k in out), key=lambda k: out[k]["frac"])
    return out


# ------------------------------------------------------------ CPU baseline

def _oracle_worker(args):
    from oracle import simulate as osim
    cfg_name, traj, steps = args
    cfg = ps.config(cfg_name)
    osim.run(cfg.net, cfg.seed, np.asarray(traj), steps, targets=cfg.targets)
    return len(traj)


def cpu_baseline(cfg_name, ntraj, steps):
    """The oracle as it stands, one worker per host core of this process's CPU
    share, on a bounded sample.  The share is the affinity set, at most 16
    cores: the GPU machine grants one GPU's job 16 cores whatever the machine
    shows."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    chunks = [c.tolist() for c in np.array_split(np.arange(ntraj), cores) if c.size]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(len(chunks)) as pool:
        pool.map(_oracle_worker, [(cfg_name, c, steps) for c in chunks])
    dt = time.perf_counter() - t0
    n = ps.config(cfg_name).net["n"]
    return {"value": ntraj * steps * n / dt, "unit": "node-updates/s", "cores": len(chunks),
            "host_cores_visible": os.cpu_count(), "affinity_cores": len(os.sched_getaffinity(0)),
            "kind": "oracle", "sample": f"{cfg_name}: {ntraj} trajectories x {steps} steps "
                                        f"(numpy oracle, unreduced network, one worker per core), "
                                        f"{dt:.1f} s wall"}


# --------------------------------------------------------------- GPU path

def run_step(api, torch, cfg, opts, plain, chunk, events, wpb=0, tpw=1):
    """One pass of the hot path.  Returns (estimate, half-width, prep seconds)."""
    net = cfg.net
    interest = sorted({a for tg in cfg.targets for a, _ in tg})
    t0 = time.perf_counter()
    plan = api.Plan(net, interest=interest, **opts)
    tg = plan.targets(cfg.targets)
    prep = time.perf_counter() - t0
    plan.device()
    state = api.state_init(plan, cfg.seed, cfg.ntraj)
    counts = api.new_counts(len(cfg.targets), cfg.ntraj)
    total = cfg.burn_in + cfg.steps
    step = 0
    stream = torch.cuda.current_stream()
    while step < total:
        c = min(chunk, total - step)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        api.simulate(plan, cfg.seed, state, counts, tg, step, c, count_from=cfg.burn_in, plain=plain,
                     waves_per_block=wpb, traj_per_wave=tpw)
        e1.record(stream)
        events.append((e0, e1, c))
        step += c
    # steady-state estimate of the first target through the library's
    # estimator (t interval over the trajectories' means)
    est = api.estimate(counts[0].cpu().numpy(), cfg.steps, conf=0.95)    # synchronises
    return plan, est["p_hat"], est["half_width"], prep


def tuned_opts_for(api, torch, nets, seed, ntraj=256, sample=4):
    """Autotune on a few networks spread over the size range; the options that
    win most often are used for all of them (ties: the faster total).  Also
    returns, per sampled network, the fastest trial with one trajectory per
    wavefront against the fastest with several (the batch kernel runs one)."""
    from paper_1605_00854_amd import autotune
    order = sorted(range(len(nets)), key=lambda k: nets[k]["n"])
    picks = [order[int(round(i * (len(order) - 1) / max(1, sample - 1)))] for i in range(sample)]
    votes = {}
    tpw_trials = []
    for k in picks:
        net = nets[k]
        tg = [ps.non_leaf_targets(net, 2)]
        interest = [a for a, _ in tg[0]]
        best, wpb, trials = autotune.tune(net, interest, tg, ntraj, seed=seed, probe_steps=500, quick=True,
                                          key=("multi", k, seed))
        key = tuple(sorted(best.items()))
        ok = [t for t in trials if "node_updates_per_s" in t]
        rate = max(t["node_updates_per_s"] for t in ok)
        v = votes.setdefault(key, [0, 0.0, wpb])
        v[0] += 1
        v[1] += rate
        one = max((t for t in ok if t.get("tpw", 1) == 1), key=lambda t: t["node_updates_per_s"])
        many = [t for t in ok if t.get("tpw", 1) > 1]
        row = {"n": int(net["n"]), "passes": one["passes"], "tpw1": one["node_updates_per_s"]}
        if many:
            m = max(many, key=lambda t: t["node_updates_per_s"])
            row.update({"best_tpw": m["tpw"], "tpw_rate": m["node_updates_per_s"],
                        "tpw_over_1": m["node_updates_per_s"] / one["node_updates_per_s"]})
        tpw_trials.append(row)
    best = max(votes.items(), key=lambda kv: (kv[1][0], kv[1][1]))
    return dict(best[0]), best[1][2], tpw_trials


def config_compare(api, torch, name, chunk, tag=None):
    """One full run of a fixed-length workload with the autotuned plan, then
    the reduction-only and the plain kernel on the same workload; the product
    kernel's launch times (HIP events on its stream) give its roofline."""
    from paper_1605_00854_amd import autotune
    cfg = ps.config(name)
    net = cfg.net
    n = net["n"]
    interest = sorted({a for tg in cfg.targets for a, _ in tg})
    t0 = time.perf_counter()
    opts, wpb, trials = autotune.tune(net, interest, cfg.targets, cfg.ntraj, seed=cfg.seed, quick=True)
    tpw = autotune.best_launch(trials)[1]
    t_tune = time.perf_counter() - t0
    work = cfg.ntraj * (cfg.burn_in + cfg.steps) * n
    out = {"workload": f"{name}: random PBN n={n}, p={net['p']}, {cfg.ntraj} trajectories x {cfg.steps} steps "
                       f"(+{cfg.burn_in} burn-in)", "autotune_seconds": t_tune, "autotune_trials": len(trials)}
    legs = {"product": (opts, not opts.get("group", 0), wpb, tpw), "reduction": (PLANS["reduction"], True, 0, 1),
            "plain": (PLANS["plain"], True, 0, 1)}
    for label, (o, plain, w, k) in legs.items():
        ev = []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plan, p_hat, hw, _ = run_step(api, torch, cfg, o, plain, chunk, ev, w, k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        kt = sum(e0.elapsed_time(e1) * 1e-3 for e0, e1, _ in ev)
        leg = {"node_updates_per_s": work / dt, "kernel_node_updates_per_s": work / kt, "seconds": dt,
               "plan": o, "waves_per_block": w or 4, "traj_per_wave": k, "n_kept": plan.info["n_kept"],
               "slots": plan.info["n_slots"],
               "table_slots": plan.info["n_table_slots"], "passes": plan.info["n_passes"],
               "image_in_lds": plan.info["image_in_lds"], "estimate": {"p_hat": p_hat, "half_width_95": hw}}
        if label == "product":
            durs = [(e0.elapsed_time(e1) * 1e-3, c) for e0, e1, c in ev]
            avg_launch = sum(d for d, _ in durs) / len(durs)
            avg_steps = sum(c for _, c in durs) / len(durs)
            npairs = sum(len(t) for t in cfg.targets)
            sd = slot_work(net, plan)
            w_step = algorithmic_ops(net, plan.info, sd, len(cfg.targets), npairs)
            rates = measure_gather_rates(api, torch, plan)
            ceil = ceilings(w_step, lds_work(net, plan, sd), rates, cfg.ntraj * avg_steps / avg_launch)
            leg["roofline"] = {**roofline_head(ceil, w_step * cfg.ntraj * avg_steps / avg_launch,
                                               cfg.ntraj * avg_steps / avg_launch),
                               "alu_frac": ceil["alu"]["frac"], "ceilings": ceil, "gather_rates": rates,
                               "traffic": measured_traffic(name, o),
                               "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                               "copy-calibrated)",
                               "kernel": "k_simulate", "ops_per_traj_step": w_step,
                               "avg_launch_ms": avg_launch * 1e3, "steps_per_launch": avg_steps}
        out[label] = leg
    out["product_over_plain"] = out["product"]["node_updates_per_s"] / out["plain"]["node_updates_per_s"]
    out["product_over_reduction"] = out["product"]["node_updates_per_s"] / out["reduction"]["node_updates_per_s"]
    out["reduction_over_plain"] = out["reduction"]["node_updates_per_s"] / out["plain"]["node_updates_per_s"]
    return out


def bench_batch(args):
    """C4: 512 uneven networks x 256 trajectories in one persistent launch per
    chunk, the chunks captured in one HIP graph."""
    import torch
    from paper_1605_00854_amd import api
    torch.cuda.set_device(0)
    nets = ps.batch_c4()
    ntraj, burn, T = 256, 10**4, 10**5
    if args.sim_steps:
        T = args.sim_steps
        burn = min(burn, T // 10)
    total = burn + T
    chunk = args.chunk if args.chunk < total else total
    passes = (total + chunk - 1) // chunk
    total = passes * chunk
    results = {}
    from paper_1605_00854_amd import autotune
    for label, opts in (("product", None), ("plain", dict(reduce=0, group=0))):
        if opts is None:
            opts, _, tpw_trials = tuned_opts_for(api, torch, nets, 4)
        t0 = time.perf_counter()
        items = []
        for k, net in enumerate(nets):
            tg = [ps.non_leaf_targets(net, 3)]
            plan = api.Plan(net, interest=[a for a, _ in tg[0]], **opts)
            items.append((plan, 1004000 + k, ntraj, tg))
        prep = time.perf_counter() - t0
        # the launch shape, timed on the batch itself (every leg alike)
        queues = args.queues or api.DEFAULT_QUEUES
        wpb, wpb_trials = autotune.batch_waves_per_block(items, count_from=burn, queues=queues)
        if args.wpb:
            wpb = args.wpb
        b = api.Batch(items, count_from=burn, waves_per_block=wpb, queues=queues)
        b.init_states()
        b.set_window(0, chunk)
        g = b.graph(passes)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.launch()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        work = sum(ntraj * total * net["n"] for net in nets)
        results[label] = {"node_updates_per_s": work / dt, "seconds": dt, "prep_seconds": prep,
                          "plan": opts, "waves_per_block": wpb, "wpb_trials": wpb_trials, "graph_passes": passes,
                          "chunk": chunk, "task_queues": queues}
        del g, b, items
    out = {"metric": "node-updates/sec on 1 MI355X (batched uneven networks, one graph replay)",
           "value": results["product"]["node_updates_per_s"], "unit": "node-updates/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"C4: 512 random PBNs n~U[20,1500], 256 trajectories each, "
                                  f"{T} steps + {burn} burn-in, hipGraph of {passes} persistent passes"},
           "compare": results,
           "product_over_plain": results["product"]["node_updates_per_s"] / results["plain"]["node_updates_per_s"],
           "traj_per_wave_trials": tpw_trials}
    print(json.dumps(out))


def serve_compare(api, torch, nq, query_chunk):
    """C5 served by the autotuned product plan and by the plain kernel: p50/p99
    latency from arrival to result and node-updates/s of each."""
    from paper_1605_00854_amd import serve
    nets = ps.served_c5()
    results = {}
    for label in ("product", "plain"):
        if label == "product":
            opts, wpb, tpw_trials = tuned_opts_for(api, torch, nets, 5)
        else:
            opts, wpb, tpw_trials = dict(reduce=0, group=0), 4, None
        srv = serve.Server(nets, [1005000 + k for k in range(len(nets))], plan_opts=opts, traj_per_query=256,
                           chunk=query_chunk, burn_in=1000, min_counted=1000, max_steps=200000,
                           waves_per_block=wpb)
        qs = serve.poisson_queries(nets, nq, rate=200.0, seed=2005)
        m = srv.run(qs, realtime=True)
        m["plan"] = opts
        if tpw_trials is not None:
            m["traj_per_wave_trials"] = tpw_trials
        results[label] = m
    return results


def bench_serve(args):
    """C5: Poisson stream of 2000 queries at 200/s over 64 resident networks."""
    import torch
    from paper_1605_00854_amd import api
    torch.cuda.set_device(0)
    nq = args.queries
    results = serve_compare(api, torch, nq, args.query_chunk)
    out = {"metric": "p50/p99 query latency and node-updates/sec on 1 MI355X (served queries)",
           "value": results["product"]["p99_latency_s"], "unit": "s (p99 latency)", "n_gpus": 1,
           "higher_is_better": False, "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"C5: {nq} queries, Poisson 200/s, 64 resident PBNs n~U[50,3000], "
                                  "1-5 target nodes, r in {1e-2, 5e-3}, conf 0.95, 256 trajectories per query, "
                                  f"chunks of {args.query_chunk} x 1, 2 or 4 steps by network cost"},
           "compare": results}
    print(json.dumps(out))


def bench_planner_fit(args):
    """Speedup of the autotuned plan over the plain kernel on synthetic networks
    spread over the paper's leaf-fraction and density ranges; Equation 7's
    form fit to them (R^2, 10-fold cross-validated R^2, held-out R^2)."""
    import torch
    from paper_1605_00854_amd import api, autotune, planner
    torch.cuda.set_device(0)
    ntraj, probe = 2048, 1000
    rows = {}
    for label, nets in (("fit", ps.planner_population(args.planner_fit, 2007)),
                        ("held_out", ps.planner_population(max(3, args.planner_fit // 3), 2008))):
        xs1, xs2, ys, rs = [], [], [], []
        for k, net in enumerate(nets):
            tg = [ps.non_leaf_targets(net, 3)]
            interest = [a for a, _ in tg[0]]
            x1, x2, _ = planner.features(net, interest)
            rs.append(planner.lane_pass_ratio(net, interest))
            plain = api.Plan(net, interest=interest, reduce=0, group=0)
            dt = autotune._probe(torch, plain, plain.targets(tg), 7, ntraj, probe, 4, True)
            r_plain = ntraj * probe * net["n"] / dt
            _, _, trials = autotune.tune(net, interest, tg, ntraj, seed=7, probe_steps=probe, quick=True,
                                         key=(label, k))
            r_best = max(t["node_updates_per_s"] for t in trials if "node_updates_per_s" in t)
            xs1.append(x1)
            xs2.append(x2)
            ys.append(max(r_best, r_plain) / r_plain)
            print(f"[planner] {label} {k} n={net['n']} leaf={x1:.3f} D={x2:.2f} speedup={ys[-1]:.3f}",
                  file=sys.stderr, flush=True)
        rows[label] = (np.array(xs1), np.array(xs2), np.array(ys), np.array(rs))
    x1, x2, y, r = rows["fit"]
    coeffs, r2 = planner.fit(x1, x2, y)
    cv = planner.cross_validated_r2(x1, x2, y)
    h1, h2, hy, hr = rows["held_out"]
    hp = planner.predict(h1, h2, coeffs)
    hr2 = 1.0 - float(((hy - hp) ** 2).sum()) / float(((hy - hy.mean()) ** 2).sum())
    # the same form per lane-pass ratio (the device's work comes in 64-lane passes)
    pcoeffs, pr2 = planner.fit_per_pass(x1, x2, r, y)
    pcv = planner.cross_validated_r2(x1, x2, y, ratio=r)
    pp = hr * planner.predict(h1, h2, pcoeffs)
    phr2 = 1.0 - float(((hy - pp) ** 2).sum()) / float(((hy - hy.mean()) ** 2).sum())
    out = {"metric": "planner speedup model (Equation 7 form) refit on MI355X", "value": r2, "unit": "R^2",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{args.planner_fit} + {h1.size} synthetic networks, {ntraj} trajectories, "
                                  f"{probe}-step probes"},
           "coeffs": coeffs, "r2": r2, "cv10_r2": cv, "held_out_r2": hr2,
           "held_out_mean_abs_error": float(np.abs(hy - hp).mean()),
           "per_pass": {"coeffs": pcoeffs, "r2": pr2, "cv10_r2": pcv, "held_out_r2": phr2,
                        "held_out_mean_abs_error": float(np.abs(hy - pp).mean())},
           "speedup_range": [float(y.min()), float(y.max())],
           "rows": {k: [list(map(float, v)) for v in r] for k, r in rows.items()}}
    print(json.dumps(out))


def bench_rl(args):
    """The paper's estimation procedure end to end on one trajectory: simulate,
    record the target indicator, diagnose (thinning, burn-in, sample size) and
    extend until the run is long enough (pbn_rl_run)."""
    cfg = ps.config(args.config)
    n = cfg.net["n"]
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.config, 1, 20000)
    import torch
    from paper_1605_00854_amd import api
    torch.cuda.set_device(0)
    interest = sorted({a for tg in cfg.targets for a, _ in tg})
    plan = api.Plan(cfg.net, interest=interest, reduce=1, group=0)
    api.rl_run(plan, cfg.seed + 1, cfg.targets, 0.05, initial_steps=1000, max_steps=1 << 20)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, _ = api.rl_run(plan, cfg.seed, cfg.targets, args.rl, initial_steps=100000, max_steps=(1 << 32) - 2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"metric": "two-state Markov chain estimate on 1 MI355X: simulated steps/s of the driver",
           "value": res["steps"] / dt, "unit": "steps/s (one trajectory)", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
           "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"{args.config}: one trajectory to precision {args.rl} at confidence 0.95 "
                                  f"(n = {n})", "plan": {"reduce": 1, "group": 0}},
           "result": {k: res[k] for k in ("status", "k", "alpha", "beta", "burn_in", "n_required", "p_hat",
                                          "steps")},
           "node_updates_per_s": res["steps"] * n / dt, "seconds": dt,
           "cpu_baseline": cpu}
    print(json.dumps(out))


def bench_skart(args):
    """The Skart stopping rule end to end on one trajectory: simulate, record the
    target indicator, analyse (batch size, spacers and warm-up, adjusted
    interval) and extend until the half-length meets the precision
    (pbn_skart_run)."""
    cfg = ps.config(args.config)
    n = cfg.net["n"]
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.config, 1, 20000)
    import torch
    from paper_1605_00854_amd import api
    torch.cuda.set_device(0)
    interest = sorted({a for tg in cfg.targets for a, _ in tg})
    plan = api.Plan(cfg.net, interest=interest, reduce=1, group=0)
    api.skart_run(plan, cfg.seed + 1, cfg.targets, 0.05, max_steps=1 << 20)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, _ = api.skart_run(plan, cfg.seed, cfg.targets, args.skart, max_steps=(1 << 32) - 2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"metric": "Skart estimate on 1 MI355X: simulated steps/s of the driver",
           "value": res["steps"] / dt, "unit": "steps/s (one trajectory)", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
           "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"{args.config}: one trajectory to precision {args.skart} at confidence 0.95 "
                                  f"(n = {n})", "plan": {"reduce": 1, "group": 0}},
           "result": {k: res[k] for k in ("status", "done", "batch_size", "batch_count", "spacer", "failures",
                                          "warmup", "ci_batches", "ci_batch_size", "p_hat", "lower", "upper",
                                          "half_width", "skewness", "lag1", "ar_factor", "steps")},
           "node_updates_per_s": res["steps"] * n / dt, "seconds": dt,
           "cpu_baseline": cpu}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--chunk", type=int, default=250000, help="simulation steps per kernel launch")
    ap.add_argument("--sim-steps", type=int, default=0, help="override T (for quick runs)")
    ap.add_argument("--ntraj", type=int, default=0, help="override the trajectory count (launch-shape studies)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain and reduction kernels")
    ap.add_argument("--no-extras", action="store_true",
                    help="default run only: skip the C3 and C5 legs (grouped product at n = 2000, served queries)")
    ap.add_argument("--wpb", type=int, default=0)
    ap.add_argument("--queues", type=int, default=0,
                    help="C4: task queues of the batched launch (default: the library's)")
    ap.add_argument("--tpw", type=int, default=0, help="trajectories per wavefront (default: the autotuner's)")
    ap.add_argument("--quick-tune", action="store_true")
    ap.add_argument("--queries", type=int, default=2000, help="C5: number of served queries")
    ap.add_argument("--query-chunk", type=int, default=500,
                    help="C5: base chunk (a query advances 1, 2 or 4 times this many steps per launch "
                         "of its lane, by its network's cost)")
    ap.add_argument("--plan", default="auto", choices=["auto", "plain", "reduction", "cone", "grouped", "alias"],
                    help="product plan: autotuned, or a fixed preparation (profiling runs)")
    ap.add_argument("--plan-opts", default="",
                    help="product plan options as JSON (e.g. '{\"reduce\": 1, \"group\": 1, \"max_parent_bits\": 5}'), "
                         "instead of the autotuner (profiling runs)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="MiB copied once by a plain device copy (HBM counter calibration in profiles)")
    ap.add_argument("--planner-fit", type=int, default=0,
                    help="refit the planner's speedup model on this many synthetic networks (plus a third "
                         "as many held out) and report the fit")
    ap.add_argument("--rl", type=float, default=0.0,
                    help="run the two-state Markov chain (Raftery-Lewis) driver on one trajectory of the "
                         "config to this precision instead of the fixed-length workload")
    ap.add_argument("--skart", type=float, default=0.0,
                    help="run the Skart driver on one trajectory of the config to this precision instead of "
                         "the fixed-length workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU only; sharding across GPUs is not implemented "
                                   "(trajectories shard by id, counters reduce with one integer all-reduce)"}))
        sys.exit(2)

    if args.planner_fit:
        return bench_planner_fit(args)
    if args.rl:
        return bench_rl(args)
    if args.skart:
        return bench_skart(args)
    if args.config == "C4":
        return bench_batch(args)
    if args.config == "C5":
        return bench_serve(args)
    cfg = ps.config(args.config)
    if args.sim_steps:
        cfg.steps = args.sim_steps
    if args.ntraj:
        cfg.ntraj = args.ntraj
    cpu = None
    if not args.no_cpu:
        # before any GPU initialisation: the pool forks
        # samples of about 10-20 s wall on 16 cores
        sample = {"C1": (1, 200000), "C2": (4096, 2000), "C2X": (2048, 1600), "C3": (256, 200)}[args.config]
        cpu = cpu_baseline(args.config, *sample)

    import torch
    from paper_1605_00854_amd import api
    torch.cuda.set_device(0)
    net = cfg.net
    n = net["n"]
    work = cfg.ntraj * (cfg.burn_in + cfg.steps) * n

    # autotuner: preparation options and launch shape, by short probe runs
    from paper_1605_00854_amd import autotune
    interest = sorted({a for tg in cfg.targets for a, _ in tg})
    if args.copy_probe:
        src = torch.ones(args.copy_probe << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t_tune = time.perf_counter()
    best_tpw = 1
    if args.plan_opts:
        best_opts, best_wpb, trials = json.loads(args.plan_opts), 4, []
    elif args.plan == "auto":
        best_opts, best_wpb, trials = autotune.tune(net, interest, cfg.targets, cfg.ntraj, seed=cfg.seed,
                                                    quick=args.quick_tune)
        best_tpw = autotune.best_launch(trials)[1]
    else:
        best_opts, best_wpb, trials = PLANS[args.plan], 4, []
    t_tune = time.perf_counter() - t_tune
    if args.wpb:
        best_wpb = args.wpb
    if args.tpw:
        best_tpw = args.tpw
    grouped_trials = [t for t in trials if t.get("opts", {}).get("group") and "node_updates_per_s" in t]
    best_grouped = max(grouped_trials, key=lambda t: t["node_updates_per_s"]) if grouped_trials else None
    product_plain = not best_opts.get("group", 0)

    for _ in range(args.warmup):
        run_step(api, torch, cfg, best_opts, product_plain, args.chunk, [], best_wpb, best_tpw)
    torch.cuda.synchronize()
    events = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan, p_hat, hw, prep = run_step(api, torch, cfg, best_opts, product_plain, args.chunk, events, best_wpb,
                                         best_tpw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.steps
    value = work * args.steps / dt

    # dominant kernel: the step kernel; algorithmic ops per launch / launch time
    durs = [(e0.elapsed_time(e1) * 1e-3, c) for e0, e1, c in events]
    avg_launch = sum(d for d, _ in durs) / len(durs)
    avg_steps = sum(c for _, c in durs) / len(durs)
    npairs = sum(len(t) for t in cfg.targets)
    sd = slot_work(net, plan)
    w_step = algorithmic_ops(net, plan.info, sd, len(cfg.targets), npairs)
    achieved = w_step * cfg.ntraj * avg_steps / avg_launch
    kernel_rate = cfg.ntraj * avg_steps * n / avg_launch
    rates = measure_gather_rates(api, torch, plan)
    ceil = ceilings(w_step, lds_work(net, plan, sd), rates, cfg.ntraj * avg_steps / avg_launch)

    compare = {}
    if not args.no_compare:
        variants = {"plain": (PLANS["plain"], True, 0), "reduction": (PLANS["reduction"], True, 0),
                    "cone": (PLANS["cone"], True, 0), "grouped_default": (PLANS["grouped"], False, 0)}
        if best_grouped:
            variants["grouped_tuned"] = (best_grouped["opts"], False, best_grouped["wpb"])
        # the paper's own sampling (Algorithms 1 and 2, one alias draw per
        # group) on the product plan: same law, different draws
        variants["alias_product"] = (dict(best_opts, sampling=1), product_plain, best_wpb)
        for name, (opts, plain, wpb) in variants.items():
            ev = []
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            pl, ph, _, _ = run_step(api, torch, cfg, opts, plain, args.chunk, ev, wpb)
            torch.cuda.synchronize()
            d = time.perf_counter() - t1
            kt = sum(e0.elapsed_time(e1) * 1e-3 for e0, e1, _ in ev)
            compare[name] = {"node_updates_per_s": work / d, "kernel_node_updates_per_s": work / kt,
                             "n_kept": pl.info["n_kept"], "slots": pl.info["n_slots"],
                             "table_slots": pl.info["n_table_slots"], "opts": opts, "p_hat": ph}
        compare["product_over_plain"] = value / compare["plain"]["node_updates_per_s"]
        compare["reduction_over_plain"] = (compare["reduction"]["node_updates_per_s"]
                                           / compare["plain"]["node_updates_per_s"])
        compare["cone_over_reduction"] = (compare["cone"]["node_updates_per_s"]
                                          / compare["reduction"]["node_updates_per_s"])
        compare["alias_over_product"] = compare["alias_product"]["node_updates_per_s"] / value
        for name in ("grouped_default", "grouped_tuned"):
            if name in compare:
                compare[name + "_over_plain"] = (compare[name]["node_updates_per_s"]
                                                 / compare["plain"]["node_updates_per_s"])

    out = {
        "metric": "node-updates/sec on 1 MI355X (grouped vs plain kernel)",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: random PBN n={n}, p={net['p']}, "
                               f"{cfg.ntraj} trajectories x {cfg.steps} steps (+{cfg.burn_in} burn-in)",
                   "n": n, "n_kept": plan.info["n_kept"], "slots": plan.info["n_slots"],
                   "table_slots": plan.info["n_table_slots"], "trajectories": cfg.ntraj,
                   "sim_steps": cfg.steps, "burn_in": cfg.burn_in,
                   "function_step_fraction": (1 - net["p"]) ** n,
                   "density": ps.density(net), "prep_seconds": prep,
                   "plan": best_opts, "waves_per_block": best_wpb, "traj_per_wave": best_tpw,
                   "autotune_seconds": t_tune,
                   "autotune_trials": len(trials),
                   "estimate": {"p_hat": p_hat, "half_width_95": hw}},
        "roofline": {**roofline_head(ceil, achieved, cfg.ntraj * avg_steps / avg_launch),
                     "ceilings": ceil, "gather_rates": rates,
                     "alu": {"achieved": achieved / 1e12, "peak": PEAK_ALU / 1e12, "frac": achieved / PEAK_ALU,
                             "unit": "Tops/s (int32 VALU lane-ops)", "philox_slots_per_call": PHILOX_SLOTS},
                     "traffic": measured_traffic(args.config, best_opts),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "k_simulate", "ops_per_traj_step": w_step,
                     "avg_launch_ms": avg_launch * 1e3, "steps_per_launch": avg_steps,
                     "kernel_node_updates_per_s": kernel_rate},
        "compare": compare,
        "cpu_baseline": cpu,
    }
    if args.config == "C2" and not args.no_extras:
        # the metric's other halves: the grouped product at the large workload
        # (C3) and served-query latency (C5), each against the plain kernel
        print("[bench] C3 product vs reduction vs plain", file=sys.stderr, flush=True)
        out["extra"] = {"C3": config_compare(api, torch, "C3", args.chunk)}
        print("[bench] C5 served queries", file=sys.stderr, flush=True)
        c5 = serve_compare(api, torch, args.queries, args.query_chunk)
        out["extra"]["C5"] = {"workload": f"C5: {args.queries} queries, Poisson 200/s, 64 resident PBNs "
                                          f"n~U[50,3000], chunks of {args.query_chunk} x 1, 2 or 4 steps "
                                          "by network cost",
                              **{k: {m: v[m] for m in ("p50_latency_s", "p99_latency_s", "node_updates_per_s",
                                                       "plan", "lanes") if m in v} for k, v in c5.items()}}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
