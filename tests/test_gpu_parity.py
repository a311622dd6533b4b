"""GPU parity: the HIP step kernel (through the C ABI) against the CPU oracle.

Trajectories are compared bit for bit on the kept nodes (the oracle simulates
the unreduced, ungrouped network; reduction and grouping must not change any
kept node, Section 3.1), together with the per-target hit and transition
counters.  Cases span several lane passes and a ragged last pass, Philox fills
that cover many steps and fills that need several lane passes, chains with
several perturbations, LDS- and global-resident plan images, combined tables
with several multi-predictor members, ragged trajectory counts and chunked
launches.
"""
import functools
import math
import sys

import numpy as np
import pytest

import pbn_synth as ps
from oracle import contract, exact
from oracle import simulate as osim

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1605_00854_amd import api  # noqa: E402

NONE = 0xFFFFFFFF


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# --------------------------------------------------------------- networks

def all_multi(n, seed, p=2e-3):
    return ps.random_pbn(n, p, seed, nfn=lambda r: int(r.integers(2, 5)),
                         nparents=lambda r: int(r.integers(1, 4)))


def all_single(n, seed, p=5e-3):
    return ps.random_pbn(n, p, seed, nfn=lambda r: 1, nparents=lambda r: int(r.integers(1, 6)))


def sparse_multi(n, seed, p=3e-3):
    # few parents per predictor so groups of multi-predictor nodes fit a table
    return ps.random_pbn(n, p, seed, nfn=lambda r: int(r.integers(1, 4)),
                         nparents=lambda r: int(r.integers(0, 3)), leaf_frac=0.2)


NETS = {
    "c1": ps.tiny_c1,
    "c2": ps.medium_c2,
    "c2_hot": lambda: ps.medium_c2(n=100, p=0.02, seed=31),
    "c2_small": lambda: ps.medium_c2(n=37, p=0.01, seed=8),
    "multi400": lambda: all_multi(400, 12),
    "single200": lambda: all_single(200, 13),
    "sparse120": lambda: sparse_multi(120, 14),
    "c3_slice": lambda: ps.large_c3(n=1500, p=2e-4, seed=15),
    "modules": lambda: ps.with_detached_modules(ps.medium_c2(n=60, p=3e-3, seed=16), 3, 20, seed=17),
    "wide40": lambda: ps.random_pbn(40, 1e-2, 18, nfn=lambda r: int(r.integers(1, 4)),
                                    nparents=lambda r: int(r.integers(1, 8)), leaf_frac=0.1),
    "interleaved": ps.interleaved_cone,
    "single64": lambda: all_single(64, 27, p=2e-3),
}


@functools.lru_cache(maxsize=None)
def net_of(name):
    return NETS[name]()


def targets_of(net):
    t1 = ps.non_leaf_targets(net, 3)
    t2 = [(t1[0][0], 0)]
    t3 = [(a, (a + 1) % 2) for a, _ in ps.non_leaf_targets(net, 2)]
    return [t1, t2, t3]


@functools.lru_cache(maxsize=None)
def oracle_run(name, seed, traj0, ntraj, steps, count_from):
    net = net_of(name)
    say(f"[oracle] {name} seed={seed} traj={traj0}+{ntraj} steps={steps}")
    return osim.run(net, seed, np.arange(traj0, traj0 + ntraj), steps, targets=targets_of(net),
                    count_from=count_from)


def gpu_run(name, opts, seed, traj0, ntraj, chunks, count_from=0, plain=False, wpb=0, tpw=1):
    net = net_of(name)
    tgs = targets_of(net)
    interest = sorted({a for tg in tgs for a, _ in tg})
    plan = api.Plan(net, interest=interest, **opts)
    say(f"[gpu] {name} opts={opts} info={plan.info} traj={traj0}+{ntraj} chunks={chunks} plain={plain} wpb={wpb} "
        f"tpw={tpw}")
    tg = plan.targets(tgs)
    state = api.state_init(plan, seed, ntraj, traj0=traj0)
    counts = api.new_counts(len(tgs), ntraj)
    step = 0
    for c in chunks:
        api.simulate(plan, seed, state, counts, tg, step, c, traj0=traj0, count_from=count_from,
                     plain=plain, waves_per_block=wpb, traj_per_wave=tpw)
        step += c
    orig = api.unpack_bits(api.to_original(plan, state).cpu().numpy(), plan.n)
    torch.cuda.synchronize()
    return plan, orig, counts.cpu().numpy(), state.cpu().numpy()


def check(name, opts, seed, traj0, ntraj, chunks, count_from=0, plain=False, wpb=0, tpw=1):
    ref = oracle_run(name, seed, traj0, ntraj, sum(chunks), count_from)
    plan, orig, counts, _ = gpu_run(name, opts, seed, traj0, ntraj, chunks, count_from, plain, wpb, tpw)
    kept = plan.node_pos() != NONE
    bad = np.nonzero((orig[:, kept] != ref["state"][:, kept]).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} trajectories differ, first {traj0 + bad[0]}"
    assert np.array_equal(counts[:, :, 0], ref["hits"])
    assert np.array_equal(counts[:, :, 1], ref["n01"])
    assert np.array_equal(counts[:, :, 2], ref["n10"])
    return plan


PLAIN = dict(reduce=0, group=0)
REDUCED = dict(reduce=1, group=0)
GROUPED = dict(reduce=1, group=1)
MULTI_GROUPS = dict(reduce=1, group=1, weight_mode=0, theta=10**6, max_table_entries=1 << 14,
                    max_parent_bits=12)
GLOBAL_IMAGE = dict(reduce=1, group=1, lds_budget_bytes=0)
CONE = dict(reduce=2, group=0)
CONE_GROUPED = dict(reduce=2, group=1)

CASES = [
    # name, opts, seed, traj0, ntraj, chunks, count_from, plain, wpb
    ("c1", PLAIN, 1, 0, 4, (3000,), 0, True, 0),
    ("c1", GROUPED, 1, 0, 4, (3000,), 0, False, 0),
    ("c2", PLAIN, 2, 0, 24, (300,), 0, True, 0),
    ("c2", REDUCED, 2, 0, 24, (300,), 0, True, 0),
    ("c2", GROUPED, 2, 0, 24, (300,), 0, False, 0),
    ("c2", MULTI_GROUPS, 2, 0, 24, (300,), 0, False, 0),
    ("c2", GLOBAL_IMAGE, 2, 0, 24, (300,), 0, False, 0),
    ("c2_hot", GROUPED, 3, 5, 16, (120, 80), 50, False, 2),
    ("c2_small", GROUPED, 4, 0, 37, (77, 23), 10, False, 4),
    ("multi400", GROUPED, 5, 0, 6, (60,), 0, False, 1),
    ("multi400", PLAIN, 5, 0, 6, (60,), 0, True, 3),
    ("single200", GROUPED, 6, 0, 8, (200,), 0, False, 0),
    ("sparse120", MULTI_GROUPS, 7, 0, 12, (150,), 0, False, 0),
    ("c3_slice", GROUPED, 8, 0, 3, (25,), 0, False, 0),
    ("modules", CONE, 18, 0, 20, (400,), 0, True, 0),
    ("modules", CONE_GROUPED, 18, 0, 20, (250, 150), 100, False, 2),
    ("single64", REDUCED, 22, 0, 30, (200, 123), 60, True, 0),    # one pass, no selection: predictor 0 undrawn
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{i}" for i, c in enumerate(CASES)])
def test_trajectories_bit_exact(case):
    name, opts, seed, traj0, ntraj, chunks, count_from, plain, wpb = case
    plan = check(name, opts, seed, traj0, ntraj, chunks, count_from, plain, wpb)
    if opts is MULTI_GROUPS and name == "sparse120":
        assert plan.info["n_multi_groups"] > 0, "case must exercise multi-member tables"
    if opts is GLOBAL_IMAGE:
        assert plan.info["image_in_lds"] == 0
    if name == "single64":
        # one pass of more than 60 slots: state bytes in LDS, not the 64-bit register form
        assert plan.info["n_passes"] == 1 and plan.info["n_kept"] > 60, plan.info
    if opts is CONE:
        # the cone reduction removes the detached modules, which Definition 1 keeps
        leaf = api.Plan(net_of(name), interest=sorted({a for tg in targets_of(net_of(name)) for a, _ in tg}),
                        **REDUCED)
        assert plan.info["n_kept"] < leaf.info["n_kept"]


@pytest.mark.parametrize("name,opts", [("c2", GROUPED), ("c3_slice", REDUCED), ("c1", PLAIN)])
def test_initial_state_matches_oracle(name, opts):
    net = net_of(name)
    plan = api.Plan(net, interest=[0, 1, 2], **opts)
    say(f"[gpu] init {name}")
    state = api.state_init(plan, 11, 50, traj0=1000)
    orig = api.unpack_bits(api.to_original(plan, state).cpu().numpy(), plan.n)
    ref = contract.initial_state(net, 11, np.arange(1000, 1050))
    kept = plan.node_pos() != NONE
    assert np.array_equal(orig[:, kept], ref[:, kept])


def test_chunked_launch_equals_single_launch():
    a = gpu_run("c2", GROUPED, 9, 0, 64, (1000,))
    b = gpu_run("c2", GROUPED, 9, 0, 64, (1, 2, 333, 664))
    assert np.array_equal(a[3], b[3])
    assert np.array_equal(a[2], b[2])


def test_trajectory_subset_is_exact():
    full = gpu_run("c2", GROUPED, 10, 0, 100, (500,))
    part = gpu_run("c2", GROUPED, 10, 40, 10, (500,))
    assert np.array_equal(full[3][40:50], part[3])


def test_plain_reduced_grouped_agree_on_kept_nodes():
    runs = [gpu_run("c2", o, 12, 0, 256, (2000,), plain=(o is not GROUPED)) for o in (PLAIN, REDUCED, GROUPED)]
    kept = runs[1][0].node_pos() != NONE
    for r in runs[1:]:
        assert np.array_equal(r[1][:, kept], runs[0][1][:, kept])
        assert np.array_equal(r[2], runs[0][2])


def test_full_size_c2_sampled_against_oracle():
    """C2 at its full trajectory count and launch shape; 8 sampled trajectories
    (spread over the id range) are recomputed by the oracle."""
    cfg = ps.config("C2")
    net = cfg.net
    plan = api.Plan(net, interest=[a for a, _ in cfg.targets[0]], **GROUPED)
    tg = plan.targets(cfg.targets)
    steps = 400
    say("[gpu] full-size C2 4096 trajectories")
    state = api.state_init(plan, cfg.seed, cfg.ntraj)
    counts = api.new_counts(1, cfg.ntraj)
    api.simulate(plan, cfg.seed, state, counts, tg, 0, steps)
    orig = api.unpack_bits(api.to_original(plan, state).cpu().numpy(), plan.n)
    c = counts.cpu().numpy()
    sample = np.array([0, 1, 777, 1500, 2048, 3000, 4000, 4095])
    ref = osim.run(net, cfg.seed, sample, steps, targets=cfg.targets)
    kept = plan.node_pos() != NONE
    assert np.array_equal(orig[sample][:, kept], ref["state"][:, kept])
    assert np.array_equal(c[0, sample, 0], ref["hits"][0])


def test_c1_estimate_matches_power_method():
    """C1: one trajectory of 10^6 steps; batch-means interval around the exact
    steady state of the 2^10-state chain (Eq. 1)."""
    cfg = ps.config("C1")
    net = cfg.net
    plan = api.Plan(net, interest=[0, 1], **GROUPED)
    tg = plan.targets(cfg.targets)
    state = api.state_init(plan, cfg.seed, 1)
    B = 50
    per = cfg.steps // B
    batch = []
    say("[gpu] C1 10^6 steps in 50 batches")
    for b in range(B):
        counts = api.new_counts(1, 1)
        api.simulate(plan, cfg.seed, state, counts, tg, b * per, per)
        batch.append(int(counts.cpu().numpy()[0, 0, 0]))
    pi = exact.steady_state(net)
    want = exact.target_probability(pi, cfg.targets[0])
    means = np.array(batch) / per
    p_hat = means.mean()
    hw = 3.29 * means.std(ddof=1) / math.sqrt(B)
    assert abs(p_hat - want) < hw, (p_hat, want, hw)


@pytest.mark.parametrize("name", ["c2", "sparse120"])
def test_autotune_candidates_are_bit_identical(name):
    """Every preparation the autotuner may pick simulates the same kept-node bits."""
    from paper_1605_00854_amd import autotune
    net = net_of(name)
    tgs = targets_of(net)
    interest = sorted({a for tg in tgs for a, _ in tg})
    ref = None
    for opts in autotune.candidates(quick=True):
        plan = api.Plan(net, interest=interest, **opts)
        say(f"[gpu] autotune candidate {name} {opts} slots={plan.info['n_slots']}")
        tg = plan.targets(tgs)
        state = api.state_init(plan, 21, 40)
        counts = api.new_counts(len(tgs), 40)
        api.simulate(plan, 21, state, counts, tg, 0, 500, plain=plan.info["n_table_slots"] == 0,
                     waves_per_block=2)
        orig = api.unpack_bits(api.to_original(plan, state).cpu().numpy(), plan.n)
        kept = plan.node_pos() != NONE
        c = counts.cpu().numpy()
        if ref is None:
            ref = (orig, kept, c)
        common = kept & ref[1]
        assert np.array_equal(orig[:, common], ref[0][:, common]), opts
        assert np.array_equal(c, ref[2]), opts


BITS = dict(reduce=1, group=0, state_bits=1)
BITS_GROUPED = dict(reduce=1, group=1, state_bits=1, lds_budget_bytes=150000)
BITS_TUNED = dict(reduce=1, group=1, state_bits=1, max_parent_bits=5, max_group_nodes=4, lds_budget_bytes=150000)
BITS_MULTI = dict(MULTI_GROUPS, state_bits=1)
BITS_GLOBAL = dict(reduce=1, group=1, state_bits=1, lds_budget_bytes=0)
BITS_PLAIN = dict(reduce=0, group=0, state_bits=1)

BITS_CASES = [
    # (network, plan, seed, traj0, ntraj, chunks, count_from, plain, wpb)
    ("c2", "BITS", 51, 0, 70, (150, 113), 40, True, 4),                 # FN passes only: ballot words
    ("c2", "BITS_GROUPED", 52, 5, 67, (263,), 0, False, 8),             # table passes: DPP-combined nibbles
    ("c2_hot", "BITS_GROUPED", 53, 0, 45, (120, 80), 30, False, 4),     # chains flip bits most steps
    ("multi400", "BITS_MULTI", 54, 0, 20, (60, 40), 10, False, 2),      # combined tables of several members
    ("c3_slice", "BITS_TUNED", 55, 0, 24, (90, 70), 20, False, 16),     # many passes, a mixed table/FN pass
    ("c3_slice", "BITS_GLOBAL", 56, 3, 11, (100,), 0, False, 4),        # image in global memory
    ("sparse120", "BITS_GROUPED", 57, 0, 33, (200,), 50, False, 4),
    ("wide40", "BITS", 58, 0, 29, (120, 33), 15, True, 4),              # predictors of up to 7 parents
    ("c1", "BITS_PLAIN", 59, 0, 9, (300,), 0, True, 4),
    ("modules", "BITS_GROUPED", 60, 0, 40, (160,), 20, False, 4),
]


@pytest.mark.parametrize("case", BITS_CASES, ids=lambda c: f"{c[0]}-{c[1]}")
def test_packed_bit_state_matches_the_oracle(case):
    """Plans built with the packed-bit state (parents read as bits, each pass's
    results written as whole words): every kept node and every counter equals
    the oracle's."""
    name, opts, seed, traj0, ntraj, chunks, count_from, plain, wpb = case
    plan = check(name, globals()[opts], seed, traj0, ntraj, chunks, count_from, plain, wpb)
    if opts in ("BITS_GROUPED", "BITS_TUNED", "BITS_MULTI") and name != "c2_hot":
        assert plan.info["n_table_slots"] > 0


@pytest.mark.parametrize("opts,seed,traj0,ntraj,chunks,count_from,plain,wpb",
                         [(CONE, 20, 0, 24, (300,), 0, True, 0), (CONE_GROUPED, 21, 3, 17, (150, 90), 40, False, 2)],
                         ids=["cone", "cone-grouped"])
def test_short_plans_with_many_draw_blocks_match_the_oracle(opts, seed, traj0, ntraj, chunks, count_from, plain, wpb):
    """Plans of one or two lane passes whose steps need more than 64 Philox
    calls (kept nodes spread over the rank order of a larger network) run in
    the streaming form: trajectories and counters equal the oracle's."""
    plan = check("interleaved", opts, seed, traj0, ntraj, chunks, count_from, plain, wpb)
    assert plan.info["n_passes"] <= 2 and plan.info["n_jobs"] > 64, plan.info


MULTI_CASES = [
    # (network, plan, trajectories per wave, seed, traj0, ntraj, chunks, count_from, plain, wpb)
    ("c2", "REDUCED", 2, 41, 0, 131, (150, 113), 40, True, 0),      # 170 virtual slots: 3 passes
    ("c2", "REDUCED", 3, 42, 7, 100, (263,), 0, True, 8),           # 255 of 256 lanes: 4 passes; ragged last wave
    ("c2", "PLAIN", 2, 43, 0, 64, (90, 90), 5, True, 2),            # 200 virtual slots
    ("c2_hot", "REDUCED", 2, 44, 0, 61, (120, 80), 30, True, 4),    # two perturbations per step on average
    ("c2_small", "PLAIN", 4, 45, 3, 50, (200,), 10, True, 4),       # 148 virtual slots in 3 passes
    ("c2_small", "REDUCED", 4, 46, 0, 7, (90, 90), 0, False, 8),    # 2 passes; fewer trajectories than one wave holds
    ("modules", "CONE", 4, 47, 0, 90, (160,), 20, True, 4),         # cone plan, 4 passes
    ("wide40", "REDUCED", 3, 48, 0, 45, (120, 33), 15, True, 4),    # predictors of up to 7 parents
]


@pytest.mark.parametrize("case", MULTI_CASES, ids=lambda c: f"{c[0]}-{c[1]}-k{c[2]}")
def test_several_trajectories_per_wave_match_the_oracle(case):
    """Several trajectories sharing a wavefront's lane passes: every kept node
    and every counter equals the oracle's, whatever the trajectory count, the
    chunking, the burn-in boundary and the perturbation rate."""
    name, opts, tpw, seed, traj0, ntraj, chunks, count_from, plain, wpb = case
    check(name, globals()[opts], seed, traj0, ntraj, chunks, count_from, plain, wpb, tpw)


def test_several_trajectories_per_wave_reject_unsupported_plans():
    net = net_of("c2")
    tgs = targets_of(net)
    interest = sorted({a for tg in tgs for a, _ in tg})
    plan = api.Plan(net, interest=interest, **GROUPED)
    tg = plan.targets(tgs)
    state = api.state_init(plan, 1, 8)
    counts = api.new_counts(len(tgs), 8)
    with pytest.raises(api._lib.PbnError, match="traj_per_wave"):
        api.simulate(plan, 1, state, counts, tg, 0, 10, traj_per_wave=2)          # table slots
    red = api.Plan(net, interest=interest, **REDUCED)
    state = api.state_init(red, 1, 8)
    with pytest.raises(api._lib.PbnError, match="traj_per_wave"):
        api.simulate(red, 1, state, counts, red.targets(tgs), 0, 10, traj_per_wave=4)   # 340 virtual slots


def test_full_size_c2_product_configuration():
    """C2's product configuration as timed by the benchmark (leaf reduction,
    group size 1, every trajectory, 2 and 8 waves per workgroup): 8 sampled
    trajectories against the oracle over 400 steps; then one 250 000-step
    launch, the benchmark's chunk, against the unreduced plain kernel run in
    two chunks with another launch shape -- the keyed draws make every kept
    node and counter identical at any depth."""
    cfg = ps.config("C2")
    net = cfg.net
    interest = [a for a, _ in cfg.targets[0]]
    red = api.Plan(net, interest=interest, **REDUCED)
    plain = api.Plan(net, interest=interest, **PLAIN)
    kept = red.node_pos() != NONE
    sample = np.array([0, 3, 511, 1024, 2047, 2600, 3333, 4095])
    ref = osim.run(net, cfg.seed, sample, 400, targets=cfg.targets)
    for wpb in (2, 8):
        say(f"[gpu] C2 product configuration, 400 steps, wpb={wpb}")
        tg = red.targets(cfg.targets)
        state = api.state_init(red, cfg.seed, cfg.ntraj)
        counts = api.new_counts(1, cfg.ntraj)
        api.simulate(red, cfg.seed, state, counts, tg, 0, 400, waves_per_block=wpb)
        orig = api.unpack_bits(api.to_original(red, state).cpu().numpy(), red.n)
        assert np.array_equal(orig[sample][:, kept], ref["state"][:, kept])
        assert np.array_equal(counts.cpu().numpy()[0, sample, 0], ref["hits"][0])
    deep = 250000
    runs = []
    for plan, chunks, wpb, use_plain in ((red, (deep,), 2, True), (plain, (deep // 2, deep - deep // 2), 8, True)):
        say(f"[gpu] C2 {deep} steps, chunks={chunks}, wpb={wpb}, n_kept={plan.info['n_kept']}")
        tg = plan.targets(cfg.targets)
        state = api.state_init(plan, cfg.seed, cfg.ntraj)
        counts = api.new_counts(1, cfg.ntraj)
        step = 0
        for c in chunks:
            api.simulate(plan, cfg.seed, state, counts, tg, step, c, count_from=1000, plain=use_plain,
                         waves_per_block=wpb)
            step += c
        runs.append((api.unpack_bits(api.to_original(plan, state).cpu().numpy(), plan.n), counts.cpu().numpy()))
    assert np.array_equal(runs[0][0][:, kept], runs[1][0][:, kept])
    assert np.array_equal(runs[0][1], runs[1][1])
    c = runs[0][1][0]
    assert np.all(c[:, 0] <= deep - 1000) and np.all(np.abs(c[:, 1].astype(np.int64) - c[:, 2]) <= 1)


def test_full_size_c3_product_configuration():
    """C3 at its full trajectory count with the autotuner's plan (grouping into
    at most 5 union bits and 4 nodes, 8 waves per workgroup): 64 trajectories
    spread over the 65 536 against the oracle, every kept node and all three
    counters -- over steps 0-249 counted from step 0, and over one 500-step
    launch from step 0 counted from step 250, so that the counters cross the
    burn-in boundary inside a launch; then 20 000 steps against the
    reduction-only plain kernel at another launch shape."""
    cfg = ps.config("C3")
    net = cfg.net
    interest = sorted({a for tg in cfg.targets for a, _ in tg})
    tuned = api.Plan(net, interest=interest, reduce=1, group=1, max_parent_bits=5, max_group_nodes=4)
    red = api.Plan(net, interest=interest, **REDUCED)
    assert tuned.info["n_table_slots"] > 0
    kept = tuned.node_pos() != NONE
    sample = np.linspace(0, cfg.ntraj - 1, 64).round().astype(np.int64)
    say("[gpu] C3 full size: oracle on 64 trajectories x 500 steps")
    nw = osim.Network(net)
    ref_a = osim.run(net, cfg.seed, sample, 250, targets=cfg.targets, nw=nw)
    ref_b = osim.run(net, cfg.seed, sample, 250, step0=250, count_from=250, targets=cfg.targets, nw=nw,
                     state=ref_a["state"])
    tg = tuned.targets(cfg.targets)
    for steps, count_from, ref in ((250, 0, ref_a), (500, 250, ref_b)):
        say(f"[gpu] C3 full size, {steps} steps in one launch, counted from step {count_from}")
        state = api.state_init(tuned, cfg.seed, cfg.ntraj)
        counts = api.new_counts(len(cfg.targets), cfg.ntraj)
        api.simulate(tuned, cfg.seed, state, counts, tg, 0, steps, count_from=count_from, waves_per_block=8)
        orig = api.unpack_bits(api.to_original(tuned, state).cpu().numpy(), tuned.n)
        c = counts.cpu().numpy()
        assert np.array_equal(orig[sample][:, kept], ref["state"][:, kept]), steps
        assert np.array_equal(c[:, sample, 0], ref["hits"]), steps
        assert np.array_equal(c[:, sample, 1], ref["n01"]), steps
        assert np.array_equal(c[:, sample, 2], ref["n10"]), steps
    assert ref_b["hits"].sum() > 0 and (ref_b["n01"].sum() + ref_b["n10"].sum()) > 0
    runs = []
    for plan, wpb, use_plain in ((tuned, 8, False), (red, 2, True)):
        say(f"[gpu] C3 20000 steps, n_slots={plan.info['n_slots']}, wpb={wpb}")
        tg = plan.targets(cfg.targets)
        state = api.state_init(plan, cfg.seed, cfg.ntraj)
        counts = api.new_counts(len(cfg.targets), cfg.ntraj)
        api.simulate(plan, cfg.seed, state, counts, tg, 0, 20000, count_from=10000, plain=use_plain,
                     waves_per_block=wpb)
        runs.append((api.unpack_bits(api.to_original(plan, state).cpu().numpy(), plan.n), counts.cpu().numpy()))
    assert np.array_equal(runs[0][0][:, kept], runs[1][0][:, kept])
    assert np.array_equal(runs[0][1], runs[1][1])
