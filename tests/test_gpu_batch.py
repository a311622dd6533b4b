"""Batched persistent launch over networks of uneven size (C4 pattern):
per-network results must match the per-network oracle and single-network
launches bit for bit, also when the launches are captured in a HIP graph and
replayed."""
import sys

import numpy as np
import pytest

import pbn_synth as ps
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


def make_items(count, seed, nmin, nmax, ntraj, grouped):
    rng = np.random.default_rng(seed)
    items, nets = [], []
    for k in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        p = float(rng.choice([1e-3, 1e-2]))
        net = ps.medium_c2(n=n, p=p, seed=seed * 100 + k)
        tgs = [ps.non_leaf_targets(net, 2), [(ps.non_leaf_targets(net, 1)[0][0], 0)]]
        interest = sorted({a for tg in tgs for a, _ in tg})
        opts = dict(reduce=1, group=1, max_parent_bits=6) if grouped and k % 2 else dict(reduce=1, group=0)
        plan = api.Plan(net, interest=interest, **opts)
        items.append((plan, 1000 + k, ntraj[k % len(ntraj)], tgs))
        nets.append(net)
    return items, nets


@pytest.mark.parametrize("grouped", [False, True])
def test_batch_matches_oracle_per_network(grouped):
    items, nets = make_items(10, 3 + grouped, 20, 260, [5, 9, 4], grouped)
    say(f"[gpu] batch of {len(items)} networks grouped={grouped}")
    b = api.Batch(items, count_from=30, waves_per_block=4)
    b.init_states()
    b.set_window(0, 150)
    b.launch()
    b.set_window(150, 90)           # a second window continues the same trajectories
    b.launch()
    torch.cuda.synchronize()
    for k, ((plan, seed, ntraj, tgs), net) in enumerate(zip(items, nets)):
        ref = osim.run(net, seed, np.arange(ntraj), 240, targets=tgs, count_from=30)
        orig = api.unpack_bits(api.to_original(plan, b.states[k]).cpu().numpy(), plan.n)
        kept = plan.node_pos() != NONE
        assert np.array_equal(orig[:, kept], ref["state"][:, kept]), f"network {k}"
        c = b.counts[k].cpu().numpy()
        assert np.array_equal(c[:, :, 0], ref["hits"]), f"network {k}"
        assert np.array_equal(c[:, :, 1], ref["n01"]), f"network {k}"
        assert np.array_equal(c[:, :, 2], ref["n10"]), f"network {k}"


def single_launch_states(items, steps):
    out = []
    for plan, seed, ntraj, tgs in items:
        tg = plan.targets(tgs)
        st = api.state_init(plan, seed, ntraj)
        cn = api.new_counts(tg.ntargets, ntraj)
        api.simulate(plan, seed, st, cn, tg, 0, steps, plain=plan.info["n_table_slots"] == 0)
        out.append((st.cpu().numpy(), cn.cpu().numpy()))
    return out


@pytest.mark.parametrize("wpt", [1, 2])
def test_batch_graph_replays_match_eager_launches(wpt):
    """Graph replays (two captured passes of 100 steps each) give the states
    and counters of single-network launches, with one or two waves per
    trajectory; eager work runs between the replays."""
    items, _ = make_items(24, 7, 20, 700, [16, 7, 33], True)
    ref_a = single_launch_states(items, 200)
    ref_b = single_launch_states(items, 400)
    b = api.Batch(items, waves_per_block=4, waves_per_traj=wpt)
    b.init_states()
    b.set_window(0, 100)
    say(f"[gpu] capture batch graph (2 passes x 100 steps, {wpt} waves per trajectory)")
    g = b.graph(2)
    torch.cuda.synchronize()
    for replay, ref in ((0, ref_a), (1, ref_b)):
        say(f"[gpu] graph replay {replay}")
        g.launch()
        torch.cuda.synchronize()
        # eager work between replays
        junk = torch.arange(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert int(junk) == 499500
        for k in range(len(items)):
            assert np.array_equal(b.states[k].cpu().numpy(), ref[k][0]), f"replay {replay} network {k}"
            assert np.array_equal(b.counts[k].cpu().numpy(), ref[k][1]), f"replay {replay} network {k}"
    assert b.step0() == 400


def test_batch_large_uneven_sampled():
    """Uneven sizes up to 1500 nodes (the batched workload's range); two networks
    are recomputed by the oracle on a trajectory subset."""
    items, nets = make_items(40, 11, 20, 1500, [64, 40], False)
    b = api.Batch(items, waves_per_block=4)
    b.init_states()
    b.set_window(0, 60)
    say("[gpu] batch of 40 networks up to 1500 nodes")
    b.launch()
    torch.cuda.synchronize()
    for k in (0, int(np.argmax([it[0].n for it in items]))):
        plan, seed, ntraj, tgs = items[k]
        sample = np.array([0, ntraj // 2, ntraj - 1])
        ref = osim.run(nets[k], seed, sample, 60, targets=tgs)
        orig = api.unpack_bits(api.to_original(plan, b.states[k]).cpu().numpy(), plan.n)
        kept = plan.node_pos() != NONE
        assert np.array_equal(orig[sample][:, kept], ref["state"][:, kept])


def test_full_size_c4_batch_configuration():
    """The batched workload at full size in the benchmark's configuration: 512
    networks (n ~ U[20, 1500]) x 256 trajectories, leaf-reduction plans, 4
    waves per workgroup, 10^4 burn-in + 10^5 counted steps in one persistent
    pass captured in a HIP graph.  Sampled networks match single-network
    launches of the same plans over the same steps (states and every counter);
    a 20-step batch of all 512 networks matches the oracle on sampled
    trajectories."""
    nets = ps.batch_c4()
    ntraj, burn, total = 256, 10**4, 11 * 10**4

    def items_for():
        out = []
        for k, net in enumerate(nets):
            tg = [ps.non_leaf_targets(net, 3)]
            plan = api.Plan(net, interest=[a for a, _ in tg[0]], reduce=1, group=0)
            out.append((plan, 1004000 + k, ntraj, tg))
        return out

    items = items_for()
    sizes = np.array([net["n"] for net in nets])
    picks = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 7, 200, 511})
    say("[gpu] C4 full size: 512 networks x 256 trajectories x 110000 steps, one graph pass")
    b = api.Batch(items, count_from=burn, waves_per_block=4)
    b.init_states()
    b.set_window(0, total)
    g = b.graph(1)
    g.launch()
    torch.cuda.synchronize()
    for k in picks:
        plan, seed, nt, tg = items[k]
        say(f"[gpu] C4 network {k} (n={plan.n}) against a single-network launch")
        state = api.state_init(plan, seed, nt)
        counts = api.new_counts(1, nt)
        api.simulate(plan, seed, state, counts, plan.targets(tg), 0, total, count_from=burn, plain=True)
        assert np.array_equal(b.states[k].cpu().numpy(), state.cpu().numpy()), k
        assert np.array_equal(b.counts[k].cpu().numpy(), counts.cpu().numpy()), k
    del g, b
    say("[gpu] C4 full size: 20 steps against the oracle on sampled trajectories")
    b = api.Batch(items, count_from=0, waves_per_block=4)
    b.init_states()
    b.set_window(0, 20)
    b.launch()
    torch.cuda.synchronize()
    sample = np.array([0, 101, 255])
    for k in picks[:3]:
        plan, seed, nt, tg = items[k]
        ref = osim.run(nets[k], seed, sample, 20, targets=tg)
        orig = api.unpack_bits(api.to_original(plan, b.states[k]).cpu().numpy(), plan.n)
        kept = plan.node_pos() != NONE
        assert np.array_equal(orig[sample][:, kept], ref["state"][:, kept]), k
        assert np.array_equal(b.counts[k].cpu().numpy()[:, sample, 0], ref["hits"]), k


def test_full_size_c4_against_the_oracle_over_1000_steps():
    """C4's 512 networks x 256 trajectories in one persistent launch of 1000
    steps counted from step 500; 4 trajectories of the smallest, the largest
    and three more networks against the oracle: every kept node and all three
    counters.  The oracle runs in worker processes (no GPU use) while the GPU
    runs the batch."""
    import multiprocessing as mp

    import oracle_jobs
    nets = ps.batch_c4()
    ntraj, steps, count_from = 256, 1000, 500
    items = []
    for k, net in enumerate(nets):
        tg = [ps.non_leaf_targets(net, 3)]
        plan = api.Plan(net, interest=[a for a, _ in tg[0]], reduce=1, group=0)
        items.append((plan, 1004000 + k, ntraj, tg))
    sizes = np.array([net["n"] for net in nets])
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 200, 511})
    sample = [0, 85, 170, 255]
    jobs = [(k, items[k][1], sample, steps, count_from, items[k][3]) for k in picks]
    say(f"[gpu] C4 full size, 1000 steps; oracle on networks {picks} (n = {sizes[picks].tolist()})")
    with mp.get_context("spawn").Pool(len(jobs)) as pool:
        pending = pool.map_async(oracle_jobs.c4_network_run, jobs)
        b = api.Batch(items, count_from=count_from, waves_per_block=4)
        b.init_states()
        b.set_window(0, steps)
        b.launch()
        torch.cuda.synchronize()
        refs = pending.get(timeout=600)
    for k, ref in zip(picks, refs):
        plan = items[k][0]
        orig = api.unpack_bits(api.to_original(plan, b.states[k]).cpu().numpy(), plan.n)
        kept = plan.node_pos() != NONE
        c = b.counts[k].cpu().numpy()
        assert np.array_equal(orig[sample][:, kept], ref["state"][:, kept]), k
        assert np.array_equal(c[:, sample, 0], ref["hits"]), k
        assert np.array_equal(c[:, sample, 1], ref["n01"]), k
        assert np.array_equal(c[:, sample, 2], ref["n10"]), k


def test_batch_mixes_wide_and_narrow_predictor_records():
    """Networks whose predictors read up to 7 parents (packed images where only
    the slots reading 6-7 parents have two-unit records) batched with networks
    of one-unit records: every network matches the oracle."""
    items, nets = [], []
    for k in range(8):
        wide = k % 2 == 0
        n = 60 + 37 * k
        if wide:
            net = ps.random_pbn(n, 1e-2, 900 + k, nfn=lambda r: int(r.integers(1, 4)),
                                nparents=lambda r: int(r.integers(1, 8)), leaf_frac=0.1)
        else:
            net = ps.medium_c2(n=n, p=1e-2, seed=950 + k)
        tgs = [ps.non_leaf_targets(net, 2)]
        plan = api.Plan(net, interest=[a for a, _ in tgs[0]], reduce=1, group=k % 4 == 0,
                        lds_budget_bytes=0 if wide else 65536)
        if wide:
            assert plan.info["max_fn_parents"] > 5
        items.append((plan, 2000 + k, 5 + k, tgs))
        nets.append(net)
    say("[gpu] batch of wide and narrow predictor records")
    b = api.Batch(items, count_from=10, waves_per_block=4)
    b.init_states()
    b.set_window(0, 120)
    b.launch()
    torch.cuda.synchronize()
    for k, ((plan, seed, ntraj, tgs), net) in enumerate(zip(items, nets)):
        ref = osim.run(net, seed, np.arange(ntraj), 120, targets=tgs, count_from=10)
        orig = api.unpack_bits(api.to_original(plan, b.states[k]).cpu().numpy(), plan.n)
        kept = plan.node_pos() != NONE
        assert np.array_equal(orig[:, kept], ref["state"][:, kept]), f"network {k}"
        assert np.array_equal(b.counts[k].cpu().numpy()[:, :, 0], ref["hits"]), f"network {k}"


def test_batch_launch_shape_probe_leaves_results_unchanged():
    """The batch autotuner times the batch itself for each workgroup size; a
    batch run with whichever size it picks gives the same states and
    counters as one with the default."""
    from paper_1605_00854_amd import autotune
    items, _ = make_items(12, 21, 20, 400, [64, 33], False)
    say("[gpu] batch launch-shape probe")
    wpb, trials = autotune.batch_waves_per_block(items, count_from=20, wpbs=(2, 4, 8), probe_steps=100)
    assert wpb in (2, 4, 8) and [t["wpb"] for t in trials] == [2, 4, 8]
    assert all(t["seconds"] > 0 for t in trials)
    runs = []
    for w in (4, wpb):
        b = api.Batch(items, count_from=20, waves_per_block=w)
        b.init_states()
        b.set_window(0, 150)
        b.launch()
        torch.cuda.synchronize()
        runs.append(([s.cpu().numpy() for s in b.states], [c.cpu().numpy() for c in b.counts]))
    for k in range(len(items)):
        assert np.array_equal(runs[0][0][k], runs[1][0][k]) and np.array_equal(runs[0][1][k], runs[1][1][k]), k


def test_task_queues_leave_results_unchanged():
    """Networks dealt to one, three, eight, 32 or 64 task queues (workgroups
    steal from other queues once their own is empty, and most of the 64
    queues hold no network): which workgroup runs a trajectory changes nothing
    in its states or counters, also over a second window and for an
    oracle-checked network."""
    items, nets = make_items(13, 23, 20, 600, [64, 9, 130], True)
    say("[gpu] batch task queues 1 / 3 / 8 / 32 / 64")
    runs = []
    for nq in (1, 3, 8, 32, api.BATCH_QUEUES):
        b = api.Batch(items, count_from=20, waves_per_block=4, queues=nq)
        assert b.queue_first[-1] == b.ntasks
        b.init_states()
        b.set_window(0, 90)
        b.launch()
        b.set_window(90, 60)
        b.launch()
        torch.cuda.synchronize()
        runs.append(([s.cpu().numpy() for s in b.states], [c.cpu().numpy() for c in b.counts], b))
    for r in runs[1:]:
        for k in range(len(items)):
            assert np.array_equal(runs[0][0][k], r[0][k]) and np.array_equal(runs[0][1][k], r[1][k]), k
    plan, seed, ntraj, tgs = items[2]
    ref = osim.run(nets[2], seed, np.arange(ntraj), 150, targets=tgs, count_from=20)
    orig = api.unpack_bits(api.to_original(plan, runs[-1][2].states[2]).cpu().numpy(), plan.n)
    kept = plan.node_pos() != NONE
    assert np.array_equal(orig[:, kept], ref["state"][:, kept])
    c = runs[-1][1][2]
    assert np.array_equal(c[:, :, 0], ref["hits"]) and np.array_equal(c[:, :, 1], ref["n01"])
    assert np.array_equal(c[:, :, 2], ref["n10"])


def test_waves_per_trajectory_leave_results_unchanged():
    """Two, three or four waves advancing each trajectory together (shared
    state and draws in LDS, the lane passes split between them, one barrier
    per step) give the states and counters of one wave per trajectory: plans
    of one to 24 passes, with and without table slots, one with more than 64
    Philox jobs per step (single-step fills split between the waves), and a
    perturbation-heavy one (most steps walk the chain); two windows, and an
    oracle check of the largest network."""
    items, nets = make_items(6, 29, 20, 400, [7, 3], True)
    big = ps.medium_c2(n=1500, p=1e-3, seed=2931)
    hot = ps.medium_c2(n=300, p=1e-2, seed=2932)
    for k, net in enumerate((big, hot)):
        tgs = [ps.non_leaf_targets(net, 2)]
        plan = api.Plan(net, interest=[a for a, _ in tgs[0]], reduce=1, group=k)
        items.append((plan, 4000 + k, 5, tgs))
        nets.append(net)
    assert max(it[0].info["n_jobs"] for it in items) > 64
    assert max(it[0].info["n_passes"] for it in items) >= 20
    say("[gpu] batch waves per trajectory 1 / 2 / 3 / 4")
    runs = []
    for wpt in (1, 2, 3, 4):
        b = api.Batch(items, count_from=15, waves_per_block=4, waves_per_traj=wpt)
        b.init_states()
        b.set_window(0, 70)
        b.launch()
        b.set_window(70, 50)
        b.launch()
        torch.cuda.synchronize()
        runs.append(([s.cpu().numpy() for s in b.states], [c.cpu().numpy() for c in b.counts], b))
    for wpt, r in zip((2, 3, 4), runs[1:]):
        for k in range(len(items)):
            assert np.array_equal(runs[0][0][k], r[0][k]), (wpt, k)
            assert np.array_equal(runs[0][1][k], r[1][k]), (wpt, k)
    k = len(items) - 2
    plan, seed, ntraj, tgs = items[k]
    ref = osim.run(nets[k], seed, np.arange(ntraj), 120, targets=tgs, count_from=15)
    orig = api.unpack_bits(api.to_original(plan, runs[-1][2].states[k]).cpu().numpy(), plan.n)
    kept = plan.node_pos() != NONE
    assert np.array_equal(orig[:, kept], ref["state"][:, kept])
    c = runs[-1][1][k]
    assert np.array_equal(c[:, :, 0], ref["hits"]) and np.array_equal(c[:, :, 1], ref["n01"])
    assert np.array_equal(c[:, :, 2], ref["n10"])


def test_waves_per_trajectory_with_a_three_level_chain_search():
    """A network of more than 4096 nodes: the chain's search runs three
    radix-64 levels (the top one from registers, the others from the LDS copy
    of Q), with about five flips per step at p = 1e-3; four waves per
    trajectory give the one-wave results, and the oracle's."""
    net = ps.medium_c2(n=5000, p=1e-3, seed=2941)
    tgs = [ps.non_leaf_targets(net, 2)]
    plan = api.Plan(net, interest=[a for a, _ in tgs[0]], reduce=1, group=0)
    items = [(plan, 4100, 3, tgs)]
    say("[gpu] batch waves per trajectory, n = 5000")
    runs = []
    for wpt in (1, 4):
        b = api.Batch(items, count_from=5, waves_per_block=4, waves_per_traj=wpt)
        b.init_states()
        b.set_window(0, 40)
        b.launch()
        torch.cuda.synchronize()
        runs.append((b.states[0].cpu().numpy(), b.counts[0].cpu().numpy(), b))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    ref = osim.run(net, 4100, np.arange(3), 40, targets=tgs, count_from=5)
    orig = api.unpack_bits(api.to_original(plan, runs[1][2].states[0]).cpu().numpy(), plan.n)
    kept = plan.node_pos() != NONE
    assert np.array_equal(orig[:, kept], ref["state"][:, kept])
    assert np.array_equal(runs[1][1][:, :, 0], ref["hits"])


def test_waves_per_trajectory_fall_back_when_the_chain_tables_do_not_fit():
    """A 13 000-node network: its chain tables (12 bytes a node) do not fit in
    LDS beside its states and ring, so a launch asked for four waves per
    trajectory runs one; the results equal those of one wave."""
    net = ps.medium_c2(n=13000, p=1e-4, seed=2951)
    tgs = [ps.non_leaf_targets(net, 2)]
    plan = api.Plan(net, interest=[a for a, _ in tgs[0]], reduce=1, group=0)
    say("[gpu] batch waves per trajectory, n = 13000 (chain tables beyond LDS)")
    runs = []
    for wpt in (1, 4):
        b = api.Batch([(plan, 4200, 2, tgs)], count_from=3, waves_per_block=1, waves_per_traj=wpt)
        b.init_states()
        b.set_window(0, 30)
        b.launch()
        torch.cuda.synchronize()
        runs.append((b.states[0].cpu().numpy(), b.counts[0].cpu().numpy()))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
