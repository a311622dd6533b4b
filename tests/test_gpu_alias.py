"""GPU parity of the alias sampling mode (Algorithms 1, 2 and 5's per-group
draws; Sections 2.2, 3.2-3.4) through the C ABI.

* Bit-exact trajectories and counters against the oracle's reduced-network
  simulator under the same draw contract: unreduced and reduced networks,
  combined tables with several multi-predictor members, LDS- and
  global-resident images, two-unit FN records, plans of more than two lane
  passes, more than 64 Philox calls per step, chunked launches.
* The law: long-run target frequencies match the exact steady state (Eq. 1,
  power method) within statistical error, and agree with the keyed mode's
  estimates on a network too large for the exact chain.
"""
import functools
import sys

import numpy as np
import pytest

import pbn_synth as ps
from oracle import alias, exact

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1605_00854_amd import api  # noqa: E402

CAPS = dict(max_group_nodes=4, max_parent_bits=12, max_table_entries=4096)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def wide7(seed=12, n=70):
    rng = np.random.default_rng(seed)
    fns = []
    for _ in range(n):
        l = int(rng.integers(1, 4))
        probs = rng.dirichlet(np.ones(l))
        ks = [int(rng.integers(1, 8)) for _ in range(l)]
        fns.append([(probs[j], list(rng.choice(n, size=ks[j], replace=False)), rng.integers(0, 2, 1 << ks[j]))
                    for j in range(l)])
    return ps.assemble(n, 2e-3, fns)


NETS = {
    "c1": ps.tiny_c1,
    "c2": ps.medium_c2,
    "c2_hot": lambda: ps.medium_c2(n=100, p=0.02, seed=31),
    "multi400": lambda: ps.random_pbn(400, 2e-3, 12, nfn=lambda r: int(r.integers(2, 5)),
                                      nparents=lambda r: int(r.integers(1, 4))),
    "sparse120": lambda: ps.random_pbn(120, 3e-3, 14, nfn=lambda r: int(r.integers(1, 4)),
                                       nparents=lambda r: int(r.integers(0, 3)), leaf_frac=0.2),
    "wide7": wide7,
}


@functools.lru_cache(maxsize=None)
def net_of(name):
    return NETS[name]()


def targets_of(net):
    t1 = ps.non_leaf_targets(net, 3)
    t2 = [(t1[0][0], 0)]
    t3 = [(a, (a + 1) % 2) for a, _ in ps.non_leaf_targets(net, 2)]
    return [t1, t2, t3]


def interest_of(net):
    return sorted({a for tg in targets_of(net) for a, _ in tg})


def plan_opts(opts):
    return dict(CAPS, sampling=1, **opts)


def oracle_plan(net, opts):
    return alias.alias_plan(net, interest_of(net), reduce=opts.get("reduce", 1), group=opts.get("group", 1),
                            theta=opts.get("theta", 65536), weight_mode=opts.get("weight_mode", 1),
                            caps=(CAPS["max_group_nodes"], CAPS["max_parent_bits"], CAPS["max_table_entries"]))


PLAIN = dict(reduce=0, group=0)
REDUCED = dict(reduce=1, group=0)
GROUPED = dict(reduce=1, group=1)
MULTI_GROUPS = dict(reduce=1, group=1, weight_mode=0, theta=10 ** 6)
GLOBAL_IMAGE = dict(reduce=1, group=1, weight_mode=0, theta=10 ** 6, lds_budget_bytes=0)
PACKED = dict(reduce=1, group=0, lds_budget_bytes=0)   # packed image: per-slot FN record units

CASES = [
    # name, opts, seed, traj0, ntraj, chunks, count_from, plain, wpb
    ("c1", PLAIN, 1, 0, 5, (2000,), 0, True, 0),
    ("c1", MULTI_GROUPS, 1, 0, 5, (1200, 800), 300, False, 0),
    ("c2", REDUCED, 2, 0, 24, (300,), 0, True, 0),
    ("c2", MULTI_GROUPS, 2, 0, 24, (300,), 0, False, 0),
    ("c2", GLOBAL_IMAGE, 2, 3, 19, (150, 150), 40, False, 3),
    ("c2_hot", GROUPED, 3, 5, 16, (120, 80), 50, False, 2),
    ("multi400", GROUPED, 5, 0, 6, (60,), 0, False, 1),
    ("sparse120", MULTI_GROUPS, 7, 0, 12, (150,), 0, False, 0),
    ("wide7", REDUCED, 9, 0, 10, (200,), 0, True, 0),
    ("wide7", PACKED, 9, 2, 10, (120, 80), 20, True, 0),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{i}" for i, c in enumerate(CASES)])
def test_alias_trajectories_bit_exact(case):
    name, opts, seed, traj0, ntraj, chunks, count_from, plain, wpb = case
    net = net_of(name)
    tgs = targets_of(net)
    plan = api.Plan(net, interest=interest_of(net), **plan_opts(opts))
    ref_plan = oracle_plan(net, opts)
    say(f"[gpu] alias {name} opts={opts} info={plan.info} traj={traj0}+{ntraj} chunks={chunks} plain={plain}")
    tg = plan.targets(tgs)
    state = api.state_init(plan, seed, ntraj, traj0=traj0)
    counts = api.new_counts(len(tgs), ntraj)
    step = 0
    for c in chunks:
        api.simulate(plan, seed, state, counts, tg, step, c, traj0=traj0, count_from=count_from, plain=plain,
                     waves_per_block=wpb)
        step += c
    orig = api.unpack_bits(api.to_original(plan, state).cpu().numpy(), plan.n)
    counts = counts.cpu().numpy()
    say(f"[oracle] alias {name} steps={step}")
    ref = alias.simulate(net, ref_plan, seed, np.arange(traj0, traj0 + ntraj), step, targets=tgs,
                         count_from=count_from)
    kept = ref_plan["kept"]
    assert plan.info["n_kept"] == len(kept)
    bad = np.nonzero((orig[:, kept] != ref["state"][:, kept]).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} trajectories differ, first {traj0 + bad[0]}"
    assert np.array_equal(counts[:, :, 0], ref["hits"])
    assert np.array_equal(counts[:, :, 1], ref["n01"])
    assert np.array_equal(counts[:, :, 2], ref["n10"])
    assert ref["perturbed"].sum() > 0
    if opts is MULTI_GROUPS and name in ("c2", "sparse120"):
        assert any(len(g) > 1 for g in ref_plan["groups"]), "case must draw combined functions"
    if name == "multi400":
        assert plan.info["n_jobs"] > 64 and plan.info["n_passes"] > 2
    if opts is GLOBAL_IMAGE or opts is PACKED:
        assert plan.info["image_in_lds"] == 0
    if name == "wide7":
        assert plan.info["max_fn_parents"] > 5


def _long_run(net, opts, seed, ntraj, burn, steps, targets):
    plan = api.Plan(net, interest=sorted({a for tg in targets for a, _ in tg}), **opts)
    tg = plan.targets(targets)
    state = api.state_init(plan, seed, ntraj)
    counts = api.new_counts(len(targets), ntraj)
    api.simulate(plan, seed, state, counts, tg, 0, burn + steps, count_from=burn)
    torch.cuda.synchronize()
    hits = counts.cpu().numpy()[:, :, 0].astype(float) / steps      # (targets, ntraj)
    return hits.mean(axis=1), hits.std(axis=1, ddof=1) / np.sqrt(ntraj)


@pytest.mark.parametrize("opts", [PLAIN, MULTI_GROUPS])
def test_alias_steady_state_matches_exact_chain(opts):
    net = ps.random_pbn(9, 0.03, 51, nfn=lambda r: int(r.integers(1, 4)), nparents=lambda r: int(r.integers(1, 4)),
                        leaf_frac=0.25)
    targets = targets_of(net)
    pi = exact.steady_state(net)
    want = np.array([exact.target_probability(pi, tg) for tg in targets])
    say(f"[gpu] alias steady state opts={opts}")
    mean, se = _long_run(net, plan_opts(opts), 21, 4096, 2000, 20000, targets)
    assert np.all(np.abs(mean - want) < 5 * se + 1e-4), (mean, want, se)


def test_alias_and_keyed_modes_estimate_the_same_steady_state():
    net = net_of("c2_hot")
    targets = targets_of(net)
    say("[gpu] alias vs keyed on c2_hot")
    m_alias, se_a = _long_run(net, plan_opts(GROUPED), 23, 4096, 2000, 20000, targets)
    m_keyed, se_k = _long_run(net, dict(GROUPED), 24, 4096, 2000, 20000, targets)
    assert np.all(np.abs(m_alias - m_keyed) < 5 * np.hypot(se_a, se_k) + 1e-4), (m_alias, m_keyed)


def test_rl_driver_under_alias_sampling():
    # the two-state driver runs an alias-sampling plan unchanged: its recorded
    # indicator sequence is the alias oracle's trajectory and its estimate is
    # within the requested precision of the exact steady state
    from oracle import stats as ost
    cfg = ps.config("C1")
    net = cfg.net
    plan = api.Plan(net, interest=[0, 1], reduce=0, group=1, weight_mode=0, theta=10 ** 6, sampling=1)
    ref_plan = alias.alias_plan(net, [0, 1], reduce=0, group=1, theta=10 ** 6, weight_mode=0,
                                caps=(CAPS["max_group_nodes"], CAPS["max_parent_bits"], CAPS["max_table_entries"]))
    r = 0.01
    say("[gpu] rl_run C1 alias r=0.01")
    res, record = api.rl_run(plan, cfg.seed, cfg.targets, r, initial_steps=20000, max_steps=1 << 22)
    assert res["status"] == 0, res
    n = res["steps"]
    bits = api.unpack_record(record.cpu().numpy(), n)
    pre = min(n, 3000)
    z = np.zeros(pre, dtype=np.uint8)
    s = None
    for t in range(pre):       # the oracle, one step at a time, reading the target after each step
        out = alias.simulate(net, ref_plan, cfg.seed, np.arange(1), 1, step0=t, state=s)
        s = out["reduced"]
        z[t] = all(out["state"][0, a] == v for a, v in cfg.targets[0])
    assert np.array_equal(bits[:pre], z)
    want = ost.rl92_diagnose(bits, r, conf=0.95, eps=1e-3, kmax=100)
    assert res["k"] == want["k"]
    assert res["p_hat"] == pytest.approx(want["p_hat"], rel=1e-9)
    pi = exact.target_probability(exact.steady_state(net), cfg.targets[0])
    assert abs(res["p_hat"] - pi) < r * 3.29 / 1.96, (res, pi)


def test_alias_single_kept_node_and_many_leaves():
    # edge case: the cone of the node of interest is that node alone (it reads
    # only itself), so Algorithm 2 has one group of one node (g = k = k' = 1)
    # and every other node is a removed leaf (Algorithm 1's t = (1-p)^(n-1))
    n, p = 12, 0.02
    fns = [[(0.6, [0], np.array([1, 0])), (0.4, [0], np.array([0, 1]))]]           # node 0: not / copy of itself
    for i in range(1, n):
        fns.append([(1.0, [0, (i + 1) % n], np.array([0, 1, 1, 0]))])
    net = ps.assemble(n, p, fns)
    tgs = [[(0, 1)]]
    plan = api.Plan(net, interest=[0], **plan_opts(dict(reduce=2, group=0)))
    ref_plan = alias.alias_plan(net, [0], reduce=2, group=0)
    assert plan.info["n_kept"] == 1 and (ref_plan["g"], ref_plan["k"], ref_plan["kp"]) == (1, 1, 1)
    ntraj, steps, seed = 7, 3000, 31
    say("[gpu] alias single kept node")
    tg = plan.targets(tgs)
    state = api.state_init(plan, seed, ntraj)
    counts = api.new_counts(1, ntraj)
    api.simulate(plan, seed, state, counts, tg, 0, steps)
    orig = api.unpack_bits(api.to_original(plan, state).cpu().numpy(), plan.n)
    ref = alias.simulate(net, ref_plan, seed, np.arange(ntraj), steps, targets=tgs)
    assert np.array_equal(orig[:, 0], ref["state"][:, 0])
    assert np.array_equal(counts.cpu().numpy()[0, :, 0], ref["hits"][0])
    assert ref["perturbed"].sum() > 0


def test_alias_full_size_c2_sampled_against_oracle():
    # the benchmark's alias leg at full size: all 4096 trajectories of C2 on the
    # leaf-reduction plan at 8 waves per workgroup; 6 sampled trajectories
    # recomputed by the alias oracle over 300 steps
    cfg = ps.config("C2")
    net = cfg.net
    interest = [a for a, _ in cfg.targets[0]]
    plan = api.Plan(net, interest=interest, reduce=1, group=0, sampling=1)
    ref_plan = alias.alias_plan(net, interest, reduce=1, group=0)
    sample = np.array([0, 5, 1023, 2048, 3071, 4095])
    say("[gpu] alias C2 full size")
    tg = plan.targets(cfg.targets)
    state = api.state_init(plan, cfg.seed, cfg.ntraj)
    counts = api.new_counts(1, cfg.ntraj)
    api.simulate(plan, cfg.seed, state, counts, tg, 0, 300, waves_per_block=8)
    orig = api.unpack_bits(api.to_original(plan, state).cpu().numpy(), plan.n)
    ref = alias.simulate(net, ref_plan, cfg.seed, sample, 300, targets=cfg.targets)
    kept = ref_plan["kept"]
    assert np.array_equal(orig[sample][:, kept], ref["state"][:, kept])
    assert np.array_equal(counts.cpu().numpy()[0, sample, 0], ref["hits"][0])
