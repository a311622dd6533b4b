"""Host side of the alias sampling mode (Algorithms 1, 2, 5; Sections 2.2,
3.2-3.4): the plan blob's tables are the oracle's, bit for bit.

* header: Algorithm 2's g, k, k' for the kept nodes, Algorithm 1's leaf
  threshold, the number of draw words;
* the 2^k pattern table (thresholds and aliases) and the kept-node positions;
* one alias record per selecting slot, numbered by smallest member id, with
  the table of the slot's combined indices, wired into the slot record.
"""
import numpy as np
import pytest

import pbn_synth as ps
from oracle import alias
from paper_1605_00854_amd import api

FIELDS = ("magic version blob_bytes plan_id n n_kept n_slots n_passes state_dwords state_words n_jobs "
          "fill_steps image_bytes image_off q_off o2p_off p2o_off blk_off pass_off zero_pos max_pmax "
          "image_in_lds has_table dummy_fn n_table fn_base fn_units fn_jshift fn_hoff sampling q_img o2p_img "
          "pert_off kpos_off alias_k alias_g alias_kp leaf_thr n_sel fn_var").split()

CAPS = dict(max_group_nodes=4, max_parent_bits=12, max_table_entries=4096)


def header(blob):
    words = np.frombuffer(blob[:4 * len(FIELDS)].tobytes(), dtype="<u4")
    return dict(zip(FIELDS, (int(w) for w in words)))


def u32(blob, off, count):
    return np.frombuffer(blob[off:off + 4 * count].tobytes(), dtype="<u4").astype(np.int64)


def nets():
    return {
        "c2": ps.medium_c2(n=100, p=1e-3, seed=1002),
        "multi60": ps.random_pbn(60, 5e-3, 41, nfn=lambda r: int(r.integers(1, 5)),
                                 nparents=lambda r: int(r.integers(1, 5)), leaf_frac=0.2),
        "tiny": ps.random_pbn(9, 0.02, 42, nfn=lambda r: int(r.integers(1, 4)),
                              nparents=lambda r: int(r.integers(1, 4)), leaf_frac=0.25),
        "single_fn": ps.random_pbn(20, 1e-3, 43, nfn=lambda r: 1, nparents=lambda r: 2),
    }


NETS = nets()
OPTS = [dict(reduce=0, group=0), dict(reduce=1, group=0), dict(reduce=1, group=1),
        dict(reduce=1, group=1, weight_mode=0, theta=10 ** 6), dict(reduce=2, group=1, lds_budget_bytes=0)]


def expected_fill(njobs, npass):
    """Steps per Philox fill: most lanes used over at most 4 rounds of 64 calls
    (1 round for plans of more than two lane passes), ties to more steps."""
    if njobs > 64:
        return 1
    rounds = 4 if npass <= 2 else 1
    best, best_use = 1, 0.0
    for f in range(1, 33):
        if f * njobs > 64 * rounds:
            break
        use = f * njobs / (64 * -(-(f * njobs) // 64))
        if use >= best_use - 1e-12:
            best, best_use = f, use
    return best


def interest_of(net):
    leaves = set(int(x) for x in net["designated_leaves"])
    return [v for v in range(int(net["n"])) if v not in leaves][:3]


def oracle_plan(net, opts):
    return alias.alias_plan(net, interest_of(net), reduce=opts.get("reduce", 1), group=opts.get("group", 1),
                            theta=opts.get("theta", 65536), weight_mode=opts.get("weight_mode", 1),
                            caps=(CAPS["max_group_nodes"], CAPS["max_parent_bits"], CAPS["max_table_entries"]))


@pytest.mark.parametrize("oi", range(len(OPTS)))
@pytest.mark.parametrize("name", sorted(NETS))
def test_alias_tables_match_oracle(name, oi):
    net, opts = NETS[name], OPTS[oi]
    plan = api.Plan(net, interest=interest_of(net), sampling=1, **opts)
    ref = oracle_plan(net, opts)
    blob = plan.blob()
    h = header(blob)
    assert h["sampling"] == 1
    assert h["n_kept"] == len(ref["kept"])
    assert (h["alias_g"], h["alias_k"], h["alias_kp"]) == (ref["g"], ref["k"], ref["kp"])
    assert h["leaf_thr"] == ref["leaf_thr"]
    assert h["n_sel"] == len(ref["groups"])
    assert h["n_jobs"] == ref["n_jobs"] == plan.info["n_jobs"]
    assert h["fill_steps"] == expected_fill(h["n_jobs"], h["n_passes"])
    assert plan.fill_steps == h["fill_steps"]
    # pattern table: 2^k entries {threshold, alias}
    L = 1 << h["alias_k"]
    tab = u32(blob, h["pert_off"], 2 * L).reshape(L, 2)
    assert tab[:, 0].tolist() == ref["pattern"][0]
    assert tab[:, 1].tolist() == ref["pattern"][1]
    pos = plan.node_pos()
    assert u32(blob, h["kpos_off"], h["n_kept"]).tolist() == [int(pos[v]) for v in ref["kept"]]
    # selecting slots: slot record z -> {draw offset, L, s, 0} + table
    img = h["image_off"]
    slot, _ = plan.slots()
    seen = set()
    for s_idx, members in enumerate(ref["groups"]):
        slots = {int(slot[v]) for v in members}
        assert len(slots) == 1, "a selecting group is one slot"
        (sl,) = slots
        z = int(u32(blob, img + 16 * sl + 8, 1)[0])
        hdr = u32(blob, img + z, 4).tolist()
        Lg = int(np.prod([int(net["fn_off"][v + 1] - net["fn_off"][v]) for v in members]))
        assert hdr == [4 * (2 + 2 * h["alias_g"] + s_idx), Lg, s_idx, 0]
        t = u32(blob, img + z + 16, 2 * Lg).reshape(Lg, 2)
        assert t[:, 0].tolist() == ref["tables"][s_idx][0]
        assert t[:, 1].tolist() == ref["tables"][s_idx][1]
        seen.add(sl)
    assert len(seen) == h["n_sel"]


def test_keyed_plans_carry_no_alias_tables():
    net = NETS["c2"]
    plan = api.Plan(net, interest=interest_of(net))
    h = header(plan.blob())
    assert h["sampling"] == 0 and h["n_sel"] == 0 and h["alias_g"] == 0


def test_sampling_option_is_validated():
    with pytest.raises(RuntimeError):
        api.Plan(NETS["tiny"], interest=[0], sampling=2)


def test_pattern_table_law_within_quantisation():
    # the library's 2^k table for the kept nodes of C2 encodes Algorithm 2's
    # pattern law to 2^-31 and Theorem 1's masked marginals to p
    net = NETS["c2"]
    plan = api.Plan(net, interest=interest_of(net), sampling=1, reduce=1, group=0)
    blob = plan.blob()
    h = header(blob)
    k, kp, p = h["alias_k"], h["alias_kp"], float(net["p"])
    tab = u32(blob, h["pert_off"], 2 << k).reshape(1 << k, 2)
    law = alias.quantised_law(tab[:, 0].tolist(), tab[:, 1].tolist(), 1 << k, column_bits=k)
    dist = [w / 2.0 ** 64 for w in law]
    want = alias.pattern_probs(k, p)
    assert max(abs(a - b) for a, b in zip(dist, want)) < 2 ** -31
    assert np.allclose(alias.masked_marginals(dist, kp), p, rtol=1e-6)


def test_batch_entry_points_reject_alias_plans():
    import ctypes as C
    from paper_1605_00854_amd._lib import lib
    plan = api.Plan(NETS["tiny"], interest=[0], sampling=1)
    arr = (C.c_void_p * 1)(plan.handle.value)
    ntraj = (C.c_uint32 * 1)(4)
    nt = C.c_uint32()
    assert lib().pbn_batch_tasks(arr, ntraj, 1, 4, 1, None, None, None, C.byref(nt)) != 0
    keyed = api.Plan(NETS["tiny"], interest=[0])
    arr = (C.c_void_p * 1)(keyed.handle.value)
    assert lib().pbn_batch_tasks(arr, ntraj, 1, 4, 1, None, None, None, C.byref(nt)) == 0 and nt.value == 1


@pytest.mark.parametrize("opts", [dict(reduce=1, group=0), dict(reduce=1, group=1, lds_budget_bytes=0),
                                  dict(reduce=0, group=0, sampling=1)])
def test_image_carries_the_chain_tables(opts):
    # the perturbation chain reads Q[0..n] and the orig -> position map from
    # the image (LDS-resident with it): copies of the blob's own tables
    net = NETS["c2"]
    plan = api.Plan(net, interest=interest_of(net), **opts)
    blob = plan.blob()
    h = header(blob)
    n = h["n"]
    img = h["image_off"]
    assert h["q_img"] % 16 == 0 and h["o2p_img"] >= h["q_img"] + 8 * (n + 1)
    assert h["o2p_img"] + 4 * n <= h["image_bytes"]
    q_blob = np.frombuffer(blob[h["q_off"]:h["q_off"] + 8 * (n + 1)].tobytes(), dtype="<u8")
    q_img = np.frombuffer(blob[img + h["q_img"]:img + h["q_img"] + 8 * (n + 1)].tobytes(), dtype="<u8")
    assert np.array_equal(q_blob, q_img)
    assert u32(blob, img + h["o2p_img"], n).tolist() == [int(x) for x in plan.node_pos()]
