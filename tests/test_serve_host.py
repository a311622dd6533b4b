"""Host logic of the query server (no device): the chunk a query advances per
launch of its lane depends only on its own plan and the resident networks,
and the footprint admission keeps the budget."""
import types

import numpy as np
import pytest

from paper_1605_00854_amd import serve


def bare_server(nets, passes, chunk=500, chunk_classes=3):
    """A Server with only the fields chunk_of reads (its constructor builds
    device plans); the costliest resident network sets the reference."""
    srv = serve.Server.__new__(serve.Server)
    srv.nets = nets
    srv.chunk = chunk
    srv.max_mult = 1 << (chunk_classes - 1)
    plans = [types.SimpleNamespace(info={"n_passes": p}) for p in passes]
    srv.cost_max = max(srv._cost(k, plans[k]) for k in range(len(nets)))
    return srv, plans


def test_step_cost_weighs_passes_by_unperturbed_steps():
    nets = [{"n": 1000, "p": 1e-4}, {"n": 1000, "p": 1e-3}]
    srv, plans = bare_server(nets, [16, 16])
    f0, f1 = (1 - 1e-4) ** 1000, (1 - 1e-3) ** 1000
    assert srv._cost(0, plans[0]) == pytest.approx(f0 * 16 + (1 - f0) * serve.PERT_PASSES)
    assert srv._cost(1, plans[1]) == pytest.approx(f1 * 16 + (1 - f1) * serve.PERT_PASSES)
    assert srv._cost(1, plans[1]) < srv._cost(0, plans[0])     # most of its steps only walk the chain


def test_chunks_are_powers_of_two_of_the_base_up_to_the_class_limit():
    nets = [{"n": 3000, "p": 1e-4}, {"n": 1500, "p": 1e-4}, {"n": 700, "p": 1e-4}, {"n": 100, "p": 1e-4},
            {"n": 3000, "p": 1e-3}]
    srv, plans = bare_server(nets, [40, 20, 10, 2, 40])
    chunks = [srv.chunk_of(k, plans[k]) for k in range(len(nets))]
    assert chunks[0] == 500                       # the costliest network keeps the base chunk
    # costs 31.7, 18.3, 9.9, 2.1 and 9.6 passes per step: twice 18.3 exceeds
    # 31.7; the smallest network is capped at 4x
    assert chunks[:4] == [500, 500, 1000, 2000]
    for k, c in enumerate(chunks):
        m = c // 500
        assert c % 500 == 0 and m & (m - 1) == 0
        # the multiple never makes a launch costlier than the reference's
        assert m * srv._cost(k, plans[k]) <= srv.cost_max + 1e-12
        if m < srv.max_mult:
            assert 2 * m * srv._cost(k, plans[k]) > srv.cost_max
    # a high perturbation rate makes a large network cheap per step
    assert chunks[4] == 1000


def test_one_chunk_class_keeps_the_base_chunk_everywhere():
    nets = [{"n": 3000, "p": 1e-4}, {"n": 100, "p": 1e-4}]
    srv, plans = bare_server(nets, [40, 2], chunk=400, chunk_classes=1)
    assert [srv.chunk_of(k, plans[k]) for k in range(2)] == [400, 400]


def test_footprint_budget_takes_and_gives_back():
    fp = serve.Footprint(waves=1000, lds_bytes=10_000, hbm_bytes=1 << 20)
    need = np.array([256, 4000, 1000], dtype=np.float64)
    assert fp.fits(need)
    fp.take(need)
    fp.take(need)
    assert not fp.fits(need)                      # the third exceeds the LDS budget
    fp.give(need)
    assert fp.fits(need) and np.allclose(fp.used, need)
    assert fp.exceeds_device(np.array([2000, 1, 1], dtype=np.float64))


def test_lane_waves_per_trajectory_follow_the_chunk_class():
    srv, _ = bare_server([{"n": 100, "p": 1e-4}], [2], chunk=500, chunk_classes=3)
    srv.wpt = (4, 4, 2)
    assert [srv.wpt_of(c) for c in (500, 1000, 2000, 4000)] == [4, 4, 2, 2]
    srv.wpt = (1,)
    assert [srv.wpt_of(c) for c in (500, 1000, 2000)] == [1, 1, 1]


def test_footprint_counts_waves_and_chain_tables_of_multi_wave_lanes():
    srv = serve.Server.__new__(serve.Server)
    srv.ntraj = 256
    plan = types.SimpleNamespace(info={"n_jobs": 100, "state_bytes": 3008, "state_words": 94, "n": 3000},
                                 fill_steps=1)
    one = srv.footprint(plan, 1)
    four = srv.footprint(plan, 4)
    assert one[0] == 256 and four[0] == 1024                 # waves
    chain = (8 * 3001 + 15) // 16 * 16 + (4 * 3000 + 15) // 16 * 16
    assert four[1] - one[1] == 256 * chain                   # LDS: the chain tables of each trajectory
    assert four[2] == one[2]                                 # HBM: states and counters only
