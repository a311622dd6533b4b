"""Host side of the batched launch (no device): the task schedule that deals
networks to the per-XCD task queues, and the launch's checks of the queue
bounds, which reject bad bounds before anything touches a device."""
import ctypes as C
import os

import numpy as np
import pytest

import pbn_synth as ps
from paper_1605_00854_amd import api
from paper_1605_00854_amd._lib import EINVAL, lib

WPB = 4


@pytest.fixture(scope="module")
def batch():
    rng = np.random.default_rng(5)
    plans, ntraj = [], []
    for k in range(23):
        n = int(rng.integers(20, 700))
        net = ps.medium_c2(n=n, p=1e-3, seed=700 + k)
        plans.append(api.Plan(net, interest=[a for a, _ in ps.non_leaf_targets(net, 2)], reduce=1, group=0))
        ntraj.append(int(rng.choice([1, 5, 64, 256])))
    arr = (C.c_void_p * len(plans))(*[p.handle.value for p in plans])
    return plans, arr, np.asarray(ntraj, dtype=np.uint32)


def cost(plan):
    return plan.info["n_passes"] * plan.info["n_jobs"] + plan.info["n_slots"]


def test_header_constants_match_the_binding():
    root = os.path.dirname(os.path.dirname(os.path.abspath(api.__file__)))
    text = open(os.path.join(root, "include", "pbn.h")).read()
    assert f"#define PBN_BATCH_QUEUES {api.BATCH_QUEUES}" in text
    # control block: step0, nsteps, ntasks, reserved, one counter per queue
    assert api.CTL_WORDS == 4 + api.BATCH_QUEUES
    assert 1 <= api.DEFAULT_QUEUES <= api.BATCH_QUEUES and api.DEFAULT_QUEUES % 8 == 0


@pytest.mark.parametrize("nqueues", [1, 3, 8, 32, 64])
def test_schedule_deals_whole_networks_to_queues(batch, nqueues):
    plans, arr, ntraj = batch
    tasks, first, qf = api.batch_schedule(arr, ntraj, WPB, nqueues)
    ntasks = int(sum((int(t) + WPB - 1) // WPB for t in ntraj))
    assert tasks.size == ntasks and qf.size == nqueues + 1 and qf[0] == 0 and qf[-1] == ntasks
    assert np.all(np.diff(qf.astype(np.int64)) >= 0)
    queue_of = {}
    load = np.zeros(nqueues, dtype=np.int64)
    for j in range(nqueues):
        seg_items = tasks[qf[j]:qf[j + 1]]
        seg_first = first[qf[j]:qf[j + 1]]
        # each network's tasks are one contiguous run of one queue, covering its
        # trajectories in steps of WPB
        runs = [seg_items[0]] if seg_items.size else []
        for a, b in zip(seg_items[:-1], seg_items[1:]):
            if a != b:
                runs.append(b)
        assert len(runs) == len(set(runs))
        for k in runs:
            assert k not in queue_of
            queue_of[int(k)] = j
            sel = seg_first[seg_items == k]
            assert np.array_equal(sel, np.arange(0, int(ntraj[k]), WPB))
            load[j] += cost(plans[k]) * sel.size
        # largest networks first within a queue
        costs = [cost(plans[k]) for k in runs]
        assert costs == sorted(costs, reverse=True)
    assert sorted(queue_of) == list(range(len(plans)))
    # dealt largest first to the least-loaded queue: no queue exceeds another
    # by more than the largest single network's work
    biggest = max(cost(p) * ((int(t) + WPB - 1) // WPB) for p, t in zip(plans, ntraj))
    assert load.max() - load.min() <= biggest


def test_one_queue_keeps_the_global_largest_first_order(batch):
    plans, arr, ntraj = batch
    tasks, first, qf = api.batch_schedule(arr, ntraj, WPB, 1)
    costs = [cost(plans[k]) for k in tasks]
    assert costs == sorted(costs, reverse=True)
    assert list(qf) == [0, tasks.size]


def test_schedule_rejects_bad_queue_counts(batch):
    _, arr, ntraj = batch
    nt = C.c_uint32()
    for nq in (0, api.BATCH_QUEUES + 1):
        assert lib().pbn_batch_tasks(arr, api._ptr(ntraj, C.c_uint32), ntraj.size, WPB, nq, None, None, None,
                                     C.byref(nt)) != 0


@pytest.mark.parametrize("bounds,message", [
    ([1, 2, 3, 4, 5, 6, 7, 8, 10], b"queue bounds"),        # does not start at 0
    ([0, 2, 3, 4, 5, 6, 7, 8, 9], b"queue bounds"),         # does not end at ntasks
    ([0, 5, 3, 6, 7, 8, 9, 10, 10], b"queue bounds"),       # decreasing
    ([0] * (api.BATCH_QUEUES + 1) + [10], b"nqueues"),      # more queues than the launch holds
])
def test_launch_rejects_bad_queue_bounds_before_any_device_work(batch, bounds, message):
    plans, arr, _ = batch
    qf = np.asarray(bounds, dtype=np.uint32)
    fake = C.c_void_p(256)                # never dereferenced: the bounds are checked first
    st = lib().pbn_batch_launch(arr, 1, fake, fake, fake, 10, api._ptr(qf, C.c_uint32), qf.size - 1, fake, WPB, 1,
                                None)
    assert st == EINVAL
    assert message in lib().pbn_last_error()


@pytest.mark.parametrize("wpb,wpt", [(4, 2), (1, 0), (1, 17)])
def test_launch_rejects_bad_waves_per_trajectory(batch, wpb, wpt):
    plans, arr, _ = batch
    fake = C.c_void_p(256)                # never dereferenced: the shape is checked first
    st = lib().pbn_batch_launch(arr, 1, fake, fake, fake, 10, None, 1, fake, wpb, wpt, None)
    assert st == EINVAL
    assert b"waves_per_traj" in lib().pbn_last_error()


@pytest.mark.parametrize("nqueues", [5, 64])
def test_schedule_equals_a_longest_processing_time_deal(batch, nqueues):
    """The queue of every network, recomputed: networks in order of per-step
    cost (largest first, stable on ties), each dealt to the queue with the
    least work so far (work = cost x tasks; ties: the lowest queue)."""
    plans, arr, ntraj = batch
    tasks, first, qf = api.batch_schedule(arr, ntraj, WPB, nqueues)
    order = sorted(range(len(plans)), key=lambda k: -cost(plans[k]))
    load = [0] * nqueues
    want = {}
    for k in order:
        j = min(range(nqueues), key=lambda q: (load[q], q))
        want[k] = j
        load[j] += cost(plans[k]) * ((int(ntraj[k]) + WPB - 1) // WPB)
    got = {}
    for j in range(nqueues):
        for k in tasks[qf[j]:qf[j + 1]]:
            got[int(k)] = j
    assert got == want
    # within a queue, networks appear in the deal's order
    for j in range(nqueues):
        seen = []
        for k in tasks[qf[j]:qf[j + 1]]:
            if not seen or seen[-1] != int(k):
                seen.append(int(k))
        assert seen == [k for k in order if want[k] == j]
