"""Allocation-free batch launch (pbn_batch_launch_noalloc): the control block
and task schedule live in the library's device array, and the result must be
the existing entry point's (pbn_batch_launch with caller-owned workspace),
state and counters bit for bit, on two calls in a row, the second with a
smaller batch (the array keeps the first call's schedule, which must not
leak into the second)."""
import sys

import numpy as np
import pytest

import pbn_synth as ps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1605_00854_amd import _lib, api  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def items_of(count, seed, ntraj):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.integers(20, 400))
        net = ps.medium_c2(n=n, p=float(rng.choice([1e-3, 1e-2])), seed=seed * 100 + k)
        tgs = [ps.non_leaf_targets(net, 2)]
        opts = dict(reduce=1, group=1, max_parent_bits=6) if k % 2 else dict(reduce=1, group=0)
        plan = api.Plan(net, interest=[a for a, _ in tgs[0]], **opts)
        out.append((plan, 5000 + k, ntraj[k % len(ntraj)], tgs))
    return out


def run_both(items, step0, nsteps, wpb):
    ref = api.Batch(items, count_from=10, waves_per_block=wpb)
    new = api.Batch(items, count_from=10, waves_per_block=wpb)
    ref.init_states()
    new.init_states()
    ref.set_window(step0, nsteps)
    ref.launch()
    new.launch_noalloc(step0, nsteps)
    torch.cuda.synchronize()
    for k in range(len(items)):
        assert torch.equal(ref.states[k], new.states[k]), f"state of item {k}"
        assert torch.equal(ref.counts[k], new.counts[k]), f"counters of item {k}"
    assert sum(int(c[:, :, 0].sum()) for c in new.counts) > 0, "no step was counted"
    return new


def test_noalloc_batch_matches_the_workspace_launch_twice_second_smaller():
    say("[gpu] allocation-free batch: 12 networks, then 3")
    big = items_of(12, 31, [37, 9, 64, 5])
    run_both(big, 0, 300, 4)
    small = items_of(3, 32, [6, 2])
    run_both(small, 40, 120, 4)


def test_noalloc_batch_rejects_more_tasks_than_its_array():
    items = items_of(2, 33, [4])
    b = api.Batch(items, waves_per_block=1)
    b._ntraj = np.asarray([70000, 4], dtype=np.uint32)    # host counts beyond the array's 65 536 tasks
    with pytest.raises(_lib.PbnError, match="tasks"):
        b.launch_noalloc(0, 10)
