"""Continuous-batching server for steady-state queries.

A query asks for P(target state set) of one resident network at precision r
and confidence conf (the estimate of Section 4.2).  Network plans stay resident
on the device.  Each query owns its trajectory slots: its trajectories are
keyed by seed = H(network seed, query id), run a burn-in, then advance in
chunks; after every chunk its own counters decide (t interval over its
trajectories) whether its precision is met.  Because the keying and the chunk
schedule depend only on the query, its result is bit-identical whether it runs
alone or mixed with others; the mix only changes latency.

Queries advance in lanes.  A lane holds the admitted queries of one chunk
length and moves all of them by one chunk per persistent batched launch
(pbn_batch_launch) on its own stream; lanes run concurrently and each starts
its next launch as soon as the host has decided on its previous one, so a
query on a small network never waits for the step latency of a large one.  A
query's chunk is fixed by its own plan: the base chunk times the power of two
(up to 2^(chunk_classes - 1)) that brings its estimated step cost closest to,
without exceeding, that of the costliest resident network, so lanes take
about equally long per launch.  In the lanes of the costlier networks several
waves advance each trajectory together (four in the two costliest chunk
classes, two in the next), which shortens the step latency that a query's
latency is made of; the results do not depend on it.  Queries that arrive while others are on the
device join their lane at its next launch as soon as their footprint
(resident waves, LDS bytes, HBM bytes) fits, and leave when their precision
is met.  A lane's work items, task list and control block stay on the device
and are rewritten only when its set of queries changes; its step window
advances on the device after each launch, and each item's step offset is
fixed at the launch its query joined.  Counters come back through an
asynchronous copy into pinned host memory and an event the host polls.
"""
import hashlib
import time
from dataclasses import dataclass, field

import numpy as np

from . import _lib, api


@dataclass
class Query:
    qid: int
    net: int                    # index of the resident network
    targets: list               # [(node, value)]
    precision: float
    conf: float = 0.95
    arrival: float = 0.0        # seconds since the start of the run
    # filled by the server
    status: str = "queued"
    admitted: float = None
    finished: float = None
    steps: int = 0
    result: dict = field(default_factory=dict)
    error: str = None


def query_seed(net_seed, qid):
    h = hashlib.sha256(f"{net_seed}:{qid}".encode()).digest()
    return int.from_bytes(h[:8], "little")


def non_sink_nodes(net):
    """Nodes that some predictor reads (at least one child): the interest set
    of a resident plan, so Definition 1 removes exactly the network's sinks."""
    used = np.zeros(int(net["n"]), dtype=bool)
    used[np.asarray(net["parents"], dtype=np.int64)] = True
    return frozenset(np.nonzero(used)[0].tolist())


class Footprint:
    """Device budget for admission: resident waves, LDS bytes, HBM bytes."""

    def __init__(self, waves=256 * 32, lds_bytes=256 * 160 * 1024, hbm_bytes=8 << 30):
        self.cap = np.array([waves, lds_bytes, hbm_bytes], dtype=np.float64)
        self.used = np.zeros(3)

    def fits(self, need):
        return bool(np.all(self.used + need <= self.cap))

    def exceeds_device(self, need):
        return bool(np.any(need > self.cap))

    def take(self, need):
        self.used += need

    def give(self, need):
        self.used -= need


class _Resident:
    """Device buffers that outlive ticks: work items, tasks, first trajectory
    of each task, control block; grown (never shrunk) by doubling."""

    def __init__(self, torch):
        self.torch = torch
        self.items = torch.zeros(0, dtype=torch.uint8, device="cuda")
        self.tasks = torch.zeros(0, dtype=torch.int32, device="cuda")
        self.first = torch.zeros(0, dtype=torch.int32, device="cuda")

    def _fit(self, buf, nelem, dtype):
        if buf.numel() >= nelem:
            return buf
        return self.torch.zeros(max(nelem, 2 * buf.numel()), dtype=dtype, device="cuda")

    def upload(self, works, tasks, first):
        torch = self.torch
        raw = np.frombuffer(bytes(works), dtype=np.uint8)
        self.items = self._fit(self.items, raw.size, torch.uint8)
        self.tasks = self._fit(self.tasks, tasks.size, torch.int32)
        self.first = self._fit(self.first, first.size, torch.int32)
        # stream-ordered copies: they run after the launches already enqueued
        self.items[:raw.size].copy_(torch.from_numpy(raw.copy()).pin_memory(), non_blocking=True)
        self.tasks[:tasks.size].copy_(torch.from_numpy(tasks.astype(np.int32)).pin_memory(), non_blocking=True)
        self.first[:first.size].copy_(torch.from_numpy(first.astype(np.int32)).pin_memory(), non_blocking=True)


# Estimated cost of a perturbation-only step, in lane passes of an
# unperturbed one: the skip-chain walk with its reads of Q and of the
# position map (served networks: about 8 passes' worth per step)
PERT_PASSES = 8.0


class _Lane:
    """Queries of one chunk length: one batched launch of `chunk` steps at a
    time on the lane's own stream, with resident work items, task list and
    control block."""

    def __init__(self, torch, chunk):
        self.chunk = int(chunk)
        self.stream = torch.cuda.Stream()           # default priority
        with torch.cuda.stream(self.stream):
            self.res = _Resident(torch)
            self.ctl = api.new_ctl(0, self.chunk)
        self.window = 0            # host mirror of the control block's step window
        self.dirty = True          # the lane's query set changed since its items were written
        self.active = []
        self.ntasks = 0
        self.queue_first = None    # the launch's task-queue bounds (host)
        self.wpt = 1               # waves per trajectory of the lane's launches
        self.plans_arr = None
        self.inflight = None       # (queries, steps after the launch, pinned counts, event)
        self.launches = 0

    def wpb(self, wpb):
        """Trajectories per task: one when several waves share a trajectory."""
        return 1 if self.wpt > 1 else wpb


class Server:
    def __init__(self, nets, net_seeds, *, plan_opts=None, traj_per_query=256, chunk=1000, burn_in=1000,
                 min_counted=1000, max_steps=400000, waves_per_block=4, footprint=None, chunk_classes=3,
                 task_queues=api.DEFAULT_QUEUES, waves_per_traj=(4, 4, 2)):
        import torch
        self.torch = torch
        self.nets = nets
        self.net_seeds = list(net_seeds)
        self.opts = dict(plan_opts or dict(reduce=1, group=0))
        self.ntraj = int(traj_per_query)
        self.chunk = int(chunk)
        self.max_mult = 1 << max(0, int(chunk_classes) - 1)
        self.burn_in = int(burn_in)
        self.min_counted = int(min_counted)
        self.max_steps = int(max_steps)
        self.wpb = int(waves_per_block)
        self.task_queues = int(task_queues)   # per launch: networks dealt to the CU groups' task queues
        # waves per trajectory of the lane of chunk base x 2^j: entry j (the
        # last one for larger j); the costliest networks run in the base lane.
        # (4, 4, 2) served the 2000-query Poisson stream fastest of those
        # measured: one wave per trajectory gave p50 12.6 / p99 34.4 ms, this
        # 8.2 / 23.4 ms, (8, 4, 2) 9.4 / 30.9 ms
        self.wpt = tuple(int(w) for w in (waves_per_traj if isinstance(waves_per_traj, (tuple, list))
                                          else (waves_per_traj,)))
        self.fp = footprint or Footprint()
        self.plans = {}
        self.base_interest = [non_sink_nodes(net) for net in nets]
        self.cost_max = max(self._cost(k, self._plan(k, ())) for k in range(len(nets)))
        self.queue, self.done = [], []
        self.lanes = {}
        self.node_updates = 0
        self.ticks = 0

    # -- resident plans: interest = every node some predictor reads, plus the
    # nodes of queries that asked for a removed node
    def _plan(self, k, extra):
        key = (k, self.base_interest[k] | frozenset(extra))
        if key not in self.plans:
            plan = api.Plan(self.nets[k], interest=sorted(key[1]), **self.opts)
            plan.device()
            self.plans[key] = plan
        return self.plans[key]

    def _resident(self, k, targets):
        plan = self._plan(k, ())
        try:
            return plan, plan.targets([targets])
        except _lib.PbnError:
            # a query on a node the reduction removed: prepare with that node kept
            plan = self._plan(k, [a for a, _ in targets])
            return plan, plan.targets([targets])

    def _cost(self, k, plan):
        """Estimated time of one trajectory-step, in lane passes: a step
        without perturbation (probability (1-p)^n) evaluates every pass."""
        net = self.nets[k]
        f = (1.0 - float(net["p"])) ** int(net["n"])
        return f * plan.info["n_passes"] + (1.0 - f) * PERT_PASSES

    def chunk_of(self, k, plan):
        """The query's chunk: the base chunk times the largest power of two
        (at most max_mult) whose multiple of this plan's step cost stays
        within the costliest resident network's."""
        m, c = 1, self._cost(k, plan)
        while 2 * m <= self.max_mult and 2 * m * c <= self.cost_max:
            m *= 2
        return self.chunk * m

    def footprint(self, plan, wpt=1):
        """(waves, LDS bytes, HBM bytes) of one query: wpt waves per trajectory
        share its LDS state and ring, and with wpt > 1 a copy of the chain
        tables (Q and the position map, 12 bytes a node)."""
        ring = plan.info["n_jobs"]
        fill = min(32, plan.fill_steps) if ring <= 64 else 1
        traj_lds = 2 * plan.info["state_bytes"] + 16 * (fill * ring if ring <= 64 else ring)
        if wpt > 1:
            n = plan.info["n"]
            traj_lds += ((8 * (n + 1) + 15) & ~15) + ((4 * n + 15) & ~15)
        hbm = self.ntraj * (4 * plan.info["state_words"] + 24)
        return np.array([self.ntraj * wpt, self.ntraj * traj_lds, hbm], dtype=np.float64)

    def wpt_of(self, chunk):
        """Waves per trajectory of the lane of this chunk length."""
        j = max(0, (chunk // self.chunk).bit_length() - 1)
        return self.wpt[min(j, len(self.wpt) - 1)]

    # -- queue management
    def submit(self, q, now):
        try:
            plan, tg = self._resident(q.net, q.targets)
        except _lib.PbnError as e:
            q.status, q.error, q.finished = "rejected", str(e), now
            self.done.append(q)
            return
        chunk = self.chunk_of(q.net, plan)
        need = self.footprint(plan, self.wpt_of(chunk))
        if self.fp.exceeds_device(need):
            q.status, q.error, q.finished = "rejected", "footprint exceeds the device budget", now
            self.done.append(q)
            return
        q._plan, q._tg, q._need = plan, tg, need
        q._chunk = chunk
        self.queue.append(q)

    def _lane(self, chunk):
        if chunk not in self.lanes:
            lane = _Lane(self.torch, chunk)
            lane.wpt = self.wpt_of(chunk)
            self.lanes[chunk] = lane
        return self.lanes[chunk]

    def _admit(self, now):
        while self.queue and self.fp.fits(self.queue[0]._need):
            q = self.queue.pop(0)
            self.fp.take(q._need)
            q.status, q.admitted = "running", now
            q._seed = query_seed(self.net_seeds[q.net], q.qid)
            # initial states and zero counters on the current stream; a lane
            # waits for it before its next launch
            q._state = api.state_init(q._plan, q._seed, self.ntraj)
            q._counts = api.new_counts(1, self.ntraj)
            q._tg_dev = api._to_device_bytes(q._tg)
            lane = self._lane(q._chunk)
            lane.active.append(q)
            lane.dirty = True

    def _write_items(self, lane):
        """Work items and tasks of the lane's queries into its resident
        buffers.  Item k's step offset makes its steps (offset + window)
        continue from the query's own step count."""
        act = lane.active
        works = (_lib.pbn_work * len(act))()
        for k, q in enumerate(act):
            off = (q.steps - lane.window) & 0xFFFFFFFF
            works[k] = _lib.pbn_work(q._plan.device().data_ptr(), q._tg_dev.data_ptr(), q._state.data_ptr(),
                                     q._counts.data_ptr(), q._seed, 0, self.ntraj, self.burn_in, off)
        lane.plans_arr = (api.C.c_void_p * len(act))(*[q._plan.handle.value for q in act])
        ntraj = np.full(len(act), self.ntraj, dtype=np.uint32)
        tasks, first, lane.queue_first = api.batch_schedule(lane.plans_arr, ntraj, lane.wpb(self.wpb),
                                                            self.task_queues)
        lane.res.upload(works, tasks, first)
        lane.ntasks = int(tasks.size)
        lane.dirty = False

    def _enqueue(self, lane):
        """One launch of the lane: every query of it advances one chunk; then an
        asynchronous copy of their counters and an event, all on its stream."""
        torch = self.torch
        lane.stream.wait_stream(torch.cuda.current_stream())   # states of newly admitted queries
        with torch.cuda.stream(lane.stream):
            if lane.dirty:
                self._write_items(lane)
            act = list(lane.active)
            L = _lib.lib()
            _lib.check(L.pbn_batch_launch(lane.plans_arr, len(act), api._dptr(lane.res.items),
                                          api._dptr(lane.res.tasks), api._dptr(lane.res.first), lane.ntasks,
                                          api._ptr(lane.queue_first, api.C.c_uint32), self.task_queues,
                                          api._dptr(lane.ctl), lane.wpb(self.wpb), lane.wpt,
                                          api._stream(lane.stream)))
            lane.window = (lane.window + lane.chunk) & 0xFFFFFFFF
            for q in act:
                q.steps += lane.chunk
                self.node_updates += self.ntraj * lane.chunk * q._plan.n
            counts = torch.cat([q._counts.view(-1) for q in act])
            host = torch.empty(counts.shape, dtype=counts.dtype, pin_memory=True)
            host.copy_(counts, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(lane.stream)
        lane.launches += 1
        self.ticks += 1
        lane.inflight = (act, [q.steps for q in act], host, ev)

    def _decide(self, lane, now_fn):
        """Decisions on the lane's finished launch; finished queries leave."""
        act, steps, host, ev = lane.inflight
        lane.inflight = None
        ev.synchronize()
        now = now_fn()
        counts = host.numpy()
        per = 3 * self.ntraj
        leaving = set()
        for k, (q, st) in enumerate(zip(act, steps)):
            counted = st - self.burn_in
            c = counts[k * per:(k + 1) * per].reshape(self.ntraj, 3)
            finished = False
            if counted >= self.min_counted:
                est = api.estimate(c, counted, conf=q.conf, precision=q.precision)
                q.result = est
                if est["half_width"] <= q.precision:
                    q.status = "done"
                    finished = True
                elif st >= self.max_steps:
                    q.status = "max_steps"
                    finished = True
            if finished:
                q.finished = now
                q.result["counts"] = c.copy()
                self.fp.give(q._need)
                self.done.append(q)
                leaving.add(id(q))
                for name in ("_state", "_counts", "_tg_dev"):
                    setattr(q, name, None)
        if leaving:
            lane.active = [q for q in lane.active if id(q) not in leaving]
            lane.dirty = True

    def busy(self):
        return any(lane.active or lane.inflight is not None for lane in self.lanes.values())

    def tick(self, now_fn, wait=False):
        """One scheduling round: decide on every lane whose launch has
        finished (with wait, on the oldest one in flight whatever its state),
        admit queued queries that fit, launch every idle lane that holds
        queries.  Returns whether a decision was taken or a launch made."""
        moved = False
        if wait:
            flying = [lane for lane in self.lanes.values() if lane.inflight is not None]
            if flying:
                self._decide(min(flying, key=lambda ln: ln.launches), now_fn)
                moved = True
        for lane in self.lanes.values():
            if lane.inflight is not None and lane.inflight[3].query():
                self._decide(lane, now_fn)
                moved = True
        self._admit(now_fn())
        for lane in self.lanes.values():
            if lane.inflight is None and lane.active:
                self._enqueue(lane)
                moved = True
        return moved

    def run(self, queries, realtime=True):
        """Serve `queries` (arrival times in seconds).  Returns the metrics dict."""
        pending = sorted(queries, key=lambda q: q.arrival)
        t0 = time.perf_counter()
        now = (lambda: time.perf_counter() - t0) if realtime else (lambda: float(self.ticks))
        i = 0
        while i < len(pending) or self.queue or self.busy():
            tnow = now()
            while i < len(pending) and (pending[i].arrival <= tnow or not realtime):
                self.submit(pending[i], tnow)
                i += 1
            moved = self.tick(now, wait=not realtime)
            if realtime and not moved:
                # nothing finished and nothing to launch: a short pause, or
                # until the next arrival when the device is idle
                pause = 1e-4 if self.busy() or i >= len(pending) else pending[i].arrival - now()
                time.sleep(max(0.0, min(0.01, pause)))
        self.torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return self.metrics(wall)

    def metrics(self, wall):
        lat = np.array([q.finished - q.arrival for q in self.done if q.status in ("done", "max_steps")])
        return {
            "queries": len(self.done),
            "done": sum(q.status == "done" for q in self.done),
            "max_steps": sum(q.status == "max_steps" for q in self.done),
            "rejected": sum(q.status == "rejected" for q in self.done),
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "node_updates_per_s": self.node_updates / wall if wall > 0 else None,
            "wall_s": wall,
            "ticks": self.ticks,
            "lanes": {str(c): lane.launches for c, lane in sorted(self.lanes.items())},
            "waves_per_traj": {str(c): lane.wpt for c, lane in sorted(self.lanes.items())},
        }


def poisson_queries(nets, count, rate, seed=2005, precisions=(1e-2, 5e-3), conf=0.95):
    """The served workload: Poisson arrivals, 1-5 random non-leaf nodes with a
    random ON/OFF pattern, precision drawn from `precisions`."""
    import pbn_synth as ps
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for qid in range(count):
        t += rng.exponential(1.0 / rate)
        k = int(rng.integers(0, len(nets)))
        tg = ps.random_query_targets(rng, nets[k])
        out.append(Query(qid, k, tg, float(rng.choice(precisions)), conf, t))
    return out
