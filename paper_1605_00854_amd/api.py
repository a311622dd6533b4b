"""Python binding of the PBN simulator (marshalling only: every step of the
simulation runs in the library's HIP kernels).

Device memory and streams come from PyTorch: buffers are torch tensors on the
current HIP device and launches go to torch's current stream.
"""
import ctypes as C

import numpy as np

from . import _lib
from ._lib import check, lib


def _ptr(arr, ctype):
    return arr.ctypes.data_as(C.POINTER(ctype))


class Net:
    """A validated, quantised PBN (pbn_net_create)."""

    def __init__(self, net):
        self.desc_dict = net
        self.n = int(net["n"])
        arrs = {
            "fn_off": np.ascontiguousarray(net["fn_off"], dtype=np.uint32),
            "sel_prob": np.ascontiguousarray(net["sel_prob"], dtype=np.float64),
            "par_off": np.ascontiguousarray(net["par_off"], dtype=np.uint32),
            "parents": np.ascontiguousarray(net["parents"], dtype=np.uint32),
            "tt_off": np.ascontiguousarray(net["tt_off"], dtype=np.uint32),
            "tt": np.ascontiguousarray(net["tt"], dtype=np.uint64),
        }
        if arrs["parents"].size == 0:
            arrs["parents"] = np.zeros(1, dtype=np.uint32)
        d = _lib.pbn_desc(self.n, float(net["p"]), _ptr(arrs["fn_off"], C.c_uint32),
                          _ptr(arrs["sel_prob"], C.c_double), _ptr(arrs["par_off"], C.c_uint32),
                          _ptr(arrs["parents"], C.c_uint32), _ptr(arrs["tt_off"], C.c_uint32),
                          _ptr(arrs["tt"], C.c_uint64))
        h = C.c_void_p()
        check(lib().pbn_net_create(C.byref(d), C.byref(h)))
        self.handle = h
        self._libref = lib()

    def tables(self):
        """(Q[0..n], cum[n,3], rank[n]) of the random-number contract."""
        q = np.zeros(self.n + 1, dtype=np.uint64)
        cum = np.zeros(3 * self.n, dtype=np.uint64)
        rank = np.zeros(self.n, dtype=np.int32)
        check(lib().pbn_net_tables(self.handle, _ptr(q, C.c_uint64), _ptr(cum, C.c_uint64),
                                   _ptr(rank, C.c_int32)))
        return q, cum.reshape(self.n, 3), rank

    def __del__(self):
        # the library object is held by the instance: module globals may
        # already be gone when the interpreter shuts down
        h, L = getattr(self, "handle", None), getattr(self, "_libref", None)
        if h is not None and L is not None:
            L.pbn_net_destroy(h)
            self.handle = None


def default_opts():
    o = _lib.pbn_plan_opts()
    lib().pbn_plan_opts_default(C.byref(o))
    return o


class Plan:
    """Prepared network (Algorithm 5's Preparation) and its device blob."""

    def __init__(self, net, interest=(), **opts):
        self.net = net if isinstance(net, Net) else Net(net)
        o = default_opts()
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown plan option {k}")
            setattr(o, k, int(v))
        self.opts = o
        ints = np.ascontiguousarray(sorted(set(int(x) for x in interest)), dtype=np.uint32)
        if ints.size == 0:
            ints = np.zeros(1, dtype=np.uint32)
            nint = 0
        else:
            nint = ints.size
        h = C.c_void_p()
        check(lib().pbn_plan_build(self.net.handle, _ptr(ints, C.c_uint32), nint, C.byref(o), C.byref(h)))
        self.handle = h
        self._libref = lib()
        info = _lib.pbn_plan_info()
        check(lib().pbn_plan_info_get(h, C.byref(info)))
        self.info = {name: getattr(info, name) for name, _ in info._fields_ if name != "reserved"}
        self._dev = None

    @property
    def n(self):
        return self.info["n"]

    def node_pos(self):
        pos = np.zeros(self.n, dtype=np.uint32)
        check(lib().pbn_plan_node_pos(self.handle, _ptr(pos, C.c_uint32)))
        return pos

    def slots(self):
        slot = np.zeros(self.n, dtype=np.uint32)
        is_table = np.zeros(max(1, self.info["n_slots"]), dtype=np.uint32)
        check(lib().pbn_plan_slots(self.handle, _ptr(slot, C.c_uint32), _ptr(is_table, C.c_uint32)))
        return slot, is_table[: self.info["n_slots"]]

    def _groups(self, fn):
        nm, ng = C.c_uint32(), C.c_uint32()
        check(fn(self.handle, None, C.byref(nm), None, C.byref(ng)))
        mem = np.zeros(max(1, nm.value), dtype=np.uint32)
        off = np.zeros(ng.value + 1, dtype=np.uint32)
        check(fn(self.handle, _ptr(mem, C.c_uint32), C.byref(nm), _ptr(off, C.c_uint32), C.byref(ng)))
        return [mem[off[i]:off[i + 1]].tolist() for i in range(ng.value)]

    def alg4_groups(self):
        return self._groups(lib().pbn_plan_alg4_groups)

    def single_groups(self):
        return self._groups(lib().pbn_plan_single_groups)

    def blob(self):
        size = C.c_size_t()
        check(lib().pbn_plan_export(self.handle, None, C.byref(size)))
        buf = np.zeros(size.value, dtype=np.uint8)
        check(lib().pbn_plan_export(self.handle, buf.ctypes.data_as(C.c_void_p), C.byref(size)))
        return buf

    @property
    def fill_steps(self):
        """Steps per Philox fill of the step kernel's ring (plan header word 11)."""
        if getattr(self, "_fill", None) is None:
            self._fill = int(np.frombuffer(self.blob()[44:48].tobytes(), dtype="<u4")[0])
        return self._fill

    def device(self):
        """Device copy of the blob (torch uint8 tensor on the current device)."""
        if self._dev is None:
            import torch
            self._dev = torch.from_numpy(self.blob()).to("cuda")
        return self._dev

    def targets(self, target_sets):
        """pbn_targets for a list of target sets, each a list of (node, value)."""
        node, val, tof = [], [], []
        for t, tg in enumerate(target_sets):
            for a, b in tg:
                node.append(a)
                val.append(b)
                tof.append(t)
        out = _lib.pbn_targets()
        node = np.asarray(node, dtype=np.uint32)
        val = np.asarray(val, dtype=np.uint32)
        tof = np.asarray(tof, dtype=np.uint32)
        check(lib().pbn_targets_build(self.handle, _ptr(node, C.c_uint32), _ptr(val, C.c_uint32),
                                      _ptr(tof, C.c_uint32), node.size, len(target_sets), C.byref(out)))
        return out

    def __del__(self):
        # the library object is held by the instance: module globals may
        # already be gone when the interpreter shuts down
        h, L = getattr(self, "handle", None), getattr(self, "_libref", None)
        if h is not None and L is not None:
            L.pbn_plan_destroy(h)
            self.handle = None


def eq2_lower_bound(weights, theta):
    w = np.ascontiguousarray(weights, dtype=np.uint64)
    if w.size == 0:
        w = np.zeros(1, dtype=np.uint64)
        cnt = 0
    else:
        cnt = w.size
    m = C.c_uint32()
    check(lib().pbn_eq2_lower_bound(_ptr(w, C.c_uint64), cnt, int(theta), C.byref(m)))
    return m.value or None


def estimate(counts, steps_per_unit, conf=0.95, precision=0.01):
    """pbn_estimate on host counters [units][3] of one target; returns a dict."""
    c = np.ascontiguousarray(np.asarray(counts).reshape(-1, 3), dtype=np.uint64)
    out = _lib.pbn_estimate_out()
    check(lib().pbn_estimate(_ptr(c, C.c_uint64), c.shape[0], int(steps_per_unit), float(conf),
                             float(precision), C.byref(out)))
    return {name: getattr(out, name) for name, _ in out._fields_ if name != "reserved"}


def rl_diagnose(bits, nbits, precision, conf=0.95, eps=1e-3, kmax=100):
    """pbn_rl_diagnose on a host bit array (uint32 words, bit t = z_t)."""
    w = np.ascontiguousarray(np.asarray(bits).view(np.uint32) if np.asarray(bits).dtype == np.int32
                             else np.asarray(bits, dtype=np.uint32))
    out = _lib.pbn_rl_out()
    check(lib().pbn_rl_diagnose(_ptr(w, C.c_uint32), int(nbits), float(precision), float(conf), float(eps),
                                int(kmax), C.byref(out)))
    return {name: getattr(out, name) for name, _ in out._fields_ if name != "reserved"}


def skart_analyze(bits, nbits, precision, conf=0.95):
    """pbn_skart_analyze on a host bit array (uint32 words, bit t = z_t)."""
    w = np.ascontiguousarray(np.asarray(bits).view(np.uint32) if np.asarray(bits).dtype == np.int32
                             else np.asarray(bits, dtype=np.uint32))
    out = _lib.pbn_skart_out()
    check(lib().pbn_skart_analyze(_ptr(w, C.c_uint32), int(nbits), float(precision), float(conf), C.byref(out)))
    return {name: getattr(out, name) for name, _ in out._fields_}


def skart_run(plan, seed, target_sets, precision, *, traj=0, conf=0.95, max_steps=1 << 28, waves_per_block=0,
              stream=None):
    """Skart stopping rule on one trajectory (pbn_skart_run, blocking).

    Returns (analysis dict with "status", recorded indicator words as a device tensor)."""
    import torch
    tg = plan.targets(target_sets)
    words = (int(max_steps) + 31) // 32
    state = new_state(plan, 1)
    counts = new_counts(tg.ntargets, 1)
    record = torch.zeros(words, dtype=torch.int32, device="cuda")
    lo = _lib.pbn_launch_opts(int(waves_per_block))
    out = _lib.pbn_skart_out()
    rc = lib().pbn_skart_run(plan.handle, _dptr(plan.device()), int(seed), int(traj), C.byref(tg), _dptr(state),
                             _dptr(counts), _dptr(record), words, float(precision), float(conf), int(max_steps),
                             C.byref(lo), C.byref(out), _stream(stream))
    res = {name: getattr(out, name) for name, _ in out._fields_}
    res["status"] = int(rc)
    if rc not in (0, _lib.ERANGE):
        check(rc)
    return res, record


def unpack_record(words, nbits):
    """0/1 array of the first nbits bits of recorded words (bit t of word t // 32)."""
    w = np.asarray(words).view(np.uint32).reshape(-1)
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).reshape(-1)
    return bits[:nbits].astype(np.uint8)


def rl_run(plan, seed, target_sets, precision, *, traj=0, conf=0.95, eps=1e-3, kmax=100,
           initial_steps=100000, max_steps=1 << 28, waves_per_block=0, stream=None):
    """Two-state Markov chain approach on one trajectory (pbn_rl_run, blocking).

    Returns (diagnosis dict, recorded indicator words as a device tensor)."""
    import torch
    tg = plan.targets(target_sets)
    words = (int(max_steps) + 31) // 32
    state = new_state(plan, 1)
    counts = new_counts(tg.ntargets, 1)
    record = torch.zeros(words, dtype=torch.int32, device="cuda")
    lo = _lib.pbn_launch_opts(int(waves_per_block))
    out = _lib.pbn_rl_out()
    rc = lib().pbn_rl_run(plan.handle, _dptr(plan.device()), int(seed), int(traj), C.byref(tg), _dptr(state),
                          _dptr(counts), _dptr(record), words, float(precision), float(conf), float(eps),
                          int(kmax), int(initial_steps), int(max_steps), C.byref(lo), C.byref(out),
                          _stream(stream))
    res = {name: getattr(out, name) for name, _ in out._fields_ if name != "reserved"}
    res["status"] = int(rc)
    if rc not in (0, _lib.ERANGE):
        check(rc)
    return res, record


# ------------------------------------------------------------------ device

def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def new_state(plan, ntraj):
    import torch
    return torch.zeros((ntraj, plan.info["state_words"]), dtype=torch.int32, device="cuda")


def new_counts(ntargets, ntraj):
    import torch
    return torch.zeros((ntargets, ntraj, 3), dtype=torch.int64, device="cuda")


def state_init(plan, seed, ntraj, traj0=0, state=None, stream=None):
    state = new_state(plan, ntraj) if state is None else state
    check(lib().pbn_state_init(plan.handle, _dptr(plan.device()), int(seed), int(traj0), int(ntraj),
                               _dptr(state), _stream(stream)))
    return state


def simulate(plan, seed, state, counts, targets, step0, nsteps, *, traj0=0, count_from=0, plain=False,
             waves_per_block=0, traj_per_wave=1, stream=None, record=None):
    """Advance trajectories traj0 .. traj0+ntraj-1 by nsteps (global steps step0..).

    traj_per_wave: trajectories sharing one wavefront's lane passes (1 .. 4).
    record: optional int32 device tensor [r][words]: trajectories 0 .. r-1 of
    the launch OR target 0's indicator bits into it (bit t - count_from)."""
    ntraj = state.shape[0]
    lo = _lib.pbn_launch_opts(int(waves_per_block))
    lo.traj_per_wave = int(traj_per_wave)
    if record is not None:
        lo.record_traj = int(record.shape[0])
        lo.record_words = int(record.shape[1])
        lo.d_record = record.data_ptr()
    fn = lib().pbn_simulate_plain if plain else lib().pbn_simulate
    check(fn(plan.handle, _dptr(plan.device()), int(seed), int(traj0), int(ntraj), int(step0), int(nsteps),
             int(count_from), C.byref(targets), _dptr(state), _dptr(counts), C.byref(lo), _stream(stream)))
    return state, counts


def to_original(plan, state, stream=None):
    import torch
    ntraj = state.shape[0]
    out = torch.zeros((ntraj, (plan.n + 31) // 32), dtype=torch.int32, device="cuda")
    check(lib().pbn_state_to_original(plan.handle, _dptr(plan.device()), _dptr(state), int(ntraj),
                                      _dptr(out), _stream(stream)))
    return out


def unpack_bits(words, n):
    """Host helper: [ntraj, W] int32 words -> uint8 [ntraj, n] node values."""
    w = np.asarray(words).astype(np.uint32)
    bits = ((w[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(np.uint8)
    return bits.reshape(w.shape[0], -1)[:, :n]


# ----------------------------------------------------------------- batches

def _to_device_bytes(obj):
    import torch
    raw = np.frombuffer(C.string_at(C.addressof(obj), C.sizeof(obj)), dtype=np.uint8).copy()
    return torch.from_numpy(raw).to("cuda")


# the most task queues of a batched launch (PBN_BATCH_QUEUES), the words of
# its control block (step0, nsteps, ntasks, reserved, one claim counter per
# queue) and the default queue count: 8 G queues give each group of 32 / G CUs
# of an XCD its own queue; 64 (four CUs a queue) was the fastest of 1 to 256
# on the 512-network batch
BATCH_QUEUES = 64
CTL_WORDS = 4 + BATCH_QUEUES
DEFAULT_QUEUES = 64


def new_ctl(step0=0, nsteps=0):
    """A batch control block on the device with the step window set."""
    import torch
    words = [int(step0), int(nsteps)] + [0] * (CTL_WORDS - 2)
    return torch.tensor(words, dtype=torch.int32, device="cuda")


def batch_schedule(plans_arr, ntraj, wpb, queues=DEFAULT_QUEUES):
    """pbn_batch_tasks: (item of each task, its first trajectory, the
    queues + 1 queue bounds), all uint32 host arrays."""
    ntraj = np.ascontiguousarray(ntraj, dtype=np.uint32)
    nt = C.c_uint32()
    check(lib().pbn_batch_tasks(plans_arr, _ptr(ntraj, C.c_uint32), ntraj.size, int(wpb), int(queues),
                                None, None, None, C.byref(nt)))
    tasks = np.zeros(max(1, nt.value), dtype=np.uint32)
    first = np.zeros(max(1, nt.value), dtype=np.uint32)
    qfirst = np.zeros(int(queues) + 1, dtype=np.uint32)
    check(lib().pbn_batch_tasks(plans_arr, _ptr(ntraj, C.c_uint32), ntraj.size, int(wpb), int(queues),
                                _ptr(tasks, C.c_uint32), _ptr(first, C.c_uint32), _ptr(qfirst, C.c_uint32),
                                C.byref(nt)))
    return tasks[:nt.value], first[:nt.value], qfirst


class Batch:
    """Many networks advanced by one persistent launch (pbn_batch_launch).

    items: list of (plan, seed, ntraj, target_sets); every trajectory of every
    network shares the device step window held in the control block.
    queues: task queues of the launch (1 .. BATCH_QUEUES); 1 puts every task
    in one queue.  waves_per_traj: W > 1 advances each trajectory with W
    waves of one workgroup (one trajectory per task: waves_per_block is then
    1); the results do not depend on it.
    """

    def __init__(self, items, count_from=0, waves_per_block=4, queues=DEFAULT_QUEUES, waves_per_traj=1):
        import torch
        self.plans = [it[0] for it in items]
        self.wpt = int(waves_per_traj)
        self.wpb = 1 if self.wpt > 1 else int(waves_per_block)
        self.targets, self.states, self.counts, self._tg_dev = [], [], [], []
        works = (_lib.pbn_work * len(items))()
        for k, (plan, seed, ntraj, target_sets) in enumerate(items):
            tg = plan.targets(target_sets)
            tg_dev = _to_device_bytes(tg)
            state = new_state(plan, ntraj)
            counts = new_counts(tg.ntargets, ntraj)
            self.targets.append(tg)
            self._tg_dev.append(tg_dev)
            self.states.append(state)
            self.counts.append(counts)
            works[k] = _lib.pbn_work(plan.device().data_ptr(), tg_dev.data_ptr(), state.data_ptr(),
                                     counts.data_ptr(), int(seed), 0, int(ntraj), int(count_from), 0)
            self.states[k] = state
        self.seeds = [int(it[1]) for it in items]
        self._works = works
        self.items_dev = _to_device_bytes(works)
        self._plan_arr = (C.c_void_p * len(items))(*[p.handle.value for p in self.plans])
        ntraj = np.asarray([it[2] for it in items], dtype=np.uint32)
        self._ntraj = ntraj
        self.nqueues = int(queues)
        tasks, first, self.queue_first = batch_schedule(self._plan_arr, ntraj, self.wpb, self.nqueues)
        self.ntasks = int(tasks.size)
        pad = np.zeros(1, dtype=np.uint32)    # device arrays of at least one element
        self.tasks_dev = torch.from_numpy((tasks if tasks.size else pad).astype(np.int32)).to("cuda")
        self.first_dev = torch.from_numpy((first if first.size else pad).astype(np.int32)).to("cuda")
        self.ctl = new_ctl()

    def init_states(self, stream=None):
        for plan, seed, state in zip(self.plans, self.seeds, self.states):
            check(lib().pbn_state_init(plan.handle, _dptr(plan.device()), seed, 0, state.shape[0],
                                       _dptr(state), _stream(stream)))

    def set_window(self, step0, nsteps):
        self.ctl.copy_(new_ctl(step0, nsteps))

    def step0(self):
        """The device-held first step of the next launch's window."""
        return int(self.ctl[0].item())

    def _args(self):
        return (self._plan_arr, len(self.plans), _dptr(self.items_dev), _dptr(self.tasks_dev),
                _dptr(self.first_dev), self.ntasks, _ptr(self.queue_first, C.c_uint32), self.nqueues,
                _dptr(self.ctl), self.wpb, self.wpt)

    def launch(self, stream=None):
        check(lib().pbn_batch_launch(*self._args(), _stream(stream)))

    def launch_noalloc(self, step0, nsteps, stream=None):
        """pbn_batch_launch_noalloc: the step window by value, the schedule in
        the library's device array (items in list order)."""
        check(lib().pbn_batch_launch_noalloc(self._plan_arr, _ptr(self._ntraj, C.c_uint32), len(self.plans),
                                             _dptr(self.items_dev), int(step0), int(nsteps), self.wpb,
                                             _stream(stream)))

    def graph(self, passes):
        g = C.c_void_p()
        check(lib().pbn_batch_graph_create(*self._args(), int(passes), C.byref(g)))
        return Graph(g)


class Graph:
    def __init__(self, handle):
        self.handle = handle
        self._libref = lib()

    def launch(self, stream=None):
        check(lib().pbn_graph_launch(self.handle, _stream(stream)))

    def __del__(self):
        # the library object is held by the instance: module globals may
        # already be gone when the interpreter shuts down
        h, L = getattr(self, "handle", None), getattr(self, "_libref", None)
        if h is not None and L is not None:
            L.pbn_graph_destroy(h)
            self.handle = None
