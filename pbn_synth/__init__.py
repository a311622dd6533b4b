"""Seeded synthetic probabilistic Boolean networks (PBNs) and run configurations.

This module only *draws* inputs: network structure, predictor truth tables,
selection probabilities, perturbation rate and query targets.  It holds none of
the simulation method's arithmetic (no random-number contract, no quantisation,
no state update), so both the CPU oracle and the GPU library can consume it.

A network is a plain dict of numpy arrays in the CSR form the C ABI takes
(the PBN G(X, F) of Section 2.1: each node has l(i) predictor functions with
selection probabilities summing to one, each function reads its own parent
subset, and every node flips with probability p):

    n         int       number of nodes
    p         float     perturbation rate
    fn_off    uint32[n+1]   functions of node i are fn_off[i] .. fn_off[i+1]-1
    sel_prob  float64[NF]   selection probability of each function
    par_off   uint32[NF+1]  parents of function f are parents[par_off[f]:par_off[f+1]]
    parents   uint32[...]   parent node ids; parent k is bit k of the truth-table index
    tt_off    uint32[NF+1]  truth table of f is tt[tt_off[f]:tt_off[f+1]] (64-bit words)
    tt        uint64[...]   LSB-first: the output for index j is bit (j % 64) of word j // 64

The paper's benchmark networks are not available, so these generators stand in
for them with the shapes the evaluation describes (leaf share 0-90%, density
1-8.1, sizes 20-1000; Section 4.1) and the configurations of the build plan.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "assemble", "random_pbn", "tiny_c1", "medium_c2", "large_c3", "batch_c4",
    "served_c5", "density", "network_sha256", "RunConfig", "config",
]


def assemble(n, p, functions):
    """Build the CSR dict from a per-node list of functions.

    ``functions[i]`` is a list of ``(prob, parents, tt_bits)`` where ``tt_bits``
    is a 0/1 sequence of length ``2**len(parents)``.
    """
    fn_off = [0]
    sel, par_off, pars, tt_off, tt = [], [0], [], [0], []
    for i in range(n):
        fl = functions[i]
        if not fl:
            raise ValueError(f"node {i} has no predictor function")
        for prob, parents, bits in fl:
            bits = np.asarray(bits, dtype=np.uint64)
            if bits.size != (1 << len(parents)):
                raise ValueError("truth table length must be 2**len(parents)")
            nwords = max(1, bits.size // 64)
            words = np.zeros(nwords, dtype=np.uint64)
            for j in np.nonzero(bits)[0]:
                words[j // 64] |= np.uint64(1) << np.uint64(j % 64)
            sel.append(float(prob))
            pars.extend(int(x) for x in parents)
            par_off.append(len(pars))
            tt.extend(words.tolist())
            tt_off.append(len(tt))
        fn_off.append(len(sel))
    return {
        "n": int(n),
        "p": float(p),
        "fn_off": np.asarray(fn_off, dtype=np.uint32),
        "sel_prob": np.asarray(sel, dtype=np.float64),
        "par_off": np.asarray(par_off, dtype=np.uint32),
        "parents": np.asarray(pars, dtype=np.uint32),
        "tt_off": np.asarray(tt_off, dtype=np.uint32),
        "tt": np.asarray(tt, dtype=np.uint64),
    }


def _draw_table(rng, k):
    return rng.integers(0, 2, size=1 << k, dtype=np.int64)


def random_pbn(n, p, seed, *, nfn, nparents, leaf_frac=0.0, self_loops=True):
    """Random PBN generator used by every configuration.

    ``nfn(rng)`` and ``nparents(rng)`` draw the number of predictor functions of
    a node and the number of parents of a function.  ``leaf_frac`` designates
    that share of nodes as sinks: they are excluded from every parent pool, so
    no function reads them.  Parents are drawn uniformly without replacement
    from the pool; truth-table bits are iid Bernoulli(0.5); selection
    probabilities are Dirichlet(1, ..., 1).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nleaf = int(round(leaf_frac * n))
    leaves = np.sort(rng.choice(n, size=nleaf, replace=False)) if nleaf else np.zeros(0, np.int64)
    is_leaf = np.zeros(n, dtype=bool)
    is_leaf[leaves] = True
    pool_all = np.nonzero(~is_leaf)[0]
    functions = []
    for i in range(n):
        l = int(nfn(rng))
        probs = rng.dirichlet(np.ones(l)) if l > 1 else np.ones(1)
        fl = []
        for j in range(l):
            pool = pool_all if self_loops else pool_all[pool_all != i]
            k = min(int(nparents(rng)), pool.size)
            parents = rng.choice(pool, size=k, replace=False)
            fl.append((probs[j], parents.tolist(), _draw_table(rng, k)))
        functions.append(fl)
    net = assemble(n, p, functions)
    net["designated_leaves"] = leaves.astype(np.uint32)
    return net


def _uniform_int(lo, hi):
    return lambda rng: rng.integers(lo, hi + 1)


def _trunc_geometric(rho, kmax):
    w = (1.0 - rho) ** np.arange(kmax)
    pmf = w / w.sum()
    return lambda rng: 1 + rng.choice(kmax, p=pmf)


def tiny_c1(seed=1001):
    """n = 10, two predictors per node (Dirichlet(1,1)), three parents each, p = 0.01."""
    return random_pbn(10, 0.01, seed, nfn=lambda r: 2, nparents=lambda r: 3)


def medium_c2(n=100, p=1e-3, seed=1002, leaf_frac=0.15):
    """1-4 predictors per node, 2-5 parents per predictor, 15% designated leaves."""
    return random_pbn(n, p, seed, nfn=_uniform_int(1, 4), nparents=_uniform_int(2, 5),
                      leaf_frac=leaf_frac)


def large_c3(n=2000, p=1e-4, seed=1003):
    """In-degree 1-6 from a truncated geometric (mean 2.5); 90% single predictor, 10% with 2-3."""
    one = lambda rng: 1 if rng.random() < 0.9 else int(rng.integers(2, 4))
    return random_pbn(n, p, seed, nfn=one, nparents=_trunc_geometric(0.30999, 6))


def with_detached_modules(core, modules, size, seed, nparents=(2, 4)):
    """The core network plus `modules` extra regions of `size` nodes each.

    A module node reads 2-4 parents drawn from its own module and the core, so
    every module contains feedback cycles (its nodes are parents of one
    another) while no core node ever reads a module node: nothing in the core
    depends on the modules.  Each extra node has one predictor (probability 1)
    with an iid Bernoulli(0.5) truth table.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n0 = int(core["n"])
    fo, po, par, sel = core["fn_off"], core["par_off"], core["parents"], core["sel_prob"]
    to, tt = core["tt_off"], core["tt"]
    functions = []
    for i in range(n0):
        fl = []
        for f in range(int(fo[i]), int(fo[i + 1])):
            k = int(po[f + 1] - po[f])
            words = tt[int(to[f]):int(to[f + 1])]
            bits = [(int(words[x // 64]) >> (x % 64)) & 1 for x in range(1 << k)]
            fl.append((float(sel[f]), [int(v) for v in par[int(po[f]):int(po[f + 1])]], bits))
        functions.append(fl)
    for m in range(modules):
        base = n0 + m * size
        pool = np.concatenate([np.arange(n0), np.arange(base, base + size)])
        for i in range(size):
            k = int(rng.integers(nparents[0], nparents[1] + 1))
            own = int(rng.integers(base, base + size))          # at least one parent inside the module
            rest = rng.choice(pool[pool != own], size=k - 1, replace=False)
            functions.append([(1.0, [own] + rest.tolist(), _draw_table(rng, k))])
    net = assemble(n0 + modules * size, core["p"], functions)
    net["designated_leaves"] = np.asarray(core.get("designated_leaves", []), dtype=np.uint32)
    return net


def interleaved_cone(n_core=100, n_other=400, p=2e-3, seed=19):
    """A core of n_core nodes whose predictors read only core nodes, and
    n_other nodes that read the core and one another, their ids interleaved
    at random (ids 0, 1, 2 are in the core).  Every node has 2-3 predictors of
    1-3 parents.  The cone of influence of core targets lies in the core,
    while the core's multi-predictor nodes are spread over the whole rank
    order, so their selection-draw blocks are many."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = n_core + n_other
    rest = rng.permutation(np.arange(3, n))
    core = np.sort(np.concatenate([np.arange(3), rest[:n_core - 3]]))
    is_core = np.zeros(n, dtype=bool)
    is_core[core] = True
    everyone = np.arange(n)
    functions = []
    for i in range(n):
        l = int(rng.integers(2, 4))
        probs = rng.dirichlet(np.ones(l))
        pool = core if is_core[i] else everyone
        fl = []
        for j in range(l):
            k = int(rng.integers(1, 4))
            parents = rng.choice(pool, size=k, replace=False)
            fl.append((probs[j], parents.tolist(), _draw_table(rng, k)))
        functions.append(fl)
    net = assemble(n, p, functions)
    net["designated_leaves"] = np.zeros(0, dtype=np.uint32)
    return net


def planner_population(count, seed):
    """Networks spread over the ranges of the paper's experiments (Section
    4.1): n ~ U[100, 1500], leaf fraction ~ U[0, 0.9], 1..lmax predictors of
    1..kmax parents (lmax ~ U{1..4}, kmax ~ U{1..6}), p = 1e-3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(count):
        n = int(rng.integers(100, 1501))
        leaf = float(rng.uniform(0.0, 0.9))
        lmax, kmax = int(rng.integers(1, 5)), int(rng.integers(1, 7))
        out.append(random_pbn(n, 1e-3, seed * 1000 + k, nfn=_uniform_int(1, lmax), nparents=_uniform_int(1, kmax),
                              leaf_frac=leaf))
    return out


def batch_c4(count=512, seed=1004):
    """Uneven batch: n ~ U[20, 1500] with the medium generator, p in {1e-3, 1e-4}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(20, 1501, size=count)
    ps = rng.choice([1e-3, 1e-4], size=count)
    return [medium_c2(int(sizes[k]), float(ps[k]), seed * 1000 + k) for k in range(count)]


def batch_c4_network(k, count=512, seed=1004):
    """Network k of batch_c4(count, seed), generated alone."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(20, 1501, size=count)
    ps = rng.choice([1e-3, 1e-4], size=count)
    return medium_c2(int(sizes[k]), float(ps[k]), seed * 1000 + k)


def served_c5(count=64, seed=1005):
    """Resident networks for the query service: n ~ U[50, 3000], p in {1e-3, 1e-4}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(50, 3001, size=count)
    ps = rng.choice([1e-3, 1e-4], size=count)
    return [medium_c2(int(sizes[k]), float(ps[k]), seed * 1000 + k) for k in range(count)]


def density(net):
    """Density D(G) = (1/n) * sum over all predictor functions of their parent count (Section 2.1)."""
    return float(np.diff(net["par_off"]).sum()) / net["n"]


def network_sha256(net):
    """Canonical digest of a network (fixed key order, little-endian arrays)."""
    h = hashlib.sha256()
    h.update(np.asarray([net["n"]], dtype="<u8").tobytes())
    h.update(np.asarray([net["p"]], dtype="<f8").tobytes())
    for key in ("fn_off", "sel_prob", "par_off", "parents", "tt_off", "tt"):
        h.update(key.encode())
        h.update(np.ascontiguousarray(net[key]).astype(net[key].dtype.newbyteorder("<")).tobytes())
    return h.hexdigest()


def non_leaf_targets(net, count=3):
    """The `count` smallest node ids that are not designated leaves (all required ON)."""
    leaves = set(int(x) for x in net.get("designated_leaves", []))
    nodes = [i for i in range(net["n"]) if i not in leaves][:count]
    return [(i, 1) for i in nodes]


def random_query_targets(rng, net, kmin=1, kmax=5):
    """1-5 random non-leaf nodes with a random ON/OFF pattern (served queries)."""
    leaves = set(int(x) for x in net.get("designated_leaves", []))
    pool = np.asarray([i for i in range(net["n"]) if i not in leaves])
    k = int(rng.integers(kmin, kmax + 1))
    nodes = np.sort(rng.choice(pool, size=k, replace=False))
    vals = rng.integers(0, 2, size=k)
    return [(int(a), int(b)) for a, b in zip(nodes, vals)]


@dataclass
class RunConfig:
    """One simulation workload: network, trajectories, steps, burn-in, targets, seed."""
    name: str
    net: dict
    ntraj: int
    steps: int
    burn_in: int
    targets: list = field(default_factory=list)   # list of target sets; each a list of (node, value)
    seed: int = 1


def config(name):
    """The workloads of the build plan (C1 tiny, C2 medium, C3 large; C2X the
    medium network with detached modules)."""
    if name == "C1":
        net = tiny_c1()
        return RunConfig("C1", net, ntraj=1, steps=10**6, burn_in=0, targets=[[(0, 1), (1, 1)]], seed=1)
    if name == "C2":
        net = medium_c2()
        return RunConfig("C2", net, ntraj=4096, steps=10**6, burn_in=0,
                         targets=[non_leaf_targets(net)], seed=2)
    if name == "C3":
        net = large_c3()
        return RunConfig("C3", net, ntraj=65536, steps=10**5, burn_in=10**4,
                         targets=[non_leaf_targets(net)], seed=3)
    if name == "C2X":
        # the medium network plus four detached 25-node feedback modules that
        # no core node reads (the workload of the cone-of-influence reduction)
        core = medium_c2()
        net = with_detached_modules(core, 4, 25, seed=1006)
        return RunConfig("C2X", net, ntraj=4096, steps=10**6, burn_in=0,
                         targets=[non_leaf_targets(core)], seed=6)
    raise KeyError(name)
