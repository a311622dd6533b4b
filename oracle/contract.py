"""Random-number contract shared (as a written specification, not as code) by the
oracle and the GPU library.

The paper leaves the generator, the sampling of perturbations and the
representation of selection probabilities unspecified (Section 2.2 uses alias
tables of doubles; Algorithms 1 and 2 draw `rand()`).  This project fixes one
reproducible reading so that a trajectory is a pure function of
(seed, trajectory id), independent of how the simulator is organised:

* Draws come from Philox4x32-10 with key = seed and counter
  (trajectory, step, index, stream); streams INIT = 1, PERT = 2, SEL = 3.
* Initial state: bit i of s(0) is bit (i mod 32) of output word ((i >> 5) & 3)
  of the INIT call with index i >> 7 and step 0.
* Perturbation rate p becomes the table Q[h] = floor(v_h * 2^64), h = 1..n,
  with v_0 = 1 and v_{h+1} = v_h * (1 - p) in IEEE double (one rounding per
  product).  Q[h] / 2^64 is the probability that h consecutive nodes are all
  unperturbed, so the number C of unperturbed nodes before the next perturbed
  one is drawn from a 64-bit uniform u as C = #{h in 1..n : Q[h] > u}
  (geometric skip sampling of the iid Bernoulli(p) vector gamma of Eq. 1).
* Selection probabilities c_0..c_{l-1} of a node become integer thresholds
  CUM[m] = min(2^32, floor(S_m * 2^32 + 1/2)), m = 0..l-2, where S_m is
  the left-to-right double sum c_0 + ... + c_m; a 32-bit uniform u selects
  predictor j = #{m : u >= CUM[m]}.  A threshold of 2^32 is never reached, so
  predictors whose selection probability follows a partial sum of 1 are never
  chosen (Section 2.1: a predictor is chosen with its selection probability,
  and zero means never).
* Node i with l(i) >= 2 takes its uniform from word (r & 3) of the SEL call
  with index r >> 2, where r is the rank of i among all nodes with two or more
  predictors, in node-id order, in the full network.  Ranks do not depend on
  any reduction or grouping, so every simulator layout sees the same draws.
"""
import numpy as np

from .philox import philox4x32, key_of_seed

INIT, PERT, SEL = 1, 2, 3


def perturbation_table(n, p):
    """Q[0..n] as Python ints; Q[0] = 2^64 is the certain event and is never compared."""
    q = 1.0 - float(p)
    v = 1.0
    out = [1 << 64]
    for _ in range(n):
        v = v * q                       # one IEEE double product per step
        out.append(int(np.floor(np.ldexp(v, 64))))
    return out


def selection_thresholds(probs):
    """CUM[0..l-2] for one node's selection probabilities, as Python ints."""
    s = 0.0
    out = []
    for m in range(len(probs) - 1):
        s = s + float(probs[m])         # left-to-right double sum
        out.append(min(1 << 32, int(np.floor(np.ldexp(s, 32) + 0.5))))
    return out


def multi_ranks(net):
    """rank[i] among nodes with >= 2 predictors (node-id order), or -1."""
    nfn = np.diff(net["fn_off"])
    rank = np.full(net["n"], -1, dtype=np.int64)
    multi = np.nonzero(nfn >= 2)[0]
    rank[multi] = np.arange(multi.size)
    return rank


def draw(seed, traj, step, index, stream):
    """Four output words (uint64 arrays of 32-bit values) of one keyed call."""
    k0, k1 = key_of_seed(seed)
    return philox4x32(traj, step, index, stream, k0, k1)


def initial_state(net, seed, traj):
    """s(0) for trajectories `traj` (1-d array): uint8 array (len(traj), n)."""
    n = net["n"]
    traj = np.asarray(traj, dtype=np.uint64)
    s = np.zeros((traj.size, n), dtype=np.uint8)
    for blk in range((n + 127) // 128):
        words = draw(seed, traj, 0, blk, INIT)
        for i in range(blk * 128, min(n, blk * 128 + 128)):
            w = words[(i >> 5) & 3]
            s[:, i] = ((w >> np.uint64(i & 31)) & np.uint64(1)).astype(np.uint8)
    return s
