"""Exact steady state of a small PBN from its 2^n x 2^n transition matrix.

Equation 1 (Section 2.1) gives the one-step law directly:

  P(s -> s') = sum over gamma != 0 of p^|gamma| (1-p)^(n-|gamma|) [s' = s XOR gamma]
             + (1-p)^n * prod_i P(f_i(s) = s'_i),

with P(f_i(s) = 1) = sum_j c_j^(i) [f_j^(i)(s) = 1] (independent selection per
node).  Perturbations make the chain irreducible and aperiodic, so the limiting
distribution is unique (Section 2.1).  Probabilities here are the exact doubles
of the network, not the integer-quantised ones of the simulation contract; the
difference (about 2^-32 per threshold, 2^-53 per perturbation step) is far
below any statistical tolerance used with this module.

States are integers: bit i is node i.
"""
import numpy as np


def node_on_probability(net):
    """q[i, s] = P(f_i(s) = 1) for every node i and state s (n <= 12)."""
    n = int(net["n"])
    S = np.arange(1 << n, dtype=np.int64)
    q = np.zeros((n, S.size))
    for i in range(n):
        for f in range(int(net["fn_off"][i]), int(net["fn_off"][i + 1])):
            pa = net["parents"][net["par_off"][f]:net["par_off"][f + 1]].astype(np.int64)
            words = net["tt"][net["tt_off"][f]:net["tt_off"][f + 1]]
            index = np.zeros(S.size, dtype=np.int64)
            for k, par in enumerate(pa):
                index |= ((S >> par) & 1) << k
            out = np.array([(int(words[j // 64]) >> (j % 64)) & 1 for j in index], dtype=float)
            q[i] += float(net["sel_prob"][f]) * out
    return q


def transition_matrix(net):
    """Dense row-stochastic matrix P[s, s'] of Eq. 1."""
    n = int(net["n"])
    if n > 12:
        raise ValueError("exact matrix only for n <= 12")
    p = float(net["p"])
    N = 1 << n
    S = np.arange(N, dtype=np.int64)
    flips = S[:, None] ^ S[None, :]
    pop = np.zeros_like(flips)
    for b in range(n):
        pop += (flips >> b) & 1
    P = np.where(pop > 0, p ** pop * (1.0 - p) ** (n - pop), 0.0)
    q = node_on_probability(net)
    F = np.ones((N, N))
    for i in range(n):
        bit = (S[None, :] >> i) & 1                  # s'_i
        F *= np.where(bit == 1, q[i][:, None], 1.0 - q[i][:, None])
    P += (1.0 - p) ** n * F
    return P


def steady_state(net, tol=1e-15, max_iter=200000):
    """Limiting distribution by the power method, cross-checked by a linear solve."""
    P = transition_matrix(net)
    N = P.shape[0]
    pi = np.full(N, 1.0 / N)
    for _ in range(max_iter):
        nxt = pi @ P
        nxt /= nxt.sum()
        if np.abs(nxt - pi).sum() < tol:
            pi = nxt
            break
        pi = nxt
    A = P.T - np.eye(N)
    A[-1, :] = 1.0
    b = np.zeros(N)
    b[-1] = 1.0
    direct = np.linalg.solve(A, b)
    if np.abs(direct - pi).max() > 1e-9:
        raise RuntimeError("power method and linear solve disagree")
    return pi


def target_probability(pi, target):
    """P(state matches every (node, value) of the target) under distribution pi."""
    S = np.arange(pi.size, dtype=np.int64)
    ok = np.ones(pi.size, dtype=bool)
    for node, val in target:
        ok &= ((S >> node) & 1) == val
    return float(pi[ok].sum())
