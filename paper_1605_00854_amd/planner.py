"""Pre-processing-aware planner: the performance prediction of Section 4.1
(Equation 7) and the sample-size trade-off of Table 1.

The paper fits the speedup of its method over the plain simulation with
y = b1 + b2 x1 + b3 x1^2 + b4 x2 + b5 x2^2 (x1 the percentage of leaves, x2
the density D(G) of Section 2.1) over its 2307 networks, and shows that the
pre-processing pays off only above some sample size.  Here the same model form
is refit to this device's measured speedups of the autotuned plan over the
plain kernel on synthetic networks (the paper's normalisation of x1 is not
stated: x1 is the leaf fraction in [0, 1]), and `choose` picks, for a requested
number of trajectory-steps, the preparation with the smallest predicted total
time: the plain kernel (no preparation), the leaf reduction (host preparation
only), or the autotuned plan (host preparations plus device probe runs).
"""
import time

import numpy as np

from . import api, autotune

# Equation 7's form refit on MI355X: 72 synthetic networks (n 100-1500, leaf
# fraction 0.06-0.94, density 1.0-8.8), speedup of the autotuned plan over the
# plain kernel at 2048 trajectories (bench.py --planner-fit 72): R^2 0.56,
# 10-fold cross-validated 0.49, 24 held-out networks 0.68.
COEFFS = (0.589427, 0.991735, 0.975340, 0.220935, -0.018722)


def density(net):
    """D(G) = (1/n) sum over all predictor functions of their parent count."""
    return float(np.diff(np.asarray(net["par_off"], dtype=np.int64)).sum()) / int(net["n"])


def features(net, interest):
    """(leaf fraction x1, density x2, host preparation seconds of the reduction plan)."""
    t0 = time.perf_counter()
    plan = api.Plan(net, interest=interest, reduce=1, group=0)
    prep = time.perf_counter() - t0
    return 1.0 - plan.info["n_kept"] / int(net["n"]), density(net), prep


def lane_pass_ratio(net, interest):
    """Lane passes of the plain plan over those of the leaf-reduced plan: the
    step kernel's work comes in whole 64-lane passes, so a reduction pays in
    steps of ceil(n / 64) / ceil(n' / 64), which x1 alone cannot show."""
    plain = api.Plan(net, interest=interest, reduce=0, group=0)
    red = api.Plan(net, interest=interest, reduce=1, group=0)
    return plain.info["n_passes"] / max(1, red.info["n_passes"])


def design(x1, x2):
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    return np.stack([np.ones_like(x1), x1, x1 * x1, x2, x2 * x2], axis=-1)


def predict(x1, x2, coeffs=COEFFS):
    return design(x1, x2) @ np.asarray(coeffs, dtype=np.float64)


def fit(x1, x2, y):
    """Least-squares coefficients of Equation 7's form and the fraction of the
    variance they explain (R^2)."""
    A = design(x1, x2)
    y = np.asarray(y, dtype=np.float64)
    b, *_ = np.linalg.lstsq(A, y, rcond=None)
    res = y - A @ b
    tot = y - y.mean()
    r2 = 1.0 - float(res @ res) / float(tot @ tot) if float(tot @ tot) > 0 else 1.0
    return tuple(float(v) for v in b), r2


def fit_per_pass(x1, x2, ratio, y):
    """Equation 7's form fit to the speedup per lane-pass ratio (y / ratio),
    the prediction being ratio times the form; returns the coefficients and
    the R^2 of that prediction on y itself."""
    ratio = np.asarray(ratio, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    b, _ = fit(x1, x2, y / ratio)
    res = y - ratio * predict(x1, x2, b)
    tot = y - y.mean()
    return b, 1.0 - float(res @ res) / float(tot @ tot) if float(tot @ tot) > 0 else 1.0


def cross_validated_r2(x1, x2, y, folds=10, seed=0, ratio=None):
    """R^2 of out-of-fold predictions (the paper validates its fit with 10
    folds); with `ratio`, of the per-lane-pass form (fit_per_pass)."""
    """R^2 of out-of-fold predictions (the paper validates its fit with 10 folds)."""
    x1, x2, y = (np.asarray(v, dtype=np.float64) for v in (x1, x2, y))
    r = np.ones_like(y) if ratio is None else np.asarray(ratio, dtype=np.float64)
    idx = np.random.default_rng(seed).permutation(y.size)
    pred = np.empty_like(y)
    for f in range(folds):
        test = idx[f::folds]
        train = np.setdiff1d(idx, test)
        b, _ = fit(x1[train], x2[train], y[train] / r[train])
        pred[test] = r[test] * predict(x1[test], x2[test], b)
    res, tot = y - pred, y - y.mean()
    return 1.0 - float(res @ res) / float(tot @ tot)


def predicted_times(work, plain_rate, x1, x2, prep_reduction, n_candidates, probe_work, coeffs=COEFFS):
    """Predicted seconds of each preparation for `work` node-updates.

    plain: work / plain_rate.  reduction: its host preparation, then a rate
    scaled by n / n_kept = 1 / (1 - x1) (the kernel's work follows the kept
    nodes).  tuned: every candidate's host preparation and device probes
    (probe_work node-updates each, at the plain rate), then the rate scaled by
    the model's speedup (never below the reduction's)."""
    s_red = 1.0 / max(1e-9, 1.0 - x1)
    s_tuned = max(float(predict(x1, x2, coeffs)), s_red)
    return {
        "plain": work / plain_rate,
        "reduction": prep_reduction + work / (plain_rate * s_red),
        "tuned": n_candidates * (prep_reduction + probe_work / plain_rate) + work / (plain_rate * s_tuned),
    }


def choose(net, interest, target_sets, ntraj, steps, *, seed=1, coeffs=COEFFS, plain_rate=None, quick=True,
           probe_steps=2000):
    """Pick the preparation for `ntraj` trajectories of `steps` steps.

    Returns (plan options or None for "run the autotuner", waves per block,
    details).  The plain rate is measured with one short probe unless given."""
    import torch
    n = int(net["n"])
    x1, x2, prep = features(net, interest)
    if plain_rate is None:
        plan = api.Plan(net, interest=interest, reduce=0, group=0)
        tg = plan.targets(target_sets)
        dt = autotune._probe(torch, plan, tg, seed, ntraj, probe_steps, 4, True)
        plain_rate = ntraj * probe_steps * n / dt
    ncand = len(autotune.candidates(quick)) * 3
    t = predicted_times(float(ntraj) * steps * n, plain_rate, x1, x2, prep, ncand, float(ntraj) * probe_steps * n,
                        coeffs)
    pick = min(t, key=t.get)
    opts = {"plain": dict(reduce=0, group=0), "reduction": dict(reduce=1, group=0), "tuned": None}[pick]
    return opts, 4, {"choice": pick, "predicted_seconds": t, "leaf_fraction": x1, "density": x2,
                     "plain_rate": plain_rate, "predicted_speedup": float(predict(x1, x2, coeffs))}
