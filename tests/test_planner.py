"""The pre-processing-aware planner (Equation 7's model form, Table 1's
sample-size trade-off): CPU checks of its pieces."""
import math

import numpy as np
import pytest

import pbn_synth as ps
from oracle import structure
from paper_1605_00854_amd import planner


def test_fit_recovers_known_coefficients():
    rng = np.random.default_rng(3)
    x1 = rng.uniform(0, 0.9, 40)
    x2 = rng.uniform(1, 8, 40)
    b = (2.89, 2.71, 2.40, -1.65, 0.71)             # the paper's printed coefficients as a test model
    y = b[0] + b[1] * x1 + b[2] * x1 ** 2 + b[3] * x2 + b[4] * x2 ** 2
    got, r2 = planner.fit(x1, x2, y)
    assert np.allclose(got, b, rtol=1e-9, atol=1e-9) and r2 == pytest.approx(1.0)
    assert planner.cross_validated_r2(x1, x2, y) == pytest.approx(1.0)
    assert planner.predict(0.5, 3.0, b) == pytest.approx(2.89 + 2.71 * 0.5 + 2.40 * 0.25 - 1.65 * 3 + 0.71 * 9)


def test_per_pass_fit_recovers_known_coefficients():
    rng = np.random.default_rng(4)
    x1 = rng.uniform(0, 0.9, 40)
    x2 = rng.uniform(1, 8, 40)
    ratio = rng.choice([1.0, 1.5, 2.0, 3.0], 40)
    b = (1.1, 0.3, -0.2, 0.05, -0.004)
    y = ratio * (b[0] + b[1] * x1 + b[2] * x1 ** 2 + b[3] * x2 + b[4] * x2 ** 2)
    got, r2 = planner.fit_per_pass(x1, x2, ratio, y)
    assert np.allclose(got, b, rtol=1e-9, atol=1e-9) and r2 == pytest.approx(1.0)
    assert planner.cross_validated_r2(x1, x2, y, ratio=ratio) == pytest.approx(1.0)
    # the plain form cannot follow the ratio's steps
    assert planner.fit(x1, x2, y)[1] < 0.99


def test_lane_pass_ratio_counts_64_lane_passes():
    net = ps.medium_c2(n=200, seed=6, leaf_frac=0.5)
    interest = [a for a, _ in ps.non_leaf_targets(net, 3)]
    kept = 200 - len(structure.leaf_nodes(net, interest))
    assert planner.lane_pass_ratio(net, interest) == pytest.approx(math.ceil(200 / 64) / math.ceil(kept / 64))


def test_features_are_leaf_fraction_and_density():
    net = ps.medium_c2(n=120, seed=5)
    interest = [a for a, _ in ps.non_leaf_targets(net, 3)]
    x1, x2, prep = planner.features(net, interest)
    assert x1 == pytest.approx(len(structure.leaf_nodes(net, interest)) / 120)
    parents = sum(int(net["par_off"][f + 1] - net["par_off"][f]) for f in range(len(net["sel_prob"])))
    assert x2 == pytest.approx(parents / 120) and x2 == pytest.approx(ps.density(net))
    assert prep >= 0


def test_choice_follows_the_sample_size():
    # a model predicting a 4x speedup of the tuned plan (the reduction alone: 1 / (1 - 0.6) = 2.5x)
    args = dict(plain_rate=1e11, x1=0.6, x2=2.0, prep_reduction=0.01, n_candidates=30, probe_work=2e9,
                coeffs=(4.0, 0.0, 0.0, 0.0, 0.0))
    small = planner.predicted_times(1e6, **args)
    mid = planner.predicted_times(1e11, **args)
    big = planner.predicted_times(1e15, **args)
    assert min(small, key=small.get) == "plain"          # preparation costs more than it saves
    assert min(mid, key=mid.get) == "reduction"          # host preparation only
    assert min(big, key=big.get) == "tuned"              # probes amortised
    # the reduction's rate follows the kept nodes
    t = planner.predicted_times(1e12, **args)
    assert t["reduction"] == pytest.approx(0.01 + 1e12 / (1e11 / 0.4))


def test_refit_model_predicts_at_least_no_slowdown_in_range():
    for x1 in (0.0, 0.45, 0.9):
        for x2 in (1.0, 4.0, 8.0):
            assert planner.predict(x1, x2) > 0.5
            assert math.isfinite(planner.predict(x1, x2))
