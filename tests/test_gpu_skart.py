"""GPU: the Skart stopping rule on one trajectory (pbn_skart_run).

* On C1 the driver's recorded sequence is the oracle's trajectory (prefix),
  its final analysis equals the oracle's Skart run on the same bits (every
  decision, and the interval to 1e-9), it stops exactly where the procedure
  finishes, and its estimate lies within the precision of the exact steady
  state (99.9 % gate).
* On a reduced and grouped plan of a medium network the driver's analysis is
  again the oracle's on the recorded bits.
* A limit below what the procedure asks for returns PBN_ERANGE with the
  request filled in.
"""
import sys

import numpy as np
import pytest

import pbn_synth as ps
from oracle import exact
from oracle import simulate as osim
from oracle import skart as osk

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1605_00854_amd import _lib, api  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check_against_oracle(res, bits, r):
    want = osk.skart(bits.astype(np.float64), r)
    assert want["done"] and bool(res["done"])
    assert res["n_required"] == want["n_required"] == res["steps"]
    assert (res["batch_size"], res["batch_count"], res["failures"]) == (want["m"], want["k"], want["b"])
    assert (res["spacer"], res["warmup"], res["ci_batches"], res["ci_batch_size"]) == (
        want["d"], want["warmup"], want["k_ci"], want["m_ci"])
    for key in ("p_hat", "lower", "upper", "half_width", "skewness", "lag1", "ar_factor"):
        assert res[key] == pytest.approx(want[key], rel=1e-9, abs=1e-12), key
    assert res["half_width"] <= r


def test_skart_driver_on_c1():
    cfg = ps.config("C1")
    net = cfg.net
    plan = api.Plan(net, interest=[0, 1], reduce=0, group=0)
    r = 0.005
    say("[gpu] skart_run C1 r=0.005")
    res, record = api.skart_run(plan, cfg.seed, cfg.targets, r, max_steps=1 << 23)
    assert res["status"] == 0, res
    n = res["steps"]
    bits = api.unpack_record(record.cpu().numpy(), n)
    pre = min(n, 4000)
    ref = osim.run(net, cfg.seed, np.arange(1), pre, targets=cfg.targets, indicators=True)
    assert np.array_equal(bits[:pre], ref["z"][0])
    check_against_oracle(res, bits, r)
    pi = exact.target_probability(exact.steady_state(net), cfg.targets[0])
    assert abs(res["p_hat"] - pi) < r * 3.29 / 1.96, (res, pi)


def test_skart_driver_on_grouped_plan():
    net = ps.medium_c2(n=45, p=0.01, seed=19)
    targets = [ps.non_leaf_targets(net, 2)]
    plan = api.Plan(net, interest=[a for a, _ in targets[0]], reduce=1, group=1)
    r = 0.01
    say("[gpu] skart_run medium grouped r=0.01")
    res, record = api.skart_run(plan, 41, targets, r, traj=3, max_steps=1 << 23)
    assert res["status"] == 0, res
    bits = api.unpack_record(record.cpu().numpy(), res["steps"])
    ref = osim.run(net, 41, np.arange(3, 4), 1500, targets=targets, indicators=True)
    assert np.array_equal(bits[:1500], ref["z"][0])
    check_against_oracle(res, bits, r)


def test_skart_driver_limit():
    cfg = ps.config("C1")
    plan = api.Plan(cfg.net, interest=[0, 1], reduce=0, group=0)
    say("[gpu] skart_run C1 limit")
    res, _ = api.skart_run(plan, cfg.seed, cfg.targets, 1e-4, max_steps=20000)
    assert res["status"] == _lib.ERANGE
    assert not res["done"] and res["n_required"] > 20000 and res["steps"] <= 20000
