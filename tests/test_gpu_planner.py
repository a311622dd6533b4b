"""GPU: the planner measures the plain kernel's rate with one probe and picks
the preparation with the smallest predicted total time."""
import pytest

import pbn_synth as ps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1605_00854_amd import planner  # noqa: E402


def test_planner_choice_follows_sample_size():
    net = ps.medium_c2(n=150, p=1e-3, seed=27, leaf_frac=0.5)
    tgs = [ps.non_leaf_targets(net, 3)]
    interest = [a for a, _ in tgs[0]]
    print("[gpu] planner probes", flush=True)
    opts, wpb, d = planner.choose(net, interest, tgs, ntraj=1024, steps=1)
    assert d["choice"] == "plain" and opts == dict(reduce=0, group=0)
    assert d["plain_rate"] > 0 and d["predicted_seconds"]["plain"] == min(d["predicted_seconds"].values())
    opts, wpb, d = planner.choose(net, interest, tgs, ntraj=4096, steps=10**9, plain_rate=d["plain_rate"])
    assert d["choice"] in ("reduction", "tuned") and d["leaf_fraction"] >= 0.5
    assert d["predicted_seconds"][d["choice"]] == min(d["predicted_seconds"].values())
