"""What the trained proposal network does, on held-out seeded 1024x436 pairs
(seeds 4000.., never used in training), with the committed weights, by the
EPE < 3 px inlier rate of F against the synthetic ground truth and the
throughput of the whole path (descriptors, network where used, three fields,
filter) for a batch in one batched call.  The test asserts exactly what the
measurements support:

* the network alone lands within 3 px at a fifth or more of the seed points
  (an untrained network of the same architecture, the control, almost never);
* as an extra seed candidate beside the kd-tree it leaves the inlier rate
  where the plain method has it (within 0.002) and costs at most 5 % of the
  throughput (its forward pass in both directions);
* as the only seed candidate (no kd-tree) it is faster than the plain method
  by more than 10 % but loses inliers: it stays above the untrained control
  by 0.1 and below the plain method.

No mode measured so far is both faster than the plain method and at least as
accurate; the test fails if that changes without the claim being updated."""
import os
import sys

import pytest

from synth import pairs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_1508_05151_amd", "weights", "proposal_1024x436.safetensors")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_05151_amd import ff, proposal
    ff.ff_init()
    ev = pairs.layered_pairs(4000, 8, workers=8)
    return ff, proposal, ev


@pytest.mark.timeout(300)
def test_trained_network_gain_and_cost(env):
    ff, proposal, ev = env
    trained = proposal.load(WEIGHTS)
    untrained = ff.ProposalNet(seed=0)
    _say("trained")
    rt = proposal.evaluate(trained, ev, reps=5, log=_say)
    _say("untrained control")
    ru = proposal.evaluate(untrained, ev, modes=("learned",), reps=1, log=_say)
    plain, extra, only = rt["plain"], rt["plain+learned"], rt["learned"]
    assert rt["network_only_seed_points"] >= 0.2
    assert ru["network_only_seed_points"] < 0.05
    # extra candidate: accuracy unchanged, small cost
    assert abs(extra["inlier_F"] - plain["inlier_F"]) <= 0.002
    assert extra["mpx_s"] >= 0.95 * plain["mpx_s"]
    # only candidate: faster, less accurate
    assert only["mpx_s"] > 1.1 * plain["mpx_s"]
    assert only["inlier_F"] > ru["learned"]["inlier_F"] + 0.1
    assert only["inlier_F"] < plain["inlier_F"]
