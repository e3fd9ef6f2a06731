"""What the trained proposal network gains over the method without it, on
held-out seeded 1024x436 pairs (seeds never used in training), with the
committed weights: the network's flow alone at the seed points, and the whole
path in three modes -- plain (kd-tree seeds), plain + learned candidate, and
learned only (no kd-tree) -- by EPE < 3 px inlier rate of F against the
synthetic ground truth.  An untrained network (same architecture, initial
weights) is the control."""
import os
import sys

import numpy as np
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
    ev = [pairs.layered_pair(seed=4000 + i) for i in range(4)]
    return ff, proposal, ev


def test_trained_network_gain(env):
    ff, proposal, ev = env
    trained = proposal.load(WEIGHTS)
    untrained = ff.ProposalNet(seed=0)
    _say("trained")
    rt = proposal.evaluate(trained, ev, reps=1, log=_say)
    _say("untrained control")
    ru = proposal.evaluate(untrained, ev, modes=("learned",), reps=1, log=_say)
    # the network alone lands within 3 px at many seed points; untrained almost never
    assert rt["network_only_seed_points"] > 0.25
    assert ru["network_only_seed_points"] < 0.05
    # as the only seed candidate, the trained flow recovers most of the field
    assert rt["learned"]["inlier_F"] > 0.8
    assert rt["learned"]["inlier_F"] > ru["learned"]["inlier_F"] + 0.1
    # as an extra candidate it never costs accuracy
    assert rt["plain+learned"]["inlier_F"] >= rt["plain"]["inlier_F"] - 0.002
