"""Full-size parity: the benchmark's own workload (one 1024x436 layered pair,
seed 1000, r = 8, r2 = 6, k = 3, Q = 4, eps = 5) run in the benchmark's launch
configuration (three fields on three streams), and the same pair inside a
batched call with a second pair, both compared byte for byte with the oracle
on every output: F, B1, B2 with their costs, the keep mask and the filtered
field, the region filter of section 3.4 behind the check (s = 50) and the
sparsification of section 3.5 (e = 4).  The oracle needs about a minute for
this pair.  The KITTI-shaped gray pair (1242x375, eps = 1, s = 150, e = 9) is
checked the same way."""
import sys

import numpy as np
import pytest

from oracle import ffo
from synth import pairs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(600)
def test_benchmark_pair_bit_exact_single_and_batched():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_05151_amd import ff
    ff.ff_init()
    p = pairs.layered_pair(1000)
    q = pairs.layered_pair(1001)
    H, W = p.img1.shape[:2]
    i1, i2 = torch.from_numpy(p.img1).cuda(), torch.from_numpy(p.img2).cuda()
    _say("full size: single pair, three streams")
    m = ff.PairMatcher(W, H, 3, r=8, r2=6, k=3, subpel=4, eps=5, region_s=50, sparse_e=4)
    out = m.run(i1, i2, seed=1000, pair_id=0)
    torch.cuda.synchronize()
    assert m.status() == [0, 0, 0]
    got = {k: v.cpu().numpy() for k, v in out.items()}
    _say("full size: batched call with a second pair")
    bm = ff.BatchMatcher([(W, H), (W, H)])
    bout = bm.run([i1, torch.from_numpy(q.img1).cuda()], [i2, torch.from_numpy(q.img2).cuda()], seeds=[1000, 1001])
    torch.cuda.synchronize()
    assert bm.status() == 0
    _say("full size: oracle")
    ref = ffo.match_pair(p.img1, p.img2, r=8, r2=6, k=3, Q=4, eps=5, seed=1000, pair_id=0, region_s=50,
                         sparse_e=4)
    for key in ("F", "CF", "B1", "CB1", "B2", "CB2", "keep", "filtered", "region_label", "keep_region",
                "filtered_region", "pick", "sparse"):
        assert np.array_equal(got[key], ref[key]), (key, int((got[key] != ref[key]).sum()))
    for name in ("F", "B1", "B2"):
        assert np.array_equal(bout[0][name][0].cpu().numpy(), ref[name]), name
        assert np.array_equal(bout[0][name][1].cpu().numpy(), ref["C" + name]), name
    assert np.array_equal(bout[0]["keep"].cpu().numpy(), ref["keep"])
    assert np.array_equal(bout[0]["filtered"].cpu().numpy(), ref["filtered"])


@pytest.mark.timeout(600)
def test_driving_pair_bit_exact():
    """The KITTI-shaped workload at full size: one 1242x375 gray pair (radial
    expansion up to 250 px, three moving rectangles, flat blobs, noise 3),
    r = 8, r2 = 6, k = 3, Q = 4 and the strict consistency threshold eps = 1,
    every output byte for byte against the oracle (about 40 s of oracle)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_05151_amd import ff
    ff.ff_init()
    p = pairs.driving_pair(2000)
    H, W, C = p.img1.shape
    _say("driving pair: GPU", W, H, C)
    m = ff.PairMatcher(W, H, C, r=8, r2=6, k=3, subpel=4, eps=1, region_s=150, sparse_e=9)
    out = m.run(torch.from_numpy(p.img1).cuda(), torch.from_numpy(p.img2).cuda(), seed=2000)
    torch.cuda.synchronize()
    assert m.status() == [0, 0, 0]
    got = {k: v.cpu().numpy() for k, v in out.items()}
    _say("driving pair: oracle")
    ref = ffo.match_pair(p.img1, p.img2, r=8, r2=6, k=3, Q=4, eps=1, seed=2000, region_s=150, sparse_e=9)
    for key in ("F", "CF", "B1", "CB1", "B2", "CB2", "keep", "filtered", "region_label", "keep_region",
                "filtered_region", "pick", "sparse"):
        assert np.array_equal(got[key], ref[key]), (key, int((got[key] != ref[key]).sum()))
    assert 0.0 < ref["keep"].mean() < 1.0
    assert ref["keep_region"].sum() < ref["keep"].sum()
