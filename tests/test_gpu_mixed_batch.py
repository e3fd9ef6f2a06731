"""GPU parity of the mixed-size batch at its own sizes: two pairs of each of
320x240, 640x480, 1024x436 and 1242x375, taken from the 64-pair batch (pair i
has seed 3000 + i), matched in one batched call.  Every output of every pair
(F, B1, B2 and their costs, the keep mask, the filtered field) equals the
oracle's byte for byte, and equals the one-pair path's, at the band heights
the batch autotuner chooses from.  The oracle (single-threaded C++) runs the
eight pairs on eight host threads."""
import concurrent.futures as cf
import sys

import numpy as np
import pytest

from oracle import ffo
from synth import pairs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

Q = 4
# indices into the 64-pair batch: two of each size, in the batch's own order
SUBSET = (6, 17, 1, 2, 5, 12, 0, 3)
SIZES = {6: (320, 240), 17: (320, 240), 1: (640, 480), 2: (640, 480), 5: (1024, 436), 12: (1024, 436),
         0: (1242, 375), 3: (1242, 375)}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def subset():
    _say("mixed batch: drawing", len(SUBSET), "pairs")
    prs = pairs.mixed_pairs_subset(SUBSET, workers=8)
    for i, p in zip(SUBSET, prs):
        assert (p.img1.shape[1], p.img1.shape[0]) == SIZES[i], i
    return prs


@pytest.fixture(scope="module")
def oracle_out(subset):
    _say("mixed batch: oracle on 8 threads")

    def one(j):
        p = subset[j]
        return ffo.match_pair(p.img1, p.img2, r=8, r2=6, k=3, Q=Q, eps=5, seed=p.seed, pair_id=j)

    with cf.ThreadPoolExecutor(8) as ex:
        out = list(ex.map(one, range(len(subset))))
    _say("mixed batch: oracle done")
    return out


@pytest.mark.timeout(900)
def test_mixed_size_batch_equals_oracle_and_one_pair_path(subset, oracle_out):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_05151_amd import ff
    ff.ff_init()
    shapes = [(p.img1.shape[1], p.img1.shape[0]) for p in subset]
    seeds = [p.seed for p in subset]
    i1 = [torch.from_numpy(p.img1).cuda() for p in subset]
    i2 = [torch.from_numpy(p.img2).cuda() for p in subset]
    singles = {}
    for j, (w, h) in enumerate(shapes):
        sm = ff.PairMatcher(w, h, 3, r=8, r2=6, k=3, subpel=Q, eps=5)
        o = sm.run(i1[j], i2[j], seed=seeds[j], pair_id=j)
        torch.cuda.synchronize()
        assert sm.status() == [0, 0, 0]
        singles[j] = {k: v.cpu().numpy() for k, v in o.items()}
        del sm
    for bh, pipe in ((32, 0), (16, 0), (16, 1)):
        _say("mixed batch: band rows", bh, "pipelined", pipe)
        m = ff.BatchMatcher(shapes, band_rows=bh, pipeline=pipe)
        out = m.run(i1, i2, seeds=seeds)
        torch.cuda.synchronize()
        assert m.status() == 0
        for j in range(len(subset)):
            ref, one, o = oracle_out[j], singles[j], out[j]
            for name in ("F", "B1", "B2"):
                f, c = o[name][0].cpu().numpy(), o[name][1].cpu().numpy()
                assert np.array_equal(f, ref[name]), (bh, pipe, j, name)
                assert np.array_equal(c, ref["C" + name]), (bh, pipe, j, "C" + name)
                assert np.array_equal(f, one[name]) and np.array_equal(c, one["C" + name]), (j, name)
            for key in ("keep", "filtered"):
                assert np.array_equal(o[key].cpu().numpy(), ref[key]), (bh, pipe, j, key)
                assert np.array_equal(o[key].cpu().numpy(), one[key]), (j, key)
        del m
