"""Maximum sizes: an 8191 x 512 RGB pair (the largest width the descriptors
accept at Q = 4, and 4,193,792 of the 2^22 points they allow), and a
4095 x 818 RGB pair at Q = 8, k = 3 (within 0.2 % of the largest image the
sweep can address with 32-bit offsets at that Q and k: its largest target
word index is 2^30 - 1,834,625), through the benchmark's launch
configuration.  The oracle cannot match fields this size in test time, so the
test checks what holds point by point:

* every field is EMPTY exactly where its cost is infinite, and every flow's
  centre lies inside the other image (section 3.1: no flow leaves the image);
* the cost reported at sampled interior pixels equals the oracle's data term
  of the reported flow (Eq. 1 at n = 1 with the census of section 3.3),
  computed on crops of both images around the two patches -- the data term
  at n = 1 reads only the patch, one census neighbour and one interpolation
  neighbour, so a crop with a margin of r + 4 pixels gives the same value;
* the pipelined and the one-launch-per-stage schedules give the same bytes.
"""
import sys

import numpy as np
import pytest

from oracle import ffo
from synth import pairs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EMPTY = np.int32(np.uint32(0x80008000).view(np.int32))
INF = np.int32(2 ** 31 - 1)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _unpack(f):
    u = f.astype(np.int64) & 0xFFFFFFFF
    dx = ((u & 0xFFFF) ^ 0x8000) - 0x8000
    dy = (((u >> 16) & 0xFFFF) ^ 0x8000) - 0x8000
    return dx, dy


@pytest.mark.timeout(600)
@pytest.mark.parametrize("W,H,Q", [(8191, 512, 4), (4095, 818, 8)])
def test_max_size_pair_properties(W, H, Q):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_05151_amd import ff
    ff.ff_init()
    d = ff.ff_desc_init(W, H, 3, 3, Q, (8, 6))
    assert (d.off_census_t - d.off_census) // 4 + Q * Q * W * H <= 1 << 30
    _say("max size: generating the pair", W, H, "Q", Q)
    p = pairs.layered_pair(seed=3000, W=W, H=H)
    i1, i2 = torch.from_numpy(p.img1).cuda(), torch.from_numpy(p.img2).cuda()
    _say("max size: pipelined run")
    m = ff.PairMatcher(W, H, 3, r=8, r2=6, k=3, subpel=Q, eps=5)
    out = m.run(i1, i2, seed=3000)
    torch.cuda.synchronize()
    assert m.status() == [0, 0, 0]
    got = {k: v.cpu().numpy() for k, v in out.items()}
    del m
    _say("max size: one launch per stage")
    m0 = ff.PairMatcher(W, H, 3, r=8, r2=6, k=3, subpel=Q, eps=5, pipeline=0)
    out0 = m0.run(i1, i2, seed=3000)
    torch.cuda.synchronize()
    assert m0.status() == [0, 0, 0]
    for key, v in out0.items():
        assert np.array_equal(v.cpu().numpy(), got[key]), key
    del m0
    rng = np.random.default_rng(7)
    for name, r, src, dst in (("F", 8, p.img1, p.img2), ("B1", 8, p.img2, p.img1), ("B2", 6, p.img2, p.img1)):
        flow, cost = got[name], got["C" + name]
        empty = flow == EMPTY
        assert np.array_equal(cost == INF, empty), name
        assert empty.mean() < 0.01, name
        dx, dy = _unpack(flow)
        ys, xs = np.mgrid[0:H, 0:W]
        mx, my = xs * Q + dx, ys * Q + dy
        ok = ~empty
        assert ((mx[ok] >= 0) & (mx[ok] <= (W - 1) * Q) & (my[ok] >= 0) & (my[ok] <= (H - 1) * Q)).all(), name
        # sampled data terms on crops
        mg = r + 4
        tx, ty = mx // Q, my // Q
        inner = ok & (xs >= mg) & (xs < W - mg) & (ys >= mg) & (ys < H - mg) & \
            (tx >= mg) & (tx < W - mg) & (ty >= mg) & (ty < H - mg)
        cand = np.flatnonzero(inner)
        assert cand.size > 1000, name
        picks = rng.choice(cand, size=24, replace=False)
        for idx in picks:
            y, x = divmod(int(idx), W)
            cx, cy = int(tx.flat[idx]), int(ty.flat[idx])
            c1 = np.ascontiguousarray(src[y - mg:y + mg + 1, x - mg:x + mg + 1])
            c2 = np.ascontiguousarray(dst[cy - mg:cy + mg + 1, cx - mg:cx + mg + 1])
            d1, d2 = ffo.Desc(c1, 0, Q, (r,)), ffo.Desc(c2, 0, Q, (r,))
            # the same flow in crop coordinates: both crops put their centre at mg
            fx = int(dx.flat[idx]) + (x - cx) * Q
            fy = int(dy.flat[idx]) + (y - cy) * Q
            e = ffo.cost(d1, d2, 0, r, mg, mg, fx, fy)
            assert e == int(cost.flat[idx]), (name, x, y, e, int(cost.flat[idx]))
        _say("max size:", name, "checked", len(picks), "sampled costs")
