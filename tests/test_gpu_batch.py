"""GPU parity of batched matching (many pairs of mixed sizes, every stage one
launch for all fields): each pair equals the oracle and the one-pair path byte
for byte, for every propagation band height, eagerly and replayed from a HIP
graph; the one-pair path replayed from a HIP graph equals its eager run."""
import sys

import numpy as np
import pytest

from oracle import ffo
from synth import pairs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

Q = 4
SIZES = [(97, 61), (128, 96), (64, 48), (150, 37)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ff():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_05151_amd import ff as _ff
    _ff.ff_init()
    return _ff


@pytest.fixture(scope="module")
def batch_pairs():
    return [pairs.layered_pair(seed=3000 + i, W=W, H=H, nlayers=3) for i, (W, H) in enumerate(SIZES)]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(o):
    return {k: (v[0].cpu().numpy(), v[1].cpu().numpy()) if isinstance(v, tuple) else v.cpu().numpy()
            for k, v in o.items()}


def _check_against_oracle(out, prs, seeds):
    for i, p in enumerate(prs):
        ref = ffo.match_pair(p.img1, p.img2, r=8, r2=6, k=3, Q=Q, eps=5, seed=seeds[i], pair_id=i)
        o = out[i]
        for name in ("F", "B1", "B2"):
            assert np.array_equal(o[name][0].cpu().numpy(), ref[name]), (i, name)
            assert np.array_equal(o[name][1].cpu().numpy(), ref["C" + name]), (i, "C" + name)
        assert np.array_equal(o["keep"].cpu().numpy(), ref["keep"]), i
        assert np.array_equal(o["filtered"].cpu().numpy(), ref["filtered"]), i


def test_batch_equals_oracle_every_band_height(ff, batch_pairs):
    """Every band height, with and without pipelined sweep pairs, gives the
    oracle's bytes for every pair of the batch."""
    seeds = [11, 12, 13, 14]
    i1 = [_dev(p.img1) for p in batch_pairs]
    i2 = [_dev(p.img2) for p in batch_pairs]
    first = None
    for bh, pipe in ((16, 0), (8, 0), (32, 0), (16, 1), (8, 1), (32, 1)):
        _say("batch band_rows", bh, "pipeline", pipe)
        m = ff.BatchMatcher(SIZES, band_rows=bh, pipeline=pipe)
        out = m.run(i1, i2, seeds=seeds)
        torch.cuda.synchronize()
        assert m.status() == 0
        got = [_np(o) for o in out]
        if first is None:
            first = got
            _check_against_oracle(out, batch_pairs, seeds)
        else:
            for a, b in zip(first, got):
                for key in a:
                    if isinstance(a[key], tuple):
                        assert np.array_equal(a[key][0], b[key][0]) and np.array_equal(a[key][1], b[key][1]), key
                    else:
                        assert np.array_equal(a[key], b[key]), key


def test_batch_equals_single_pair_path(ff, batch_pairs):
    seeds = [5, 6, 7, 8]
    i1 = [_dev(p.img1) for p in batch_pairs]
    i2 = [_dev(p.img2) for p in batch_pairs]
    m = ff.BatchMatcher(SIZES)
    out = m.run(i1, i2, seeds=seeds)
    torch.cuda.synchronize()
    for i, (W, H) in enumerate(SIZES):
        _say("single", i)
        s = ff.PairMatcher(W, H, 3, r=8, r2=6, k=3, subpel=Q, eps=5)
        o = s.run(i1[i], i2[i], seed=seeds[i], pair_id=i)
        torch.cuda.synchronize()
        for name, key in (("F", "F"), ("B1", "B1"), ("B2", "B2")):
            assert torch.equal(o[key], out[i][name][0]), (i, name)
        assert torch.equal(o["keep"], out[i]["keep"]) and torch.equal(o["filtered"], out[i]["filtered"])


def test_batch_graph_replays(ff, batch_pairs):
    seeds = [1, 2, 3, 4]
    i1 = [_dev(p.img1) for p in batch_pairs]
    i2 = [_dev(p.img2) for p in batch_pairs]
    m = ff.BatchMatcher(SIZES)
    eager = [_np(o) for o in m.run(i1, i2, seeds=seeds)]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        m.run(i1, i2, seeds=seeds)   # allocate the workspace outside the capture
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        m.run(i1, i2, seeds=seeds)
    for rep in range(3):
        _say("graph replay", rep)
        for o in m.out:                      # scribble on the outputs between replays
            for name in ("F", "B1", "B2"):
                o[name][0].fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert m.status() == 0
        got = [_np(o) for o in m.out]
        for a, b in zip(eager, got):
            for key in a:
                if isinstance(a[key], tuple):
                    assert np.array_equal(a[key][0], b[key][0]) and np.array_equal(a[key][1], b[key][1]), key
                else:
                    assert np.array_equal(a[key], b[key]), key


def test_pair_graph_replays(ff, batch_pairs):
    """The one-pair path (three field streams forked from and joined back to
    the caller's stream by events) captured in one HIP graph: every replay,
    with eager runs and scribbled outputs between replays, equals the eager
    result byte for byte."""
    p = batch_pairs[1]
    W, H = SIZES[1]
    i1, i2 = _dev(p.img1), _dev(p.img2)
    m = ff.PairMatcher(W, H, 3, r=8, r2=6, k=3, subpel=Q, eps=5)
    out = m.run(i1, i2, seed=31)
    torch.cuda.synchronize()
    eager = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        gout = m.run(i1, i2, seed=31)
    for rep in range(3):
        _say("pair graph replay", rep)
        for key in ("F", "B1", "B2", "filtered"):
            gout[key].fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert m.status() == [0, 0, 0]
        for key, v in eager.items():
            assert np.array_equal(gout[key].cpu().numpy(), v), (rep, key)
        m.run(i1, i2, seed=5)   # eager work of its own between replays
        torch.cuda.synchronize()
