"""The load-latency probe behind the sweep's latency floor: a timed walk of a
cycle held in the vector L1 is faster per hop than one that needs the L2,
both within the range of a memory round trip, and the walk ends on the
cycle."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ff():
    from paper_1508_05151_amd import ff as _ff
    _ff.ff_init()
    return _ff


def _walk_ns(ff, n_ints, hops=4000):
    nxt = torch.from_numpy(ff.load_cycle(n_ints)).cuda()
    out = torch.zeros(2, dtype=torch.int64, device="cuda")
    ff.ff_probe_load_latency(nxt, 2 * (n_ints // 32), hops, out)
    torch.cuda.synchronize()
    ticks, last = out.tolist()
    assert last % 32 == 0 and 0 <= last < n_ints
    return ticks * 10.0 / hops


def test_l1_cycle_faster_than_l2_cycle(ff):
    l1 = min(_walk_ns(ff, 4096) for _ in range(3))
    l2 = min(_walk_ns(ff, 1 << 18) for _ in range(3))
    print(f"dependent load round trip: {l1:.1f} ns (16 KB cycle), {l2:.1f} ns (1 MB cycle)", flush=True)
    assert 10.0 < l1 < l2 < 5000.0
