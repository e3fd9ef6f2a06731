"""The no-allocation entry point (ff_match_field_noalloc: the library's
static per-device scratch instead of a caller workspace) gives the same
flows, costs and status as ff_match_field, through the C ABI, on two calls in
a row, the second with a smaller input (the scratch keeps the first call's
contents), and refuses a field whose workspace exceeds the scratch before
anything is enqueued."""
import sys

import numpy as np
import pytest

from synth import pairs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

Q = 4


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _descs(ff, p, k=3, radii=(8, 6)):
    H, W = p.img1.shape[:2]
    d = ff.ff_desc_init(W, H, 3, k, Q, radii)
    b1 = torch.empty(d.bytes, dtype=torch.uint8, device="cuda")
    b2 = torch.empty_like(b1)
    ff.ff_compute_descriptors(d, torch.from_numpy(p.img1).cuda(), b1)
    ff.ff_compute_descriptors(d, torch.from_numpy(p.img2).cuda(), b2)
    return d, b1, b2


def _with_workspace(ff, d, b1, b2, r, prm):
    ws = torch.empty(ff.ff_match_workspace_bytes(d, d, r, prm), dtype=torch.uint8, device="cuda")
    F = torch.empty((d.height, d.width), dtype=torch.int32, device="cuda")
    Cc = torch.empty_like(F)
    ff.ff_match_field(d, b1, d, b2, r, prm, None, F, Cc, ws)
    torch.cuda.synchronize()
    assert ff.ff_read_status(ws) == 0
    return F.cpu().numpy(), Cc.cpu().numpy()


def _noalloc(ff, d, b1, b2, r, prm):
    F = torch.full((d.height, d.width), 7, dtype=torch.int32, device="cuda")
    Cc = torch.full_like(F, 7)
    st = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    ff.ff_match_field_noalloc(d, b1, d, b2, r, prm, None, F, Cc, st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return F.cpu().numpy(), Cc.cpu().numpy()


@pytest.mark.timeout(300)
def test_noalloc_equals_workspace_entry_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_05151_amd import ff
    ff.ff_init()
    big = pairs.layered_pair(seed=1000)                           # 1024 x 436, the benchmark pair
    small = pairs.layered_pair(seed=1001, W=150, H=37, nlayers=2)  # smaller, ragged
    for name, p, r, kw in (("1024x436 r=8", big, 8, {}), ("150x37 r=6", small, 6, dict(seed=3, field_id=2))):
        _say("noalloc:", name)
        d, b1, b2 = _descs(ff, p)
        prm = ff.ff_default_params(**kw)
        want = _with_workspace(ff, d, b1, b2, r, prm)
        got = _noalloc(ff, d, b1, b2, r, prm)
        assert np.array_equal(got[0], want[0]), name
        assert np.array_equal(got[1], want[1]), name
    # a field whose workspace exceeds the scratch is refused before any launch
    d = ff.ff_desc_init(1920, 1080, 3, 3, Q, (8,))
    prm = ff.ff_default_params()
    assert ff.ff_match_workspace_bytes(d, d, 8, prm) > ff.NOALLOC_SCRATCH_BYTES
    F = torch.empty((1080, 1920), dtype=torch.int32, device="cuda")
    with pytest.raises(ff.FFError) as e:
        ff.ff_match_field_noalloc(d, F, d, F, 8, prm, None, F, F)
    assert e.value.code == -2
