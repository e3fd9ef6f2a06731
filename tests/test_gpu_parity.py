"""GPU parity: every stage of the HIP path against the CPU oracle, bit for bit
(all of the path is integer arithmetic).  Calls go through the C ABI
(paper_1508_05151_amd.ff); inputs come from the seeded generator."""
import sys

import numpy as np
import pytest

from oracle import ffo
from synth import pairs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

Q = 4


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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _gpu_desc(ff, img, k=3, radii=(8, 6)):
    img = np.ascontiguousarray(img)
    if img.ndim == 2:
        img = img[:, :, None]
    H, W, C = img.shape
    d = ff.ff_desc_init(W, H, C, k, Q, radii)
    blob = torch.zeros(d.bytes, dtype=torch.uint8, device="cuda")
    ff.ff_compute_descriptors(d, _dev(img), blob)
    return d, blob


def _ragged_pair(seed, W, H, C=3, nlayers=2):
    p = pairs.layered_pair(seed=seed, W=W, H=H, nlayers=nlayers)
    if C == 1:
        g = lambda im: np.ascontiguousarray(im[:, :, :1])
        p.img1, p.img2 = g(p.img1), g(p.img2)
    return p


CASES = [("square", lambda: pairs.square_pair(0), 3, (8, 6)),
         ("ragged97x61", lambda: _ragged_pair(5, 97, 61), 3, (8, 6)),
         ("gray75x50", lambda: _ragged_pair(6, 75, 50, C=1), 2, (5,)),
         ("tiny13x9", lambda: _ragged_pair(7, 13, 9), 1, (3,)),
         ("k4_200x120", lambda: _ragged_pair(8, 200, 120, nlayers=3), 4, (8, 6)),
         # degenerate sizes: one pixel, one column, one row, and a 2x2 image
         # whose every level step exceeds the image
         ("1x1", lambda: _ragged_pair(9, 1, 1), 3, (8, 6)),
         ("1x7", lambda: _ragged_pair(10, 1, 7), 2, (8, 6)),
         ("9x1", lambda: _ragged_pair(11, 9, 1), 2, (8, 6)),
         ("2x2", lambda: _ragged_pair(12, 2, 2), 3, (3,)),
         # the largest and the smallest WHT radius, odd radii, four radii
         ("radii15_1", lambda: _ragged_pair(13, 70, 40), 2, (15, 1)),
         ("gray_four_radii", lambda: _ragged_pair(14, 83, 37, C=1), 1, (2, 9, 12, 5))]


@pytest.mark.parametrize("name,make,k,radii", CASES, ids=[c[0] for c in CASES])
def test_descriptors_bit_exact(ff, name, make, k, radii):
    p = make()
    _say("descriptors", name, p.img1.shape)
    d, blob = _gpu_desc(ff, p.img1, k, radii)
    torch.cuda.synchronize()
    v = ff.blob_views(d, blob)
    o = ffo.Desc(p.img1, k, Q, radii)
    assert np.array_equal(v["lab"].cpu().numpy(), o.lab())
    for lev in range(k + 1):
        assert np.array_equal(v["smooth"][lev].cpu().numpy(), o.smooth(lev)), f"smooth level {lev}"
        cen = v["census"][lev].cpu().numpy().view(np.uint32)
        cent = v["census_t"][lev].cpu().numpy().view(np.uint32)
        for b in range(Q):
            for a in range(Q):
                ref = o.plane(lev, a, b)
                assert np.array_equal(cen[b, a], ref), f"census level {lev} phase {(a, b)}"
                assert np.array_equal(cent[b, a], ref.T), f"transposed census level {lev} phase {(a, b)}"
    for rho in radii:
        g = v["wht"][rho].cpu().numpy()[:, :, :9 * d.channels]
        assert np.array_equal(g, o.wht(rho)), f"wht {rho}"


def test_lab8_all_24bit_colours(ff):
    _say("lab8 exhaustive")
    v = np.arange(1 << 24, dtype=np.uint32)
    img = np.stack([(v >> 16) & 255, (v >> 8) & 255, v & 255], -1).astype(np.uint8).reshape(4, 1024, 4096, 3)
    # four 4096 x 1024 images (the library's limit is 2^22 pixels per image)
    d = ff.ff_desc_init(4096, 1024, 3, 0, 1, ())
    blob = torch.zeros(d.bytes, dtype=torch.uint8, device="cuda")
    for i in range(4):
        ff.ff_compute_descriptors(d, _dev(img[i]), blob)
        got = ff.blob_views(d, blob)["lab"].cpu().numpy()
        assert np.array_equal(got, ffo.lab8(img[i])), f"quarter {i}"


@pytest.mark.parametrize("W,H,rho", [(128, 96, 8), (320, 240, 6), (61, 37, 3)])
def test_kdtree_bit_exact(ff, W, H, rho):
    _say("kdtree", W, H, rho)
    p = _ragged_pair(W + H, W, H)
    d, blob = _gpu_desc(ff, p.img2, 0, (rho,))
    N = W * H
    leaf = 8
    nn = ff.ff_tree_nodes(N, leaf)
    nd = torch.empty(nn, dtype=torch.int32, device="cuda")
    ns = torch.empty(nn, dtype=torch.int32, device="cuda")
    perm = torch.empty(N, dtype=torch.int32, device="cuda")
    prm = ff.ff_default_params(k=0, leaf=leaf)
    ws = torch.empty(ff.ff_match_workspace_bytes(d, d, rho, prm), dtype=torch.uint8, device="cuda")
    ff.ff_build_kdtree(d, blob, rho, leaf, nd, ns, perm, ws)
    torch.cuda.synchronize()
    V = ffo.Desc(p.img2, 0, Q, (rho,)).wht(rho).reshape(N, -1)
    rnd, rns, rperm = ffo.kdtree_build(V, leaf)
    nd, ns, perm = nd.cpu().numpy(), ns.cpu().numpy(), perm.cpu().numpy()
    assert np.array_equal(nd, rnd)
    internal = rnd >= 0
    assert np.array_equal(ns[internal], rns[internal])
    assert np.array_equal(perm, rperm)


def _gpu_field(ff, d1, b1, d2, b2, r, **kw):
    prop = kw.pop("proposal", None)
    prm = ff.ff_default_params(**kw)
    ws = torch.empty(ff.ff_match_workspace_bytes(d1, d2, r, prm), dtype=torch.uint8, device="cuda")
    F = torch.empty((d1.height, d1.width), dtype=torch.int32, device="cuda")
    Cc = torch.empty_like(F)
    ff.ff_match_field(d1, b1, d2, b2, r, prm, prop, F, Cc, ws)
    torch.cuda.synchronize()
    assert ff.ff_read_status(ws) == 0
    return F.cpu().numpy(), Cc.cpu().numpy()


def test_field_every_step_square_pair(ff):
    p = pairs.square_pair(0)
    k, r = 3, 8
    d1, b1 = _gpu_desc(ff, p.img1, k, (r,))
    d2, b2 = _gpu_desc(ff, p.img2, k, (r,))
    o1, o2 = ffo.Desc(p.img1, k, Q, (r,)), ffo.Desc(p.img2, k, Q, (r,))
    for s in range(1, 1 + 7 + 8 * k + 1):
        _say("step", s)
        gF, gC = _gpu_field(ff, d1, b1, d2, b2, r, k=k, max_steps=s, seed=17)
        oF, oC = ffo.match_field(o1, o2, r, k=k, max_steps=s, seed=17)
        assert np.array_equal(gF, oF), f"flow differs after step {s}: {(gF != oF).sum()} px"
        assert np.array_equal(gC, oC), f"cost differs after step {s}"


@pytest.mark.parametrize("name,make,k,radii", CASES, ids=[c[0] for c in CASES])
def test_whole_pair_bit_exact(ff, name, make, k, radii):
    p = make()
    _say("pair", name)
    r = radii[0]
    r2 = radii[1] if len(radii) > 1 else radii[0]
    H, W = p.img1.shape[:2]
    Cc = 1 if p.img1.ndim == 2 else p.img1.shape[2]
    m = ff.PairMatcher(W, H, Cc, r=r, r2=r2, k=k, subpel=Q, eps=5, n_bwd=2 if len(radii) > 1 else 1)
    out = m.run(_dev(p.img1), _dev(p.img2), seed=1234, pair_id=3)
    torch.cuda.synchronize()
    assert m.status() == [0] * len(m.fields)
    ref = ffo.match_pair(p.img1, p.img2, r=r, r2=r2, k=k, Q=Q, eps=5, seed=1234, pair_id=3,
                         n_bwd=2 if len(radii) > 1 else 1)
    for key in ("F", "CF", "B1", "CB1", "keep", "filtered") + (("B2", "CB2") if len(radii) > 1 else ()):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key


def test_tree_ahead_and_split_descriptors_equal_the_whole_calls(ff):
    """ff_compute_lab_wht followed by ff_compute_census fills every region of
    a blob as ff_compute_descriptors does; a field seeded from the tree that
    ff_match_field_tree built ahead (use_kdtree = 2) equals one that builds
    it in the call; the pair with trees ahead equals the pair after whole
    descriptors."""
    p = _ragged_pair(21, 161, 97, nlayers=3)
    H, W = p.img1.shape[:2]
    N = W * H
    i1, i2 = _dev(p.img1), _dev(p.img2)
    d = ff.ff_desc_init(W, H, 3, 3, Q, (8, 6))
    whole = torch.zeros(d.bytes, dtype=torch.uint8, device="cuda")
    split = torch.zeros(d.bytes, dtype=torch.uint8, device="cuda")
    ff.ff_compute_descriptors(d, i1, whole)
    ff.ff_compute_lab_wht(d, i1, split)
    ff.ff_compute_census(d, split)
    torch.cuda.synchronize()
    regions = [(d.off_lab, 3 * N), (d.off_smooth, 4 * 3 * N * 2), (d.off_census, 4 * Q * Q * N * 4),
               (d.off_census_t, 4 * Q * Q * N * 4), (d.off_wht, 2 * N * 32 * 4)]
    for off, nb in regions:
        assert torch.equal(whole[off:off + nb], split[off:off + nb]), off
    # one field, tree built ahead vs in the call
    d2 = ff.ff_desc_init(W, H, 3, 3, Q, (8, 6))
    b2 = torch.empty(d2.bytes, dtype=torch.uint8, device="cuda")
    ff.ff_compute_descriptors(d2, i2, b2)
    outs = []
    for mode in (1, 2):
        prm = ff.ff_default_params(seed=5, field_id=0)
        ws = torch.empty(ff.ff_match_workspace_bytes(d, d2, 8, prm), dtype=torch.uint8, device="cuda")
        flow = torch.empty((H, W), dtype=torch.int32, device="cuda")
        cost = torch.empty_like(flow)
        if mode == 2:
            ff.ff_match_field_tree(d, whole, d2, b2, 8, prm, ws)
            prm.use_kdtree = 2
        ff.ff_match_field(d, whole, d2, b2, 8, prm, None, flow, cost, ws)
        torch.cuda.synchronize()
        outs.append((flow.cpu(), cost.cpu()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    # the whole pair both ways
    res = []
    for early in (False, True):
        m = ff.PairMatcher(W, H, 3, r=8, r2=6, k=3, subpel=Q, eps=5, early_trees=early)
        o = m.run(i1, i2, seed=77, pair_id=1)
        torch.cuda.synchronize()
        assert m.status() == [0] * len(m.fields)
        res.append({k: v.cpu().clone() for k, v in o.items() if v is not None})
    for key in res[0]:
        assert torch.equal(res[0][key], res[1][key]), key


def test_proposal_paths(ff):
    p = pairs.square_pair(2)
    k, r = 3, 8
    d1, b1 = _gpu_desc(ff, p.img1, k, (r,))
    d2, b2 = _gpu_desc(ff, p.img2, k, (r,))
    o1, o2 = ffo.Desc(p.img1, k, Q, (r,)), ffo.Desc(p.img2, k, Q, (r,))
    rng = np.random.default_rng(0)
    prop = ffo.pack(rng.integers(-200, 200, (12, 16)), rng.integers(-100, 100, (12, 16)))
    prop[rng.random((12, 16)) < 0.3] = ffo.EMPTY
    for use_tree in (1, 0):
        _say("proposal use_tree", use_tree)
        gF, gC = _gpu_field(ff, d1, b1, d2, b2, r, k=k, seed=5, use_kdtree=use_tree, proposal=_dev(prop))
        oF, oC = ffo.match_field(o1, o2, r, k=k, seed=5, use_kdtree=bool(use_tree), proposal=prop)
        assert np.array_equal(gF, oF) and np.array_equal(gC, oC)


def test_repeat_runs_identical(ff):
    """Schedule/race check: the wavefront's inter-band waits decide the
    result; repeated runs on a larger field must give the same bytes."""
    p = _ragged_pair(9, 256, 200, nlayers=4)
    k, r = 3, 8
    d1, b1 = _gpu_desc(ff, p.img1, k, (r,))
    d2, b2 = _gpu_desc(ff, p.img2, k, (r,))
    base = _gpu_field(ff, d1, b1, d2, b2, r, k=k, seed=3)
    for i in range(4):
        _say("repeat", i)
        got = _gpu_field(ff, d1, b1, d2, b2, r, k=k, seed=3)
        assert np.array_equal(got[0], base[0]) and np.array_equal(got[1], base[1])
    o1, o2 = ffo.Desc(p.img1, k, Q, (r,)), ffo.Desc(p.img2, k, Q, (r,))
    oF, oC = ffo.match_field(o1, o2, r, k=k, seed=3)
    assert np.array_equal(base[0], oF) and np.array_equal(base[1], oC)


@pytest.mark.parametrize("subpel", [1, 2, 8])
def test_subpel_variants_bit_exact(ff, subpel):
    """Whole pair at subpixel quanta other than the default 4: census phase
    planes, flows in 1/Q px and the filter's eps_q all change with Q."""
    p = _ragged_pair(40 + subpel, 90, 70, nlayers=3)
    _say("subpel", subpel)
    H, W = p.img1.shape[:2]
    m = ff.PairMatcher(W, H, 3, r=8, r2=6, k=3, subpel=subpel, eps=5)
    out = m.run(_dev(p.img1), _dev(p.img2), seed=99, pair_id=1)
    torch.cuda.synchronize()
    assert m.status() == [0, 0, 0]
    ref = ffo.match_pair(p.img1, p.img2, r=8, r2=6, k=3, Q=subpel, eps=5, seed=99, pair_id=1)
    for key in ("F", "CF", "B1", "CB1", "B2", "CB2", "keep", "filtered"):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key


@pytest.mark.parametrize("R,n_prop,n_rs,k,leaf", [(2, 4, 3, 3, 8), (1, 2, 1, 3, 8), (3, 6, 6, 2, 4),
                                                  (1, 4, 0, 3, 16), (1, 1, 1, 0, 8), (1, 8, 5, 2, 8),
                                                  (1, 4, 3, 0, 8), (1, 4, 3, 1, 8), (1, 4, 3, 3, 4),
                                                  (1, 4, 3, 3, 32), (1, 4, 3, 3, 64)])
def test_search_parameter_variants_bit_exact(ff, R, n_prop, n_rs, k, leaf):
    """Random-search radius multiplier, number of propagation sweeps and
    random searches per level, hierarchy depth (k = 0: no hierarchy) and
    kd-tree leaf size: one field against the oracle."""
    p = _ragged_pair(50 + R + n_prop, 96, 72, nlayers=3)
    _say("params", R, n_prop, n_rs, k, leaf)
    r = 8
    d1, b1 = _gpu_desc(ff, p.img1, k, (r,))
    d2, b2 = _gpu_desc(ff, p.img2, k, (r,))
    gF, gC = _gpu_field(ff, d1, b1, d2, b2, r, k=k, R=R, n_prop=n_prop, n_rs=n_rs, leaf=leaf, seed=7)
    o1, o2 = ffo.Desc(p.img1, k, Q, (r,)), ffo.Desc(p.img2, k, Q, (r,))
    oF, oC = ffo.match_field(o1, o2, r, k=k, R=R, n_prop=n_prop, n_rs=n_rs, leaf=leaf, seed=7)
    assert np.array_equal(gF, oF) and np.array_equal(gC, oC)


@pytest.mark.parametrize("band_rows", [8, 16, 32])
def test_pipelined_sweeps_equal_one_launch_per_stage(ff, band_rows):
    """The pipelined launches (random search behind its sweep, the next sweep
    of the same horizontal direction trailing it) give the same field as one
    launch per sweep and per search, at every band height; a ragged size so
    that the two sweeps' bands do not align."""
    p = _ragged_pair(77 + band_rows, 150, 101, nlayers=4)
    _say("pipeline", band_rows)
    k, r = 3, 8
    d1, b1 = _gpu_desc(ff, p.img1, k, (r,))
    d2, b2 = _gpu_desc(ff, p.img2, k, (r,))
    on = _gpu_field(ff, d1, b1, d2, b2, r, k=k, band_rows=band_rows, pipeline=1, seed=21)
    off = _gpu_field(ff, d1, b1, d2, b2, r, k=k, band_rows=band_rows, pipeline=0, seed=21)
    assert np.array_equal(on[0], off[0]) and np.array_equal(on[1], off[1])
    if band_rows == 16:
        o1, o2 = ffo.Desc(p.img1, k, Q, (r,)), ffo.Desc(p.img2, k, Q, (r,))
        oF, oC = ffo.match_field(o1, o2, r, k=k, seed=21)
        assert np.array_equal(on[0], oF) and np.array_equal(on[1], oC)


@pytest.mark.parametrize("pipeline", [0, 1])
def test_watchdog_reports_device_error_then_recovers(ff, pipeline):
    """Forced from the host: with a 1 us watchdog every wait of one band on
    another (and, pipelined, on another role's progress) gives up at once, the
    kernels still finish, and the call reports FF_ERR_DEVICE; the next call
    with the default watchdog is bit-exact with the oracle again."""
    p = pairs.square_pair(0)
    k, r = 3, 8
    _say("watchdog", pipeline)
    d1, b1 = _gpu_desc(ff, p.img1, k, (r,))
    d2, b2 = _gpu_desc(ff, p.img2, k, (r,))
    prm = ff.ff_default_params(k=k, seed=5, pipeline=pipeline, watchdog_us=1)
    ws = torch.empty(ff.ff_match_workspace_bytes(d1, d2, r, prm), dtype=torch.uint8, device="cuda")
    F = torch.empty((d1.height, d1.width), dtype=torch.int32, device="cuda")
    Cc = torch.empty_like(F)
    ff.ff_match_field(d1, b1, d2, b2, r, prm, None, F, Cc, ws)
    torch.cuda.synchronize()
    assert ff.ff_read_status(ws) == -6
    gF, gC = _gpu_field(ff, d1, b1, d2, b2, r, k=k, seed=5, pipeline=pipeline)
    o1, o2 = ffo.Desc(p.img1, k, Q, (r,)), ffo.Desc(p.img2, k, Q, (r,))
    oF, oC = ffo.match_field(o1, o2, r, k=k, seed=5)
    assert np.array_equal(gF, oF) and np.array_equal(gC, oC)
