"""Pins of the oracle's Flow Field search (sections 3.1 and 3.2) and of the
data term E_d (Eq. 1, Eq. 3, Eq. 4).  Expected values come from brute force,
closed forms, invariants and known-flow pairs -- never from the oracle's own
output for the same call."""
import numpy as np
import pytest

from oracle import ffo
from synth import pairs

Q = 4


def _texture(seed, H, W, C=3):
    rng = np.random.default_rng(seed)
    t = pairs._texture(rng, H, W, C)
    return np.clip(np.rint(t), 0, 255).astype(np.uint8)


def _shift_pair(seed, H, W, dx, dy, C=3):
    """Noise-free pair with I2(x + d) = I1(x): crops of one larger texture."""
    m = 8 + max(abs(dx), abs(dy))
    T = _texture(seed, H + 2 * m, W + 2 * m, C)
    I1 = T[m:m + H, m:m + W]
    I2 = T[m - dy:m - dy + H, m - dx:m - dx + W]
    return np.ascontiguousarray(I1), np.ascontiguousarray(I2)


def _grid(arr, n):
    return arr[::n, ::n]


def _level_of_step(step, k):
    # steps: 1 seed; 7 at the coarsest level; 8 (entry + 7) at each finer level
    if step <= 8:
        return k
    return k - 1 - (step - 9) // 8


def test_cost_symmetry_integer_flow():
    I1, I2 = _shift_pair(1, 20, 24, 3, -2)
    d1, d2 = ffo.Desc(I1, 2, Q, (3,)), ffo.Desc(I2, 2, Q, (3,))
    rng = np.random.default_rng(0)
    for _ in range(200):
        lev = int(rng.integers(0, 3))
        px, py = int(rng.integers(0, 24)), int(rng.integers(0, 20))
        fx, fy = int(rng.integers(-px, 24 - px)), int(rng.integers(-py, 20 - py))
        e12 = ffo.cost(d1, d2, lev, 3, px, py, fx * Q, fy * Q)
        e21 = ffo.cost(d2, d1, lev, 3, px + fx, py + fy, -fx * Q, -fy * Q)
        assert e12 == e21


def test_cost_invalid_centre_is_infinite_and_bounds():
    I1, I2 = _shift_pair(2, 16, 18, 1, 1)
    d1, d2 = ffo.Desc(I1, 1, Q, (2,)), ffo.Desc(I2, 1, Q, (2,))
    assert ffo.cost(d1, d2, 0, 2, 0, 0, -1, 0) == ffo.INF
    assert ffo.cost(d1, d2, 0, 2, 17, 15, 1, 0) == ffo.INF
    assert ffo.cost(d1, d2, 0, 2, 17, 15, 0, 0) < ffo.INF
    e = ffo.cost(d1, d2, 1, 2, 5, 5, 3, 2)
    assert 0 <= e <= 25 * 24


def test_exact_shift_cost_zero_at_true_flow():
    dx, dy = 3, -2
    I1, I2 = _shift_pair(3, 24, 28, dx, dy)
    d1, d2 = ffo.Desc(I1, 0, Q, (2,)), ffo.Desc(I2, 0, Q, (2,))
    r = 2
    for py in range(r + 3, 24 - r - 3):
        for px in range(r + 4, 28 - r - 4):
            assert ffo.cost(d1, d2, 0, r, px, py, dx * Q, dy * Q) == 0


def test_brute_force_nnf_is_lower_bound():
    """The exact NNF (Table 1's NNF row) bounds every field from below."""
    pair = pairs.layered_pair(seed=11, W=24, H=18, nlayers=2)
    r, k = 2, 1
    d1, d2 = ffo.Desc(pair.img1, k, Q, (r,)), ffo.Desc(pair.img2, k, Q, (r,))
    F, Cf = ffo.match_field(d1, d2, r, k=k, leaf=4, seed=5)
    nf, nc = ffo.brute_nnf(d1, d2, 0, r)
    assert np.all(Cf >= nc)
    # the brute force's own costs are what E says at its flows
    for (y, x) in [(0, 0), (5, 7), (17, 23)]:
        fx, fy = ffo.unpack(nf[y, x])
        assert ffo.cost(d1, d2, 0, r, x, y, int(fx), int(fy)) == nc[y, x]


def test_known_shift_field_found():
    dx, dy = 5, -3
    I1, I2 = _shift_pair(4, 40, 48, dx, dy)
    d1, d2 = ffo.Desc(I1, 2, Q, (3,)), ffo.Desc(I2, 2, Q, (3,))
    F, Cf = ffo.match_field(d1, d2, 3, k=2, seed=1)
    fx, fy = ffo.unpack(F)
    inner = np.s_[6:-6, 8:-8]
    ok = (fx[inner] == dx * Q) & (fy[inner] == dy * Q)
    assert ok.mean() > 0.95
    # away from the borders (patch radius + census stride + shift) the cost
    # at the true flow is exactly zero
    core = np.s_[3 + 1 + 3:-(3 + 1 + 3), 3 + 1 + 5:-(3 + 1 + 5)]
    assert np.all(Cf[core] == 0)


def test_steps_monotone_and_stored_cost_exact():
    pair = pairs.layered_pair(seed=21, W=48, H=36, nlayers=3)
    k, r = 2, 3
    d1, d2 = ffo.Desc(pair.img1, k, Q, (r,)), ffo.Desc(pair.img2, k, Q, (r,))
    total = 1 + 7 + 8 * k
    prev = None
    for s in range(1, total + 1):
        F, Cf = ffo.match_field(d1, d2, r, k=k, seed=9, max_steps=s)
        lev = _level_of_step(s, k)
        n = 1 << lev
        g, c = _grid(F, n), _grid(Cf, n)
        # every stored cost is E at the stored flow; EMPTY <-> INF
        assert np.array_equal(g == ffo.EMPTY, c == ffo.INF)
        ys, xs = np.nonzero(g != ffo.EMPTY)
        for y, x in zip(ys[::7], xs[::7]):
            fx, fy = ffo.unpack(g[y, x])
            assert ffo.cost(d1, d2, lev, r, x * n, y * n, int(fx), int(fy)) == c[y, x]
        # strict-improvement rule: within a level costs never rise
        if prev is not None and prev[0] == lev:
            assert np.all(c.astype(np.int64) <= prev[1].astype(np.int64))
        prev = (lev, c)
    # the last step is the full field
    F2, C2 = ffo.match_field(d1, d2, r, k=k, seed=9)
    assert np.array_equal(F, F2) and np.array_equal(Cf, C2)


def test_eleven_comparisons_per_point_per_level():
    """Table 2's text: 11 patch comparisons per point and level (4
    propagations x 2 candidates + 3 random searches).  With identical images
    every point keeps flow 0, so no point is ever empty."""
    img = _texture(6, 40, 56)
    k, r = 3, 2
    d = ffo.Desc(img, k, Q, (r,))
    F, Cf, cnt = ffo.match_field(d, d, r, k=k, skip_dup=False, counters=True)
    assert np.all(F == 0) and np.all(Cf == 0)
    for lev in range(k):
        n = 1 << lev
        Gw, Gh = -(-56 // n), -(-40 // n)
        exp = 4 * ((Gh - 1) * Gw + (Gw - 1) * Gh) + 3 * Gw * Gh
        assert cnt[1 + lev] == exp
        assert exp <= 11 * Gw * Gh
    assert cnt[0] == cnt[1:1 + k + 1].sum()


def test_duplicate_skipping_changes_nothing():
    pair = pairs.layered_pair(seed=31, W=40, H=30, nlayers=2)
    d1, d2 = ffo.Desc(pair.img1, 2, Q, (3,)), ffo.Desc(pair.img2, 2, Q, (3,))
    a = ffo.match_field(d1, d2, 3, k=2, seed=3, skip_dup=True)
    b = ffo.match_field(d1, d2, 3, k=2, seed=3, skip_dup=False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_square_pair_inlier_rate():
    p = pairs.square_pair(0)
    d1, d2 = ffo.Desc(p.img1, 3, Q, (8,)), ffo.Desc(p.img2, 3, Q, (8,))
    F, _ = ffo.match_field(d1, d2, 8, k=3, seed=0)
    assert pairs.inlier_rate(F, p, Q) > 0.9


def test_two_seed_spread():
    """Fig. 5a/b: the hierarchy spreads a field seeded at only two points (all
    other seeds 'infinity') over almost the whole image."""
    p = pairs.square_pair(0)
    k = 3
    d1, d2 = ffo.Desc(p.img1, k, Q, (8,)), ffo.Desc(p.img2, k, Q, (8,))
    Gw, Gh = 128 // 8, 96 // 8
    prop = np.full((Gh, Gw), ffo.EMPTY, np.int32)
    prop[2, 2] = ffo.pack(7 * Q, -3 * Q)
    prop[Gh - 3, Gw - 3] = ffo.pack(7 * Q, -3 * Q)
    F, Cf = ffo.match_field(d1, d2, 8, k=k, use_kdtree=False, proposal=prop, seed=2)
    assert (F != ffo.EMPTY).mean() > 0.9
    assert pairs.inlier_rate(F, p, Q) > 0.8


def test_empty_or_invalid_proposal_changes_nothing():
    p = pairs.square_pair(1)
    k = 3
    d1, d2 = ffo.Desc(p.img1, k, Q, (8,)), ffo.Desc(p.img2, k, Q, (8,))
    base = ffo.match_field(d1, d2, 8, k=k, seed=4)
    Gw, Gh = 16, 12
    empty = np.full((Gh, Gw), ffo.EMPTY, np.int32)
    far = np.full((Gh, Gw), ffo.pack(-30000, -30000), np.int32)
    for prop in (empty, far):
        got = ffo.match_field(d1, d2, 8, k=k, seed=4, proposal=prop)
        assert np.array_equal(got[0], base[0]) and np.array_equal(got[1], base[1])


def test_seed_is_first_minimum_over_leaf():
    """Eq. 1: a seed is the leaf entry of least cost, first one on ties."""
    p = pairs.layered_pair(seed=41, W=64, H=40, nlayers=2)
    k, r, leaf = 2, 3, 8
    d1, d2 = ffo.Desc(p.img1, k, Q, (r,)), ffo.Desc(p.img2, k, Q, (r,))
    F, Cf = ffo.match_field(d1, d2, r, k=k, leaf=leaf, max_steps=1)
    V2 = d2.wht(r).reshape(-1, 9 * 3)
    V1 = d1.wht(r)
    nd, ns, perm = ffo.kdtree_build(V2, leaf)
    n = 1 << k
    for gy in range(0, 40, n):
        for gx in range(0, 64, n):
            q = V1[gy, gx]
            node, st, c = 0, 0, V2.shape[0]
            while nd[node] >= 0:
                h = c // 2
                if q[nd[node]] >= ns[node]:
                    node, st, c = 2 * node + 2, st + h, c - h
                else:
                    node, c = 2 * node + 1, h
            costs = []
            for idx in perm[st:st + c]:
                fx, fy = (idx % 64 - gx) * Q, (idx // 64 - gy) * Q
                costs.append((ffo.cost(d1, d2, k, r, gx, gy, fx, fy), ffo.pack(fx, fy)))
            best = min(costs, key=lambda t: t[0])  # min() keeps the first minimum
            assert Cf[gy, gx] == best[0] and F[gy, gx] == best[1]


def test_data_term_is_local():
    """Eq. 1 at n = 1 with the census of section 3.3 reads only the patch, one
    census neighbour and one interpolation neighbour: the cost of a field's
    flow at an interior pixel equals the cost computed on crops of both
    images (margin r + 4) around the two patches, with the flow shifted by
    the crops' offset."""
    p = pairs.layered_pair(seed=8, W=96, H=72, nlayers=3)
    r, k = 8, 2
    o1, o2 = ffo.Desc(p.img1, k, Q, (r,)), ffo.Desc(p.img2, k, Q, (r,))
    F, Cst = ffo.match_field(o1, o2, r, k=k, seed=1)
    H, W = F.shape
    dx, dy = ffo.unpack(F)
    ys, xs = np.mgrid[0:H, 0:W]
    mx, my = xs * Q + dx, ys * Q + dy
    tx, ty = mx // Q, my // Q
    mg = r + 4
    inner = (F != ffo.pack(-32768, -32768)) & (xs >= mg) & (xs < W - mg) & (ys >= mg) & (ys < H - mg) & \
        (tx >= mg) & (tx < W - mg) & (ty >= mg) & (ty < H - mg)
    cand = np.flatnonzero(inner)
    assert cand.size > 50
    for idx in np.random.default_rng(1).choice(cand, size=12, replace=False):
        y, x = divmod(int(idx), W)
        cx, cy = int(tx.flat[idx]), int(ty.flat[idx])
        d1 = ffo.Desc(np.ascontiguousarray(p.img1[y - mg:y + mg + 1, x - mg:x + mg + 1]), 0, Q, (r,))
        d2 = ffo.Desc(np.ascontiguousarray(p.img2[cy - mg:cy + mg + 1, cx - mg:cx + mg + 1]), 0, Q, (r,))
        e = ffo.cost(d1, d2, 0, r, mg, mg, int(dx.flat[idx]) + (x - cx) * Q, int(dy.flat[idx]) + (y - cy) * Q)
        assert e == int(Cst.flat[idx])


@pytest.mark.parametrize("R", [1, 2])
def test_random_search_radius_scales_with_level(R):
    """Section 3.2: the random-search radius at level n is R_n = R n (pixels),
    i.e. offsets up to n R Q in 1/Q px per axis.  An exact-shift pair is
    seeded at flow 0 everywhere (no kd-tree, an all-zero proposal), so the
    first sweep changes nothing (every candidate equals the current flow) and
    every change made by the first random search of the coarsest level n = 2^k
    is one drawn offset.  The accepted offsets must stay within +-nRQ and reach
    past 3/4 of it (the true shift lies far outside every box, so any draw
    that lowers the cost is accepted, near the edge as often as near 0): a
    radius of R Q (unscaled), R (n/2) Q or 2 R n Q fails one of the bounds."""
    dx, dy = 28, -21          # px: outside every search box tested
    I1, I2 = _shift_pair(21, 96, 128, dx, dy)
    for k in (0, 1, 2, 3):
        n = 1 << k
        d1, d2 = ffo.Desc(I1, k, Q, (8,)), ffo.Desc(I2, k, Q, (8,))
        Gh, Gw = (96 + n - 1) // n, (128 + n - 1) // n
        zero = np.zeros((Gh, Gw), np.int32)
        kw = dict(k=k, R=R, use_kdtree=False, proposal=zero, seed=77)
        f_p1, _ = ffo.match_field(d1, d2, 8, max_steps=2, **kw)    # seed + P1
        f_rs, c_rs = ffo.match_field(d1, d2, 8, max_steps=3, **kw)  # ... + RS1
        a, b = _grid(f_p1, n), _grid(f_rs, n)
        assert np.all(a == 0), "the first sweep over a constant field changes nothing"
        ch = a != b
        assert ch.sum() > 20, (k, ch.sum())
        ox, oy = ffo.unpack(b[ch])
        bound = n * R * Q
        assert np.abs(ox).max() <= bound and np.abs(oy).max() <= bound, (k, R)
        big = max(np.abs(ox).max(), np.abs(oy).max())
        assert big > (n * R * Q) * 3 // 4, (k, R, big)
