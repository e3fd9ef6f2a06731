"""Pins of the oracle's SIFT-flow data term (section 3.3): dense SIFT, PCA
colours, integer smoothing of the colours and the L2 patch cost, each
checked against what geometry, the SIFT construction or linear algebra fix
rather than against itself."""
import numpy as np
import pytest

from oracle import ffo
from synth import pairs

SIG = 6.0        # Gaussian window: sigma = 2 c, c = 3
CELL = 3.0


def _ramp(W, H, a, b, c0):
    y, x = np.mgrid[0:H, 0:W]
    return (a * x + b * y + c0).astype(np.uint8)


def _texture(W, H, seed):
    rng = np.random.default_rng(seed)
    base = rng.integers(0, 256, (H // 4 + 2, W // 4 + 2)).astype(np.float64)
    up = np.kron(base, np.ones((4, 4)))[:H, :W]
    k = np.ones(3) / 3
    up = np.apply_along_axis(lambda r: np.convolve(r, k, "same"), 1, up)
    up = np.apply_along_axis(lambda r: np.convolve(r, k, "same"), 0, up)
    return np.clip(up + rng.normal(0, 3, (H, W)), 0, 255).astype(np.uint8)


def test_constant_image_has_zero_descriptors():
    D = ffo.dense_sift(np.full((20, 24), 77, np.uint8))
    assert np.all(D == 0)


def test_ramp_closed_form():
    """A linear ramp has one gradient g = (a, b) everywhere inside.  Away from
    the borders every cell histogram is then (1 - w, w) |g| on the two bins
    around atan2(b, a), times the cell's window mass, which factors into two
    1-D sums (the Gaussian and the bilinear weights are both separable):
    M_i = sum_d exp(-d^2 / (2 sigma^2)) max(0, 1 - |d / c - (i - 1.5)|)."""
    a, b = 2, 1
    L = _ramp(48, 40, a, b, 10)
    D = ffo.dense_sift(L)
    d = np.arange(-7, 8)
    M = np.array([np.sum(np.exp(-d ** 2 / (2 * SIG ** 2)) * np.maximum(0, 1 - np.abs(d / CELL - (i - 1.5))))
                  for i in range(4)])
    t = np.arctan2(b, a) / (np.pi / 4)
    o0 = int(np.floor(t))
    w = t - o0
    v = np.zeros(128)
    for j in range(4):
        for i in range(4):
            v[(4 * j + i) * 8 + o0] = (1 - w) * M[i] * M[j]
            v[(4 * j + i) * 8 + (o0 + 1) % 8] = w * M[i] * M[j]
    v /= np.linalg.norm(v)
    v = np.minimum(v, 0.2)
    v /= np.linalg.norm(v)
    for (x, y) in [(20, 20), (24, 17), (30, 22)]:
        np.testing.assert_allclose(D[y, x], v, atol=1e-12)


def test_rotation_by_90_degrees_permutes_cells_and_bins():
    """np.rot90 maps pixel (x, y) to (y, W-1-x) and a gradient (gx, gy) to
    (gy, -gx): the orientation drops by 90 degrees (two bins) and cell (i, j)
    moves to (j, 3 - i).  Exact for every pixel (borders map to borders)."""
    L = _texture(40, 32, 1)
    W = L.shape[1]
    D = ffo.dense_sift(L)
    Dr = ffo.dense_sift(np.ascontiguousarray(np.rot90(L)))
    idx = np.empty(128, np.int64)
    for j in range(4):
        for i in range(4):
            for o in range(8):
                idx[(4 * j + i) * 8 + o] = (4 * (3 - i) + j) * 8 + (o - 2) % 8
    for (x, y) in [(0, 0), (5, 7), (20, 13), (39, 31), (11, 30)]:
        np.testing.assert_allclose(Dr[W - 1 - x, y][idx], D[y, x], atol=1e-12)


def test_contrast_reversal_shifts_bins_by_four():
    L = _texture(36, 28, 2)
    D = ffo.dense_sift(L)
    Dn = ffo.dense_sift(255 - L)
    idx = np.array([(e // 8) * 8 + (e % 8 + 4) % 8 for e in range(128)])
    np.testing.assert_allclose(Dn[..., idx], D, atol=1e-12)


def test_gain_invariance_and_translation_equivariance():
    L = (_texture(40, 30, 3) // 2).astype(np.uint8)
    D = ffo.dense_sift(L)
    np.testing.assert_allclose(ffo.dense_sift(2 * L), D, atol=1e-12)
    big = _texture(60, 50, 4)
    Db = ffo.dense_sift(big)
    Dc = ffo.dense_sift(np.ascontiguousarray(big[10:40, 12:52]))
    # interior of the crop: every sample (reach 7) and gradient inside both
    np.testing.assert_allclose(Dc[8:22, 8:32], Db[18:32, 20:44], atol=1e-12)


def test_unit_length_and_clamp():
    """Unit length and non-negative everywhere; the clamp at 0.2 shows on a
    step edge, whose mass sits in bin 0 of a few cells: the clamped elements
    end up as equal maxima after the second normalisation."""
    D = ffo.dense_sift(_texture(32, 24, 5))
    np.testing.assert_allclose(np.linalg.norm(D, axis=-1), 1.0, atol=1e-12)
    assert np.all(D >= 0)
    # a single vertical step edge: every gradient points along +x, so only
    # bin 0 of the cells is non-zero; 16 cell masses, symmetric in i and j
    L = np.zeros((40, 40), np.uint8)
    L[:, 20:] = 200
    v = ffo.dense_sift(L)[20, 20]
    nz = v[v > 0]
    assert np.all(v.reshape(16, 8)[:, 1:] == 0)
    # renormalised after the clamp: the clamped elements are the equal maxima
    top = v.max()
    assert np.sum(np.isclose(v, top, rtol=0, atol=1e-12)) >= 2 and len(nz) <= 16


def test_pca_recovers_a_known_decomposition():
    """Data built with sample covariance exactly U diag(s^2) U^T (centred
    orthonormal columns times the scales times a random rotation): the PCA
    returns s^2 and the columns of U up to sign, and the sign rule holds."""
    rng = np.random.default_rng(7)
    N = 4000
    Z = rng.standard_normal((N, 128))
    Z -= Z.mean(axis=0)
    Qz, _ = np.linalg.qr(Z)
    s = np.linspace(3.0, 0.1, 128) ** 1.5
    U, _ = np.linalg.qr(rng.standard_normal((128, 128)))
    mu = rng.standard_normal(128)
    X = np.sqrt(N) * (Qz * s) @ U.T + mu
    half = N // 2
    mean, lam, V = ffo.sift_pca(X[:half], X[half:])
    np.testing.assert_allclose(mean, mu, atol=1e-9)
    np.testing.assert_allclose(lam, s ** 2, rtol=1e-9, atol=1e-12)
    for k in range(128):
        assert abs(abs(V[:, k] @ U[:, k]) - 1) < 1e-8
        m = np.argmax(np.abs(V[:, k]))
        assert V[m, k] > 0


def test_codes_quantisation():
    """Codes are round-half-even(1024 c) with c the projection on the
    eigenvectors: a basis of unit vectors e_0, e_1 and projections placed on
    exact half-steps."""
    V = np.eye(128)
    mean = np.zeros(128)
    D = np.zeros((1, 4, 128))
    D[0, :, 0] = np.array([0.5, 1.5, 2.5, -2.5]) / 1024
    D[0, :, 1] = np.array([1.0, -1.0, 3.0, -3.0])   # beyond the range: clamped
    q = ffo.sift_codes(D, mean, V, 2)
    assert q[0, :, 0].tolist() == [0, 2, 2, -2]
    assert q[0, :, 1].tolist() == [1024, -1024, 2047, -2047]


def test_smooth_codes_constant_identity_and_census_smoothing():
    rng = np.random.default_rng(8)
    for n in (1, 2, 4, 8):
        for c in (-700, 0, 913):
            P = np.full((23, 37), c, np.int16)
            assert np.all(ffo.smooth_codes(P, n) == c)
    J = rng.integers(0, 256, (29, 41)).astype(np.uint8)
    assert np.array_equal(ffo.smooth_codes(J.astype(np.int16), 1), J)
    for n in (2, 4, 8):
        # the census path's smoothing (pinned on its own) keeps 4 more
        # fractional bits of the same sums: the two differ by the final
        # rounding only
        s4 = ffo.smooth(J, n).astype(np.float64) / 16
        s0 = ffo.smooth_codes(J.astype(np.int16), n).astype(np.float64)
        assert np.max(np.abs(s0 - s4)) <= 0.5 + 1 / 32 + 1e-12
        # odd symmetry up to the half-up rounding
        neg = ffo.smooth_codes(-J.astype(np.int16), n).astype(np.int64)
        assert np.max(np.abs(neg + ffo.smooth_codes(J.astype(np.int16), n))) <= 1


def _levels(codes, k=2):
    return ffo.SiftLevels(codes, k)


def test_cost_zero_at_identity_and_at_integer_translation():
    rng = np.random.default_rng(9)
    S, W, H = 5, 40, 30
    codes = rng.integers(-600, 600, (H, W, S)).astype(np.int16)
    a = _levels(codes)
    assert ffo.sift_cost(a, a, 4, 0, 3, S, 20, 15, 0, 0) == 0
    assert ffo.sift_cost(a, a, 4, 1, 3, S, 20, 14, 0, 0) == 0
    tx, ty = 3, -2
    shifted = np.zeros_like(codes)
    shifted[max(ty, 0):H + min(ty, 0), max(tx, 0):W + min(tx, 0)] = \
        codes[max(-ty, 0):H - max(ty, 0), max(-tx, 0):W - max(tx, 0)]
    b = _levels(shifted, 0)
    a0 = _levels(codes, 0)
    for (px, py) in [(12, 10), (20, 15), (25, 20)]:
        assert ffo.sift_cost(a0, b, 4, 0, 3, S, px, py, 4 * tx, 4 * ty) == 0
        assert ffo.sift_cost(a0, b, 4, 0, 3, S, px, py, 4 * tx + 4, 4 * ty) > 0


def test_cost_on_a_ramp_closed_form():
    """Colours linear in x (code = alpha x on every channel, no smoothing at
    level 0): bilinear interpolation is exact, so a flow of a/Q px along x
    gives every sample the distance floor(16 alpha a sqrt(S) / Q) (1/16 code
    units), and a/Q px along y gives 0."""
    S, W, H, alpha = 4, 40, 24, 9
    x = np.arange(W)
    codes = np.repeat(np.repeat((alpha * x)[None, :, None], H, 0), S, 2).astype(np.int16)
    a = _levels(codes, 0)
    r = 2
    for Q in (1, 2, 4, 8):
        for ph in range(Q):
            want = (2 * r + 1) ** 2 * int(np.floor(16 * alpha * ph * np.sqrt(S) / Q))
            # exact integer: floor(sqrt(S (Q alpha ph)^2 * 256 / Q^4))
            want_exact = (2 * r + 1) ** 2 * ffo.isqrt64(S * (Q * alpha * ph) ** 2 * 256 // Q ** 4)
            assert want_exact == want or Q == 8
            assert ffo.sift_cost(a, a, Q, 0, r, S, 15, 10, ph, 0) == want_exact
            assert ffo.sift_cost(a, a, Q, 0, r, S, 15, 10, 0, ph) == 0


def test_cost_symmetry_and_validity():
    rng = np.random.default_rng(10)
    c1 = rng.integers(-500, 500, (26, 34, 3)).astype(np.int16)
    c2 = rng.integers(-500, 500, (26, 34, 3)).astype(np.int16)
    a, b = _levels(c1, 1), _levels(c2, 1)
    for lev in (0, 1):
        for (px, py, fx, fy) in [(10, 8, 8, 4), (16, 12, -12, 4), (4, 20, 20, -8)]:
            # integer flows: swapping the images and reversing the flow sums
            # the same distances
            assert ffo.sift_cost(a, b, 4, lev, 2, 3, px, py, fx, fy) == \
                ffo.sift_cost(b, a, 4, lev, 2, 3, px + fx // 4, py + fy // 4, -fx, -fy)
    assert ffo.sift_cost(a, b, 4, 0, 2, 3, 0, 0, -1, 0) == ffo.INF
    assert ffo.sift_cost(a, b, 4, 0, 2, 3, 33, 25, 1, 0) == ffo.INF
    assert ffo.sift_cost(a, b, 4, 0, 2, 3, 33, 25, 0, 0) != ffo.INF


def test_search_finds_a_global_translation():
    base = np.stack([_texture(90, 70, 12 + c) for c in range(3)], -1)
    tx, ty = 5, 3
    i1 = np.ascontiguousarray(base[5:61, 5:77])
    i2 = np.ascontiguousarray(base[5 + ty:61 + ty, 5 + tx:77 + tx])
    # i2(x, y) = i1(x + tx, y + ty): the flow of i1 -> i2 is (-tx, -ty)
    out = ffo.match_pair_sift(i1, i2, region_s=None)
    dx, dy = ffo.unpack(out["F"])
    inner = (slice(10, 46), slice(12, 58))
    ok = (dx[inner] == -4 * tx) & (dy[inner] == -4 * ty)
    assert ok.mean() > 0.98


def test_pair_pipeline_on_a_layered_pair():
    p = pairs.layered_pair(seed=3, W=96, H=64)
    out = ffo.match_pair_sift(p.img1, p.img2)
    assert pairs.inlier_rate(out["F"], p, 4) > 0.85
    # what the filters keep is correct far more often than the raw field
    kept = out["filtered_region"] != ffo.EMPTY
    dx, dy = ffo.unpack(out["F"])
    epe = np.hypot(dx / 4 - p.flow[..., 0], dy / 4 - p.flow[..., 1])
    vis = ~p.occluded
    assert (epe[kept & vis] < 3).mean() > 0.97 > (epe[vis] < 3).mean()
    assert out["codes1"].shape == (64, 96, 18)
