"""Pins of the smoothed images I^n (section 3.2: area downsampling by n, then
Lanczos upsampling) and of the census planes of the data term (section 3.3)
on subsampled patches (Eq. 3) at subpixel phases (section 3.1)."""
import numpy as np
import pytest

from oracle import ffo


def _lanczos3(t):
    t = np.asarray(t, np.float64)
    out = np.where(np.abs(t) < 3, np.sinc(t) * np.sinc(t / 3.0), 0.0)
    return out


def _smooth_float(J, n):
    """Float64 area-downsample (replicate pad to a multiple of n) then
    Lanczos-3 upsample with pixel-centre alignment and replicate borders,
    written with NumPy array operations.  The continuous taps do not sum to
    one; as in the reading taken, the shortfall goes to the centre tap."""
    H, W = J.shape
    Hc, Wc = -(-H // n), -(-W // n)
    P = np.pad(J.astype(np.float64), ((0, Hc * n - H), (0, Wc * n - W)), mode="edge")
    A = P.reshape(Hc, n, Wc, n).mean(axis=(1, 3))

    def up(axis_len, coarse_len):
        u = (np.arange(axis_len) + 0.5) / n - 0.5
        base = np.floor(np.arange(axis_len) / n).astype(int)
        M = np.zeros((axis_len, coarse_len))
        wsum = np.zeros(axis_len)
        for k in range(-3, 4):
            wsum += _lanczos3(u - (base + k))
        for k in range(-3, 4):
            idx = np.clip(base + k, 0, coarse_len - 1)
            w = _lanczos3(u - (base + k)) + (1.0 - wsum if k == 0 else 0.0)
            np.add.at(M, (np.arange(axis_len), idx), w)
        return M

    My = up(H, Hc)
    Mx = up(W, Wc)
    return My @ A @ Mx.T


@pytest.mark.parametrize("n", [2, 4, 8])
def test_lanczos_weights_partition_of_unity_and_symmetry(n):
    w = ffo.lanczos_weights(n)
    assert np.all(w.sum(1) == 16384)
    # phase ph at offset t0 mirrors phase n-1-ph at -t0
    assert np.array_equal(w, w[::-1, ::-1])
    # the centre tap carries most of the weight
    assert np.all(w[:, 3] == w.max(1))


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_constant_image_exact(n):
    for c in (0, 1, 77, 255):
        J = np.full((37, 53), c, np.uint8)
        assert np.all(ffo.smooth(J, n) == 16 * c)


@pytest.mark.parametrize("n,shape", [(2, (40, 61)), (4, (45, 70)), (8, (67, 99))])
def test_smooth_matches_float_definition(n, shape):
    rng = np.random.default_rng(n)
    J = rng.integers(0, 256, shape).astype(np.uint8)
    S = ffo.smooth(J, n).astype(np.float64) / 16.0
    ref = _smooth_float(J, n)
    # error bound in Q4 codes: the horizontal pass rounds to whole block-sum
    # units (+-1/2, i.e. 16/(2 n^2) codes, amplified by the vertical taps'
    # absolute sum), the output rounds (+-1/2), and the Q14 tap rounding adds
    # at most 7 * 2^-15 * 255 * 16 * 2 < 0.25
    w = ffo.lanczos_weights(n)
    amp = np.abs(w).sum(1).max() / 16384.0
    bound = 0.5 * 16.0 / (n * n) * amp + 0.5 + 0.25
    assert np.max(np.abs(S - ref)) * 16 <= bound


def _census_upsampled(S, n, Q, a, b):
    """Census at (XQ + a, YQ + b) of the Q-times bilinearly upsampled image,
    neighbours nQ apart in the upsampled grid.  Interior pixels only."""
    C, H, W = S.shape
    ys = np.arange(H * Q) / Q
    xs = np.arange(W * Q) / Q
    y0 = np.minimum(np.floor(ys).astype(int), H - 1)
    x0 = np.minimum(np.floor(xs).astype(int), W - 1)
    fy = (ys - y0)[:, None]
    fx = (xs - x0)[None, :]
    y1 = np.minimum(y0 + 1, H - 1)
    x1 = np.minimum(x0 + 1, W - 1)
    out = np.zeros((H, W), np.uint64)
    for c in range(C):
        P = S[c].astype(np.float64)
        U = (P[y0][:, x0] * (1 - fx) * (1 - fy) + P[y0][:, x1] * fx * (1 - fy) +
             P[y1][:, x0] * (1 - fx) * fy + P[y1][:, x1] * fx * fy)
        cy = np.arange(H) * Q + b
        cx = np.arange(W) * Q + a
        bit = 0
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == 0 and dy == 0:
                    continue
                yy = np.clip(cy + dy * n * Q, 0, H * Q - 1)
                xx = np.clip(cx + dx * n * Q, 0, W * Q - 1)
                lt = U[yy][:, xx] < U[cy][:, cx]
                out |= lt.astype(np.uint64) << np.uint64(8 * c + bit)
                bit += 1
    return out.astype(np.uint32)


def test_census_constant_is_zero():
    S = np.full((3, 20, 30), 1234, np.int16)
    for n in (1, 2, 4, 8):
        for a, b in ((0, 0), (1, 3), (3, 2)):
            assert np.all(ffo.census(S, n, 4, a, b) == 0)


@pytest.mark.parametrize("n", [1, 2, 4])
@pytest.mark.parametrize("ab", [(0, 0), (1, 0), (0, 3), (2, 1), (3, 3)])
def test_census_equals_upsampled_image_census(n, ab):
    a, b = ab
    Q = 4
    rng = np.random.default_rng(7 * n + a)
    S = rng.integers(0, 4080, (3, 30, 34)).astype(np.int16)
    got = ffo.census(S, n, Q, a, b)
    ref = _census_upsampled(S, n, Q, a, b)
    m = n + 1
    assert np.array_equal(got[m:-m, m:-m], ref[m:-m, m:-m])


def test_census_monotone_invariance():
    rng = np.random.default_rng(3)
    S = rng.integers(0, 2000, (3, 25, 31)).astype(np.int16)
    # strictly increasing affine maps commute with bilinear interpolation
    S2 = (3 * S.astype(np.int32) + 17).astype(np.int16)
    for n in (1, 2, 4):
        for a, b in ((0, 0), (1, 2), (3, 1)):
            assert np.array_equal(ffo.census(S, n, 4, a, b), ffo.census(S2, n, 4, a, b))
    # at phase (0,0) any strictly increasing map keeps the census
    S3 = (np.sqrt(S.astype(np.float64)) * 100).astype(np.int16)
    order_kept = np.all(np.diff(np.sort(np.unique(S))) > 0)
    assert order_kept
    uniq = np.unique(S)
    mapped = np.unique(S3)
    if len(uniq) == len(mapped):
        for n in (1, 2, 4):
            assert np.array_equal(ffo.census(S, n, 4, 0, 0), ffo.census(S3, n, 4, 0, 0))


def test_census_hand_example():
    # 3x3 gray image, centre 5; neighbours in raster order (-1,-1) .. (1,1):
    #   1 9 5
    #   7 5 2
    #   5 8 3
    # bits (neighbour < centre): 1<5:1, 9:0, 5:0, 7:0, 2:1, 5:0, 8:0, 3:1
    S = np.array([[[1, 9, 5], [7, 5, 2], [5, 8, 3]]], np.int16)
    got = ffo.census(S, 1, 4, 0, 0)
    assert got[1, 1] == 0b10010001
    # corner (0,0) with clamping: neighbours (-1,-1)->(0,0)=1, (0,-1)->1,
    # (1,-1)->(1,0)=9, (-1,0)->1, (1,0)=9, (-1,1)->(0,1)=7, (0,1)=7, (1,1)=5;
    # centre 1: nothing smaller
    assert got[0, 0] == 0
