"""Seeded synthetic image pairs with ground-truth flow.

This module only draws inputs: textures, layer shapes, motions, noise, and the
ground-truth flow / occlusion mask implied by them.  It holds none of the
matching method's arithmetic (no colour conversion, smoothing, census, WHT,
search or filtering), so both the CPU oracle and the GPU path can take their
inputs from here without sharing any code with each other.

Every pair is rendered from layers, back to front:

* each layer owns a 1/f-noise texture on a canvas larger than the image (so
  that regions moved in from outside the frame still have texture), a mask in
  frame-1 coordinates and an affine motion ``x -> A (x - c) + c + t`` about
  its centroid ``c``;
* frame 1 samples each texture at integer positions;
* frame 2 inverts each layer's motion and samples the texture bilinearly in
  float64; the top-most layer whose mask contains the pre-image wins;
* the ground-truth flow of a frame-1 pixel is the motion of the top-most layer
  covering it; it is occluded when its target leaves the image or is covered
  by another layer in frame 2;
* frame 2 gets a brightness gain (where the recipe asks for one), then
  Gaussian noise, then rounding and clamping to uint8.

Recipes (shapes and distributions of the paper's workloads, with synthetic
content standing in for MPI-Sintel, KITTI and Middlebury, none of which is
used): ``square_pair`` (128x96), ``layered_pair`` (Sintel-shaped 1024x436),
``driving_pair`` (KITTI-shaped 1242x375 gray), ``mixed_pairs`` (mixed sizes)
and ``layered_pairs`` (batches of layered pairs).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Pair",
    "square_pair",
    "layered_pair",
    "driving_pair",
    "mixed_pairs",
    "layered_pairs",
    "inlier_rate",
]


@dataclasses.dataclass
class Pair:
    img1: np.ndarray          # H x W x C uint8
    img2: np.ndarray          # H x W x C uint8
    flow: np.ndarray          # H x W x 2 float32, frame-1 pixel -> frame-2 offset (dx, dy)
    occluded: np.ndarray      # H x W bool
    seed: int
    recipe: str

    @property
    def shape(self):
        return self.img1.shape[1], self.img1.shape[0]


# --------------------------------------------------------------------------
# textures

def _texture(rng: np.random.Generator, h: int, w: int, channels: int, beta: float = 1.0) -> np.ndarray:
    """1/f^beta noise (beta = 1 unless a recipe asks for smoother textures):
    white noise -> FFT -> amplitude * 1/max(|k|,1)^beta -> inverse FFT ->
    stretch the 1st..99th percentile to [0, 255] (float64)."""
    out = np.empty((h, w, channels), np.float64)
    ky = np.fft.fftfreq(h)[:, None] * h
    kx = np.fft.rfftfreq(w)[None, :] * w
    amp = 1.0 / np.maximum(np.sqrt(kx * kx + ky * ky), 1.0) ** beta
    for c in range(channels):
        noise = rng.standard_normal((h, w))
        spec = np.fft.rfft2(noise) * amp
        t = np.fft.irfft2(spec, s=(h, w))
        lo, hi = np.percentile(t, [1.0, 99.0])
        t = (t - lo) * (255.0 / max(hi - lo, 1e-12))
        out[:, :, c] = np.clip(t, 0.0, 255.0)
    return out


def _bilinear(tex: np.ndarray, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """Sample tex (h x w x C) at float positions with clamped bilinear."""
    h, w = tex.shape[:2]
    xs = np.clip(xs, 0.0, w - 1.0)
    ys = np.clip(ys, 0.0, h - 1.0)
    x0 = np.minimum(np.floor(xs).astype(np.int64), w - 2 if w > 1 else 0)
    y0 = np.minimum(np.floor(ys).astype(np.int64), h - 2 if h > 1 else 0)
    fx = (xs - x0)[..., None]
    fy = (ys - y0)[..., None]
    x1 = np.minimum(x0 + 1, w - 1)
    y1 = np.minimum(y0 + 1, h - 1)
    a = tex[y0, x0]
    b = tex[y0, x1]
    c = tex[y1, x0]
    d = tex[y1, x1]
    return (a * (1 - fx) + b * fx) * (1 - fy) + (c * (1 - fx) + d * fx) * fy


# --------------------------------------------------------------------------
# layers

@dataclasses.dataclass
class _Layer:
    tex: np.ndarray                 # canvas texture (H + 2m) x (W + 2m) x C
    margin: int
    inside: callable                # (xs, ys) float arrays in frame-1 coords -> bool
    fwd: callable                   # frame-1 coords -> frame-2 coords
    inv: callable                   # frame-2 coords -> frame-1 coords


def _affine(cx, cy, tx, ty, rot_deg, scale):
    th = math.radians(rot_deg)
    a = scale * math.cos(th)
    b = -scale * math.sin(th)
    c = scale * math.sin(th)
    d = scale * math.cos(th)
    det = a * d - b * c

    def fwd(xs, ys):
        dx, dy = xs - cx, ys - cy
        return a * dx + b * dy + cx + tx, c * dx + d * dy + cy + ty

    def inv(xs, ys):
        dx, dy = xs - cx - tx, ys - cy - ty
        return (d * dx - b * dy) / det + cx, (-c * dx + a * dy) / det + cy

    return fwd, inv


def _star_polygon(rng, cx, cy, mean_r, nverts):
    ang = np.sort(rng.uniform(0.0, 2 * math.pi, nverts))
    rad = mean_r * rng.uniform(0.55, 1.45, nverts)
    return np.stack([cx + rad * np.cos(ang), cy + rad * np.sin(ang)], 1)


def _polygon_inside(poly: np.ndarray):
    px = poly[:, 0]
    py = poly[:, 1]
    qx = np.roll(px, -1)
    qy = np.roll(py, -1)

    def inside(xs, ys):
        res = np.zeros(xs.shape, bool)
        for i in range(len(px)):
            x0, y0, x1, y1 = px[i], py[i], qx[i], qy[i]
            if y0 == y1:
                continue
            cond = (y0 > ys) != (y1 > ys)
            xint = x0 + (ys - y0) * (x1 - x0) / (y1 - y0)
            res ^= cond & (xs < xint)
        return res

    return inside


def _rect_inside(x0, y0, w, h):
    def inside(xs, ys):
        return (xs >= x0) & (xs < x0 + w) & (ys >= y0) & (ys < y0 + h)
    return inside


def _render(layers, W, H, channels, rng, noise_sigma, gain, seed, recipe,
            flat_blobs=None) -> Pair:
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    # frame 1: top-most layer at identity
    owner1 = np.full((H, W), -1, np.int64)
    for li, L in enumerate(layers):
        owner1[L.inside(xs, ys)] = li
    img1 = np.zeros((H, W, channels), np.float64)
    flow = np.zeros((H, W, 2), np.float64)
    for li, L in enumerate(layers):
        m = owner1 == li
        if not m.any():
            continue
        img1[m] = L.tex[ys[m].astype(np.int64) + L.margin, xs[m].astype(np.int64) + L.margin]
        fx, fy = L.fwd(xs[m], ys[m])
        flow[m, 0] = fx - xs[m]
        flow[m, 1] = fy - ys[m]
    # frame 2: invert each layer's motion
    owner2 = np.full((H, W), -1, np.int64)
    img2 = np.zeros((H, W, channels), np.float64)
    pre = []
    for li, L in enumerate(layers):
        ix, iy = L.inv(xs, ys)
        pre.append((ix, iy))
        owner2[L.inside(ix, iy)] = li
    for li, L in enumerate(layers):
        m = owner2 == li
        if not m.any():
            continue
        ix, iy = pre[li]
        img2[m] = _bilinear(L.tex, ix[m] + L.margin, iy[m] + L.margin)
    # occlusion: target out of image, or covered by another layer in frame 2
    tx = xs + flow[..., 0]
    ty = ys + flow[..., 1]
    out = (tx < 0) | (ty < 0) | (tx > W - 1) | (ty > H - 1)
    txi = np.clip(np.rint(tx), 0, W - 1).astype(np.int64)
    tyi = np.clip(np.rint(ty), 0, H - 1).astype(np.int64)
    occ = out | (owner2[tyi, txi] != owner1)
    if gain is not None:
        img2 = img2 * gain
    img1 = img1 + 0.0
    img2 = img2 + rng.standard_normal(img2.shape) * noise_sigma
    i1 = np.clip(np.rint(img1), 0, 255).astype(np.uint8)
    i2 = np.clip(np.rint(img2), 0, 255).astype(np.uint8)
    return Pair(i1, i2, flow.astype(np.float32), occ, seed, recipe)


def _flatten_blobs(rng, tex, frac, margin, W, H):
    """Paint constant-colour discs into a texture until about `frac` of the
    visible frame area is flat (low-texture regions)."""
    h, w, _ = tex.shape
    yy, xx = np.mgrid[0:h, 0:w]
    target = frac * W * H
    area = 0.0
    while area < target:
        r = rng.uniform(8, 30)
        cx = rng.uniform(margin, margin + W)
        cy = rng.uniform(margin, margin + H)
        m = (xx - cx) ** 2 + (yy - cy) ** 2 < r * r
        tex[m] = rng.uniform(20, 235)
        area += math.pi * r * r
    return tex


# --------------------------------------------------------------------------
# recipes

def square_pair(seed: int = 0) -> Pair:
    """128x96 RGB: 1/f background moving (+7,-3), a 24x24 square on top
    moving (+18,+11), frame-2 noise sigma = 2."""
    rng = np.random.default_rng(seed)
    W, H, C, m = 128, 96, 3, 64
    bg = _texture(rng, H + 2 * m, W + 2 * m, C)
    sq = _texture(rng, H + 2 * m, W + 2 * m, C)
    x0 = rng.integers(20, W - 24 - 30)
    y0 = rng.integers(15, H - 24 - 25)
    fb, ib = _affine(0, 0, 7.0, -3.0, 0.0, 1.0)
    fs, is_ = _affine(0, 0, 18.0, 11.0, 0.0, 1.0)
    layers = [
        _Layer(bg, m, lambda xs, ys: np.ones(xs.shape, bool), fb, ib),
        _Layer(sq, m, _rect_inside(x0, y0, 24, 24), fs, is_),
    ]
    return _render(layers, W, H, C, rng, 2.0, None, seed, "square")


def _affine_layers_pair(rng, W, H, C, nlayers, seed, recipe, noise, gain_range,
                        max_t=200.0, max_rot=5.0, scale=(0.9, 1.1), motion="skewed", beta=1.0):
    m = int(max_t) + 64
    layers = []
    bg = _texture(rng, H + 2 * m, W + 2 * m, C, beta)
    f, i = _affine(W / 2, H / 2, rng.uniform(-10, 10), rng.uniform(-10, 10),
                   rng.uniform(-2, 2), rng.uniform(0.97, 1.03))
    layers.append(_Layer(bg, m, lambda xs, ys: np.ones(xs.shape, bool), f, i))
    for _ in range(nlayers):
        tex = _texture(rng, H + 2 * m, W + 2 * m, C, beta)
        frac = rng.uniform(0.05, 0.30)
        mean_r = math.sqrt(frac * W * H / math.pi)
        cx = rng.uniform(0.1 * W, 0.9 * W)
        cy = rng.uniform(0.1 * H, 0.9 * H)
        poly = _star_polygon(rng, cx, cy, mean_r, int(rng.integers(5, 12)))
        # translation up to max_t per axis: uniform on [-max_t, max_t]
        # ("uniform"), or skewed towards small motions (max_t * u * v^2,
        # u, v ~ U(-1, 1): "skewed"); the same four draws either way
        ux, uy, vx, vy = rng.uniform(-1, 1, 4)
        if motion == "uniform":
            tx, ty = max_t * ux, max_t * uy
        else:
            tx, ty = max_t * ux * vx * vx, max_t * uy * vy * vy
        f, i = _affine(cx, cy, tx, ty, rng.uniform(-max_rot, max_rot), rng.uniform(*scale))
        layers.append(_Layer(tex, m, _polygon_inside(poly), f, i))
    gain = None if gain_range is None else rng.uniform(*gain_range)
    return _render(layers, W, H, C, rng, noise, gain, seed, recipe)


def layered_pair(seed: int = 1000, W: int = 1024, H: int = 436, nlayers: int = 6, motion: str = "uniform",
                 noise: float = 2.0, beta: float = 1.0) -> Pair:
    """Sintel-shaped RGB pair: 1/f background (translation U(+-10), rotation
    U(+-2 deg), scale U(0.97, 1.03)) plus `nlayers` star polygons of 5..30 %
    area, each with an affine motion about its centroid (translation
    U(+-200) per axis, or with motion="skewed" 200 u v^2 with u, v ~ U(-1, 1),
    which keeps occlusion nearer a tenth of the frame; rotation U(+-5 deg),
    scale U(0.9, 1.1)); frame-2 gain U(0.9, 1.1) and Gaussian noise of
    standard deviation `noise` (2 in the benchmark recipe).  beta > 1 gives
    smoother 1/f^beta textures (small patches become ambiguous)."""
    rng = np.random.default_rng(seed)
    return _affine_layers_pair(rng, W, H, 3, nlayers, seed, "layered", noise, (0.9, 1.1), motion=motion,
                               beta=beta)


def driving_pair(seed: int = 2000, W: int = 1242, H: int = 375) -> Pair:
    """KITTI-shaped gray pair: radial expansion from a random vanishing point,
    |flow| growing linearly along each ray to 250 px at the border; three
    60..150 px rectangles translating U(+-80); about 5 % flat blobs; noise
    sigma = 3."""
    rng = np.random.default_rng(seed)
    C = 1
    m = 300
    vx = rng.uniform(0.3 * W, 0.7 * W)
    vy = rng.uniform(0.3 * H, 0.7 * H)

    def ray_len(dx, dy):
        # distance from v to the image border along direction (dx, dy)
        with np.errstate(divide="ignore", invalid="ignore"):
            tx = np.where(dx > 0, (W - 1 - vx) / dx, np.where(dx < 0, -vx / dx, np.inf))
            ty = np.where(dy > 0, (H - 1 - vy) / dy, np.where(dy < 0, -vy / dy, np.inf))
        t = np.minimum(tx, ty)
        return np.where(np.isfinite(t), t * np.hypot(dx, dy), 1.0)

    def fwd(xs, ys):
        dx, dy = xs - vx, ys - vy
        L = np.maximum(ray_len(dx, dy), 1.0)
        k = 1.0 + 250.0 / L
        return vx + dx * k, vy + dy * k

    def inv(xs, ys):
        dx, dy = xs - vx, ys - vy
        L = np.maximum(ray_len(dx, dy), 1.0)
        k = 1.0 + 250.0 / L
        return vx + dx / k, vy + dy / k

    bg = _texture(rng, H + 2 * m, W + 2 * m, C)
    bg = _flatten_blobs(rng, bg, 0.035, m, W, H)
    layers = [_Layer(bg, m, lambda xs, ys: np.ones(xs.shape, bool), fwd, inv)]
    for _ in range(3):
        tex = _texture(rng, H + 2 * m, W + 2 * m, C)
        tex = _flatten_blobs(rng, tex, 0.005, m, W, H)
        rw, rh = rng.uniform(60, 150, 2)
        x0 = rng.uniform(0, W - rw)
        y0 = rng.uniform(0, H - rh)
        f, i = _affine(0, 0, rng.uniform(-80, 80), rng.uniform(-80, 80), 0.0, 1.0)
        layers.append(_Layer(tex, m, _rect_inside(x0, y0, rw, rh), f, i))
    return _render(layers, W, H, C, rng, 3.0, None, seed, "driving")


MIXED_SIZES = ((320, 240), (640, 480), (1024, 436), (1242, 375))


def mixed_pairs(n_pairs: int = 64, seed0: int = 3000, sizes=MIXED_SIZES):
    """Mixed-size batch: sizes uniform over `sizes`, 2..8 affine layers each
    (layered recipe, RGB, translations U(+-min(200, W / 5)))."""
    out = []
    for i in range(n_pairs):
        seed = seed0 + i
        rng = np.random.default_rng(seed)
        W, H = sizes[int(rng.integers(0, len(sizes)))]
        nl = int(rng.integers(2, 9))
        out.append(_affine_layers_pair(rng, W, H, 3, nl, seed, "mixed", 2.0, (0.9, 1.1),
                                       max_t=min(200.0, 0.2 * W), motion="uniform"))
    return out


def _mixed_one(args):
    i, seed0, sizes = args
    return mixed_pairs(1, seed0 + i, sizes)[0]


def mixed_pairs_parallel(n_pairs: int = 64, seed0: int = 3000, sizes=MIXED_SIZES, workers: int = 8):
    """mixed_pairs with the pairs drawn in a process pool (same bytes:
    pair i only depends on its own seed seed0 + i)."""
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(_mixed_one, [(i, seed0, sizes) for i in range(n_pairs)])


def driving_pairs(first_seed: int, count: int = 8, workers: int = 0):
    """`count` KITTI-shaped pairs with seeds first_seed .. first_seed + count - 1."""
    seeds = [first_seed + i for i in range(count)]
    if workers <= 0:
        return [driving_pair(s) for s in seeds]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(min(workers, count)) as pool:
        return pool.map(driving_pair, seeds)


def mixed_pairs_subset(indices, seed0: int = 3000, sizes=MIXED_SIZES, workers: int = 8):
    """Pairs `indices` of the mixed-size batch (pair i depends only on its
    seed seed0 + i), drawn in a process pool when workers > 0."""
    args = [(i, seed0, sizes) for i in indices]
    if workers <= 0:
        return [_mixed_one(a) for a in args]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(min(workers, len(args))) as pool:
        return pool.map(_mixed_one, args)


def layered_pairs(first_seed: int, count: int = 16, W: int = 1024, H: int = 436, workers: int = 0,
                  motion: str = "uniform", noise: float = 2.0, beta: float = 1.0):
    """`count` layered pairs with seeds first_seed .. first_seed + count - 1
    (drawn in a process pool when workers > 0; same bytes either way)."""
    args = [(first_seed + i, W, H, 6, motion, noise, beta) for i in range(count)]
    if workers <= 0:
        return [layered_pair(*a) for a in args]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(min(workers, count)) as pool:
        return pool.starmap(layered_pair, args)


def inlier_rate(flow_q: np.ndarray, gt: Pair, Q: int, thresh_px: float = 3.0,
                empty: int = -2147450880):
    """Fraction of non-occluded pixels whose flow (packed int16x2 in 1/Q px,
    EMPTY counted as wrong) has an end-point error below thresh_px."""
    f = flow_q.astype(np.int64) & 0xFFFFFFFF
    dx = ((f & 0xFFFF) ^ 0x8000) - 0x8000
    dy = (((f >> 16) & 0xFFFF) ^ 0x8000) - 0x8000
    valid = flow_q != empty
    epe = np.hypot(dx / Q - gt.flow[..., 0], dy / Q - gt.flow[..., 1])
    ok = valid & (epe < thresh_px) & ~gt.occluded
    nocc = ~gt.occluded
    return float(ok.sum()) / max(int(nocc.sum()), 1)
