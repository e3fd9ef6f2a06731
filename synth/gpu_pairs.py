"""Batched, device-side generator of the Sintel-shaped layered recipe (the
same recipe as ``pairs.layered_pair``: 1/f background with a small affine
motion plus star-polygon layers with affine motions, frame-2 gain and
Gaussian noise), used to produce training pairs for the learned proposal in
bulk.  Like ``pairs``, it holds none of the matching method's arithmetic.

Differences from the NumPy generator (the training set only needs the
distribution, not the NumPy generator's exact pixels): the noise comes from a
torch device generator, the 1st/99th texture percentiles are taken on a 1/16
subsample, and the arithmetic is float32.  Evaluation pairs always come from
``pairs`` (seeded NumPy), with disjoint seeds.
"""
from __future__ import annotations

import math

import numpy as np
import torch

MAX_T = 200.0
MAX_VERTS = 11


def _textures(gen, n, h, w, device):
    """n x h x w x 3 float32 1/f-noise textures stretched to [0, 255]."""
    ky = torch.fft.fftfreq(h, device=device)[:, None] * h
    kx = torch.fft.rfftfreq(w, device=device)[None, :] * w
    amp = 1.0 / torch.clamp(torch.sqrt(kx * kx + ky * ky), min=1.0)
    out = torch.empty((n, h, w, 3), dtype=torch.float32, device=device)
    for c in range(3):
        noise = torch.randn((n, h, w), generator=gen, device=device)
        t = torch.fft.irfft2(torch.fft.rfft2(noise) * amp, s=(h, w))
        sub = t[:, ::4, ::4].reshape(n, -1)
        q = torch.quantile(sub, torch.tensor([0.01, 0.99], device=device), dim=1)
        lo, hi = q[0][:, None, None], q[1][:, None, None]
        out[..., c] = torch.clamp((t - lo) * (255.0 / torch.clamp(hi - lo, min=1e-12)), 0.0, 255.0)
    return out


def _affine_params(cx, cy, tx, ty, rot_deg, scale):
    th = math.radians(rot_deg)
    a, b = scale * math.cos(th), -scale * math.sin(th)
    c, d = scale * math.sin(th), scale * math.cos(th)
    return [cx, cy, tx, ty, a, b, c, d]


def _draw_layers(rng, W, H, nlayers, motion="uniform"):
    """Host-side draws for one pair: affine params (L x 8), polygons
    (L x MAX_VERTS x 2, padded with the first vertex; layer 0 = background),
    vertex counts, gain."""
    aff = [_affine_params(W / 2, H / 2, rng.uniform(-10, 10), rng.uniform(-10, 10), rng.uniform(-2, 2),
                          rng.uniform(0.97, 1.03))]
    polys = [np.zeros((MAX_VERTS, 2))]
    for _ in range(nlayers):
        frac = rng.uniform(0.05, 0.30)
        mean_r = math.sqrt(frac * W * H / math.pi)
        cx = rng.uniform(0.1 * W, 0.9 * W)
        cy = rng.uniform(0.1 * H, 0.9 * H)
        nv = int(rng.integers(5, 12))
        ang = np.sort(rng.uniform(0.0, 2 * math.pi, nv))
        rad = mean_r * rng.uniform(0.55, 1.45, nv)
        p = np.stack([cx + rad * np.cos(ang), cy + rad * np.sin(ang)], 1)
        p = np.concatenate([p, np.repeat(p[:1], MAX_VERTS - nv, 0)], 0)
        polys.append(p)
        ux, uy, vx, vy = rng.uniform(-1, 1, 4)
        tx, ty = (MAX_T * ux, MAX_T * uy) if motion == "uniform" else (MAX_T * ux * vx * vx, MAX_T * uy * vy * vy)
        aff.append(_affine_params(cx, cy, tx, ty, rng.uniform(-5, 5), rng.uniform(0.9, 1.1)))
    gain = rng.uniform(0.9, 1.1)
    return np.array(aff), np.stack(polys), gain


def _inside(poly, xs, ys):
    """Even-odd crossing test.  poly: B x V x 2; xs, ys: B x N -> B x N bool."""
    px, py = poly[..., 0:1], poly[..., 1:2]
    qx, qy = torch.roll(poly[..., 0], -1, 1)[..., None], torch.roll(poly[..., 1], -1, 1)[..., None]
    res = torch.zeros(xs.shape, dtype=torch.bool, device=xs.device)
    for i in range(poly.shape[1]):
        x0, y0, x1, y1 = px[:, i], py[:, i], qx[:, i], qy[:, i]
        dy = y1 - y0
        live = dy != 0
        cond = ((y0 > ys) != (y1 > ys)) & live
        xint = x0 + (ys - y0) * (x1 - x0) / torch.where(live, dy, torch.ones_like(dy))
        res ^= cond & (xs < xint)
    return res


def layered_batch(seeds, W=1024, H=436, nlayers=6, device="cuda", motion="uniform"):
    """len(seeds) pairs (B x H x W x 3 uint8 each) plus their ground-truth
    flow (B x H x W x 2 float32); motion as in synth.pairs.layered_pair."""
    B, L = len(seeds), nlayers + 1
    m = int(MAX_T) + 64
    hc, wc = H + 2 * m, W + 2 * m
    draws = [_draw_layers(np.random.default_rng(s), W, H, nlayers, motion) for s in seeds]
    aff = torch.tensor(np.stack([d[0] for d in draws]), dtype=torch.float32, device=device)     # B L 8
    polys = torch.tensor(np.stack([d[1] for d in draws]), dtype=torch.float32, device=device)   # B L V 2
    gain = torch.tensor([d[2] for d in draws], dtype=torch.float32, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seeds[0]) * 1000003 + B)
    ys, xs = torch.meshgrid(torch.arange(H, device=device, dtype=torch.float32),
                            torch.arange(W, device=device, dtype=torch.float32), indexing="ij")
    xs = xs.reshape(1, -1).expand(B, -1)
    ys = ys.reshape(1, -1).expand(B, -1)
    N = H * W
    owner1 = torch.zeros((B, N), dtype=torch.long, device=device)
    owner2 = torch.zeros((B, N), dtype=torch.long, device=device)
    pre = []
    for li in range(L):
        cx, cy, tx, ty, a, b, c, d = [aff[:, li, j:j + 1] for j in range(8)]
        det = a * d - b * c
        ix = (d * (xs - cx - tx) - b * (ys - cy - ty)) / det + cx
        iy = (-c * (xs - cx - tx) + a * (ys - cy - ty)) / det + cy
        pre.append((ix, iy))
        if li > 0:
            owner1[_inside(polys[:, li], xs, ys)] = li
            owner2[_inside(polys[:, li], ix, iy)] = li
    img1 = torch.zeros((B, N, 3), dtype=torch.float32, device=device)
    img2 = torch.zeros((B, N, 3), dtype=torch.float32, device=device)
    flow = torch.zeros((B, N, 2), dtype=torch.float32, device=device)
    xi = xs.long() + m
    yi = ys.long() + m
    for li in range(L):
        tex = _textures(gen, B, hc, wc, device).reshape(B, hc * wc, 3)
        sel1 = owner1 == li
        v1 = torch.gather(tex, 1, (yi * wc + xi).unsqueeze(-1).expand(-1, -1, 3))
        img1 = torch.where(sel1.unsqueeze(-1), v1, img1)
        cx, cy, tx, ty, a, b, c, d = [aff[:, li, j:j + 1] for j in range(8)]
        fx = a * (xs - cx) + b * (ys - cy) + cx + tx
        fy = c * (xs - cx) + d * (ys - cy) + cy + ty
        flow = torch.where(sel1.unsqueeze(-1), torch.stack([fx - xs, fy - ys], -1), flow)
        ix, iy = pre[li]
        sx = torch.clamp(ix + m, 0.0, wc - 1.0)
        sy = torch.clamp(iy + m, 0.0, hc - 1.0)
        x0 = torch.clamp(torch.floor(sx).long(), max=wc - 2)
        y0 = torch.clamp(torch.floor(sy).long(), max=hc - 2)
        ax = (sx - x0).unsqueeze(-1)
        ay = (sy - y0).unsqueeze(-1)

        def g(yy, xx):
            return torch.gather(tex, 1, (yy * wc + xx).unsqueeze(-1).expand(-1, -1, 3))

        v2 = (g(y0, x0) * (1 - ax) + g(y0, x0 + 1) * ax) * (1 - ay) + (g(y0 + 1, x0) * (1 - ax) +
                                                                       g(y0 + 1, x0 + 1) * ax) * ay
        img2 = torch.where((owner2 == li).unsqueeze(-1), v2, img2)
        del tex
    img2 = img2 * gain[:, None, None] + torch.randn(img2.shape, generator=gen, device=device) * 2.0
    i1 = torch.clamp(torch.round(img1), 0, 255).to(torch.uint8).reshape(B, H, W, 3).contiguous()
    i2 = torch.clamp(torch.round(img2), 0, 255).to(torch.uint8).reshape(B, H, W, 3).contiguous()
    return i1, i2, flow.reshape(B, H, W, 2)
