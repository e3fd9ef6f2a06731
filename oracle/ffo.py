"""ctypes front end of the CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
module.  Arrays are NumPy host arrays; every call is single-threaded C++.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libffo.so")

EMPTY = -2147450880          # packed (dx, dy) = (-32768, -32768)
INF = 2147483647

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i32 = C.c_int
        L.ffo_lab8.argtypes = [P, i32, i32, i32, i32, P]
        L.ffo_lanczos_weights.argtypes = [i32, P]
        L.ffo_lab_tables.argtypes = [P, P, P]
        L.ffo_smooth.argtypes = [P, i32, i32, i32, P]
        L.ffo_census.argtypes = [P, i32, i32, i32, i32, i32, i32, i32, P]
        L.ffo_wht.argtypes = [P, i32, i32, i32, i32, P]
        L.ffo_walsh.argtypes = [i32, i32, i32]
        L.ffo_tree_depth.argtypes = [i32, i32]
        L.ffo_kdtree_build.argtypes = [P, i32, i32, i32, P, P, P]
        L.ffo_philox4x32_10.argtypes = [P, P, P]
        L.ffo_philox4x32_10.restype = None
        L.ffo_desc_create.argtypes = [P, i32, i32, i32, i32, i32, i32, P, i32]
        L.ffo_desc_create.restype = P
        L.ffo_desc_free.argtypes = [P]
        L.ffo_desc_free.restype = None
        L.ffo_desc_lab.argtypes = [P, P]
        L.ffo_desc_smooth.argtypes = [P, i32, P]
        L.ffo_desc_plane.argtypes = [P, i32, i32, i32, P]
        L.ffo_desc_wht.argtypes = [P, i32, P]
        L.ffo_cost.argtypes = [P, P, i32, i32, i32, i32, i32, i32]
        L.ffo_match_field.argtypes = [P, P, i32, P, P, P, P, P]
        L.ffo_consistency.argtypes = [P, i32, i32, P, i32, i32, i32, i32, i32, P, P]
        L.ffo_brute_nnf.argtypes = [P, P, i32, i32, P, P]
        L.ffo_region_filter.argtypes = [P, P, i32, i32, i32, i32, P, P, P]
        L.ffo_sparsify.argtypes = [P, i32, i32, P, i32, i32, i32, i32, i32, P, P]
        L.ffo_isqrt64.argtypes = [C.c_uint64]
        L.ffo_isqrt64.restype = C.c_uint64
        L.ffo_dense_sift.argtypes = [P, i32, i32, P]
        L.ffo_smooth_codes.argtypes = [P, i32, i32, i32, P]
        L.ffo_sift_levels_create.argtypes = [P, i32, i32, i32, i32]
        L.ffo_sift_levels_create.restype = P
        L.ffo_sift_levels_free.argtypes = [P]
        L.ffo_sift_levels_free.restype = None
        L.ffo_sift_levels_get.argtypes = [P, i32, P]
        L.ffo_sift_cost.argtypes = [P, P, i32, i32, i32, i32, i32, i32, i32, i32]
        L.ffo_match_field_sift.argtypes = [P, P, P, P, i32, i32, P, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def pack(dx, dy):
    dx = np.asarray(dx, np.int64) & 0xFFFF
    dy = np.asarray(dy, np.int64) & 0xFFFF
    v = (dy << 16) | dx
    return np.where(v >= 1 << 31, v - (1 << 32), v).astype(np.int32)


def unpack(f):
    f = np.asarray(f, np.int64) & 0xFFFFFFFF
    dx = ((f & 0xFFFF) ^ 0x8000) - 0x8000
    dy = (((f >> 16) & 0xFFFF) ^ 0x8000) - 0x8000
    return dx.astype(np.int32), dy.astype(np.int32)


def lab8(img: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, np.uint8)
    H, W = img.shape[:2]
    Cc = 1 if img.ndim == 2 else img.shape[2]
    out = np.empty((Cc, H, W), np.uint8)
    assert lib().ffo_lab8(_p(img), W, H, Cc, W * Cc, _p(out)) == 0
    return out


def lab_tables():
    g = np.empty(256, np.int32)
    m = np.empty(9, np.int32)
    f = np.empty(65537, np.int32)
    lib().ffo_lab_tables(_p(g), _p(m), _p(f))
    return g, m.reshape(3, 3), f


def lanczos_weights(n: int) -> np.ndarray:
    out = np.empty((n, 7), np.int32)
    assert lib().ffo_lanczos_weights(n, _p(out)) == 0
    return out


def smooth(plane: np.ndarray, n: int) -> np.ndarray:
    plane = np.ascontiguousarray(plane, np.uint8)
    H, W = plane.shape
    out = np.empty((H, W), np.int16)
    assert lib().ffo_smooth(_p(plane), W, H, n, _p(out)) == 0
    return out


def census(S: np.ndarray, n: int, Q: int, a: int, b: int) -> np.ndarray:
    """S: C x H x W int16 smoothed planes -> H x W uint32 census plane."""
    S = np.ascontiguousarray(S, np.int16)
    Cc, H, W = S.shape
    out = np.empty((H, W), np.uint32)
    assert lib().ffo_census(_p(S), W, H, Cc, n, Q, a, b, _p(out)) == 0
    return out


def wht(lab: np.ndarray, rho: int) -> np.ndarray:
    lab = np.ascontiguousarray(lab, np.uint8)
    Cc, H, W = lab.shape
    out = np.empty((H, W, 9 * Cc), np.int32)
    assert lib().ffo_wht(_p(lab), W, H, Cc, rho, _p(out)) == 0
    return out


def walsh(s: int, t: int, rho: int) -> int:
    return lib().ffo_walsh(s, t, rho)


def tree_depth(N: int, leaf: int) -> int:
    return lib().ffo_tree_depth(N, leaf)


def kdtree_build(V: np.ndarray, leaf: int):
    """V: N x D int32.  Returns (node_dim, node_split, perm)."""
    V = np.ascontiguousarray(V, np.int32)
    N, D = V.shape
    depth = tree_depth(N, leaf)
    nn = (2 << depth) - 1
    nd = np.empty(nn, np.int32)
    ns = np.empty(nn, np.int32)
    perm = np.empty(N, np.int32)
    assert lib().ffo_kdtree_build(_p(V), N, D, leaf, _p(nd), _p(ns), _p(perm)) == depth
    return nd, ns, perm


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.empty(4, np.uint32)
    lib().ffo_philox4x32_10(_p(c), _p(k), _p(out))
    return out


class Desc:
    """Descriptors of one image (Lab8, smoothed planes, census planes for
    every level and subpixel phase, WHT vectors for each radius)."""

    def __init__(self, img: np.ndarray, k: int = 3, Q: int = 4, radii=(8, 6)):
        img = np.ascontiguousarray(img, np.uint8)
        if img.ndim == 2:
            img = img[:, :, None]
        self.H, self.W, self.C = img.shape
        self.k, self.Q = k, Q
        self.radii = tuple(radii)
        r = np.asarray(radii, np.int32)
        self._img = img
        self.h = lib().ffo_desc_create(_p(img), self.W, self.H, self.C, self.W * self.C, k, Q, _p(r), len(r))
        if not self.h:
            raise ValueError("bad descriptor arguments")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().ffo_desc_free(h)
            self.h = None

    def lab(self):
        out = np.empty((self.C, self.H, self.W), np.uint8)
        lib().ffo_desc_lab(self.h, _p(out))
        return out

    def smooth(self, lev):
        out = np.empty((self.C, self.H, self.W), np.int16)
        assert lib().ffo_desc_smooth(self.h, lev, _p(out)) == 0
        return out

    def plane(self, lev, a, b):
        out = np.empty((self.H, self.W), np.uint32)
        assert lib().ffo_desc_plane(self.h, lev, a, b, _p(out)) == 0
        return out

    def wht(self, rho):
        out = np.empty((self.H, self.W, 9 * self.C), np.int32)
        assert lib().ffo_desc_wht(self.h, rho, _p(out)) == 0
        return out


def cost(src: Desc, dst: Desc, lev: int, r: int, px: int, py: int, fx: int, fy: int) -> int:
    return lib().ffo_cost(src.h, dst.h, lev, r, px, py, fx, fy)


def match_field(src: Desc, dst: Desc, r: int, k: int = 3, R: int = 1, leaf: int = 8, n_prop: int = 4,
                n_rs: int = 3, use_kdtree: bool = True, skip_dup: bool = True, max_steps: int = -1,
                seed: int = 0, field_id: int = 0, pair_id: int = 0, proposal=None, counters: bool = False):
    """One Flow Field src -> dst.  Returns (flow, cost[, counters]) as H x W
    int32 arrays (packed int16x2 flow in 1/Q px, EMPTY / INF where unset)."""
    params = np.array([k, R, leaf, n_prop, n_rs, int(use_kdtree), int(skip_dup), max_steps,
                       seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF, field_id, pair_id], np.int64)
    flow = np.empty((src.H, src.W), np.int32)
    cst = np.empty((src.H, src.W), np.int32)
    cnt = np.zeros(8, np.int64)
    prop = None if proposal is None else np.ascontiguousarray(proposal, np.int32)
    rc = lib().ffo_match_field(src.h, dst.h, r, _p(params), None if prop is None else _p(prop), _p(flow),
                               _p(cst), _p(cnt))
    if rc < 0:
        raise ValueError(f"ffo_match_field failed ({rc})")
    if counters:
        return flow, cst, cnt
    return flow, cst


def consistency(F: np.ndarray, Bs, Q: int, eps_q: int):
    F = np.ascontiguousarray(F, np.int32)
    H1, W1 = F.shape
    Bs = [np.ascontiguousarray(b, np.int32) for b in Bs]
    H2, W2 = Bs[0].shape
    ptrs = (C.c_void_p * len(Bs))(*[b.ctypes.data for b in Bs])
    keep = np.empty((H1, W1), np.uint8)
    filt = np.empty((H1, W1), np.int32)
    assert lib().ffo_consistency(_p(F), W1, H1, C.cast(ptrs, C.c_void_p), len(Bs), W2, H2, Q, eps_q,
                                 _p(keep), _p(filt)) == 0
    return keep, filt


def region_filter(F: np.ndarray, keep: np.ndarray, Q: int, s: int):
    """Section 3.4's region filter on the consistency check's output.
    Returns (label, keep_out, filtered): region names (smallest pixel index,
    -1 outside the partly filtered field), the final mask and field."""
    F = np.ascontiguousarray(F, np.int32)
    keep = np.ascontiguousarray(keep, np.uint8)
    H, W = F.shape
    label = np.empty((H, W), np.int32)
    ko = np.empty((H, W), np.uint8)
    out = np.empty((H, W), np.int32)
    assert lib().ffo_region_filter(_p(F), _p(keep), W, H, Q, s, _p(label), _p(ko), _p(out)) == 0
    return label, ko, out


def isqrt64(v: int) -> int:
    return int(lib().ffo_isqrt64(v))


def sparsify(F: np.ndarray, Bs, Q: int, e: int):
    """Section 3.5's sparsification of the outlier-filtered field F against
    the backward fields Bs.  Returns (pick, sparse): per 3x3 block the chosen
    pixel index (-1 when fewer than e samples), and the chosen flows on an
    otherwise empty field."""
    F = np.ascontiguousarray(F, np.int32)
    H1, W1 = F.shape
    Bs = [np.ascontiguousarray(b, np.int32) for b in Bs]
    H2, W2 = Bs[0].shape
    ptrs = (C.c_void_p * len(Bs))(*[b.ctypes.data for b in Bs])
    pick = np.empty(((H1 + 2) // 3, (W1 + 2) // 3), np.int32)
    sparse = np.empty((H1, W1), np.int32)
    assert lib().ffo_sparsify(_p(F), W1, H1, C.cast(ptrs, C.c_void_p), len(Bs), W2, H2, Q, e, _p(pick),
                              _p(sparse)) == 0
    return pick, sparse


def brute_nnf(src: Desc, dst: Desc, lev: int, r: int):
    n = 1 << lev
    Gw, Gh = (src.W + n - 1) // n, (src.H + n - 1) // n
    flow = np.empty((Gh, Gw), np.int32)
    cst = np.empty((Gh, Gw), np.int32)
    lib().ffo_brute_nnf(src.h, dst.h, lev, r, _p(flow), _p(cst))
    return flow, cst


def match_pair(img1, img2, r: int = 8, r2: int = 6, k: int = 3, Q: int = 4, eps: int = 5, seed: int = 0,
               pair_id: int = 0, n_bwd: int = 2, region_s=None, sparse_e=None, **kw):
    """The whole hot path on one pair: descriptors, F (r), B1 (r), B2 (r2),
    two-way consistency filter, with region_s the region filter of section
    3.4 and then, with sparse_e, the sparsification of section 3.5.  Returns a
    dict of arrays."""
    radii = (r, r2) if n_bwd == 2 and r2 != r else (r,)
    d1 = Desc(img1, k, Q, radii)
    d2 = Desc(img2, k, Q, radii)
    F, CF = match_field(d1, d2, r, k=k, seed=seed, field_id=0, pair_id=pair_id, **kw)
    B1, CB1 = match_field(d2, d1, r, k=k, seed=seed, field_id=1, pair_id=pair_id, **kw)
    Bs = [B1]
    out = dict(F=F, CF=CF, B1=B1, CB1=CB1)
    if n_bwd == 2:
        B2, CB2 = match_field(d2, d1, r2, k=k, seed=seed, field_id=2, pair_id=pair_id, **kw)
        Bs.append(B2)
        out.update(B2=B2, CB2=CB2)
    keep, filt = consistency(F, Bs, Q, eps * Q)
    out.update(keep=keep, filtered=filt)
    if region_s is not None:
        lab, kr, fr = region_filter(F, keep, Q, region_s)
        out.update(region_label=lab, keep_region=kr, filtered_region=fr)
        if sparse_e is not None:
            pick, sp = sparsify(fr, Bs, Q, sparse_e)
            out.update(pick=pick, sparse=sp)
    return out


# ---------------------------------------------------------------------------
# Section 3.3, the SIFT-flow data term: dense SIFT on the CIELab lightness,
# PCA to S colours, per-level smoothing of the quantised colours, L2 patch
# distances; the search itself is the census one with this cost.

SIFT_DIM = 128
CODE_SCALE = 1024.0     # colours are stored as round-half-even(1024 c) int16
CODE_MAX = 2047         # |c| <= |d - mean| <= 2 for unit-length d; clamped to +-2047


def dense_sift(L: np.ndarray) -> np.ndarray:
    """H x W uint8 lightness plane -> H x W x 128 float64 SIFT vectors."""
    L = np.ascontiguousarray(L, np.uint8)
    H, W = L.shape
    out = np.empty((H, W, SIFT_DIM), np.float64)
    assert lib().ffo_dense_sift(_p(L), W, H, _p(out)) == 0
    return out


def sift_pca(D1: np.ndarray, D2: np.ndarray):
    """PCA over the SIFT vectors of both images of a pair (the reading: one
    basis per pair, from every pixel of both images).  Returns (mean,
    eigenvalues descending, eigenvectors as columns in that order); each
    eigenvector's largest-magnitude component (the first on ties) is made
    positive."""
    X = np.concatenate([D1.reshape(-1, SIFT_DIM), D2.reshape(-1, SIFT_DIM)], 0).astype(np.float64)
    mean = X.mean(axis=0)
    Xc = X - mean
    cov = Xc.T @ Xc / X.shape[0]
    lam, V = np.linalg.eigh(cov)
    lam, V = lam[::-1].copy(), V[:, ::-1].copy()
    idx = np.argmax(np.abs(V), axis=0)
    sgn = np.sign(V[idx, np.arange(SIFT_DIM)])
    sgn[sgn == 0] = 1.0
    return mean, lam, V * sgn


def sift_codes(D: np.ndarray, mean: np.ndarray, V: np.ndarray, S: int) -> np.ndarray:
    """Project H x W x 128 vectors on the first S eigenvectors and quantise:
    round-half-even(1024 c), clamped to +-2047; H x W x S int16."""
    c = (D.reshape(-1, SIFT_DIM) - mean) @ V[:, :S]
    q = np.clip(np.rint(c * CODE_SCALE), -CODE_MAX, CODE_MAX).astype(np.int16)
    return q.reshape(D.shape[:-1] + (S,))


def sift_colors(img1, img2, S: int = 18):
    """Colours of both images of a pair: (codes1, codes2, (mean, eigenvalues,
    eigenvectors))."""
    L1 = lab8(img1)[0]
    L2 = lab8(img2)[0]
    D1, D2 = dense_sift(L1), dense_sift(L2)
    mean, lam, V = sift_pca(D1, D2)
    return sift_codes(D1, mean, V, S), sift_codes(D2, mean, V, S), (mean, lam, V)


def smooth_codes(plane: np.ndarray, n: int) -> np.ndarray:
    plane = np.ascontiguousarray(plane, np.int16)
    H, W = plane.shape
    out = np.empty((H, W), np.int16)
    assert lib().ffo_smooth_codes(_p(plane), W, H, n, _p(out)) == 0
    return out


class SiftLevels:
    """Per-level smoothed colour planes of one image (levels 0..k)."""

    def __init__(self, codes: np.ndarray, k: int = 3):
        codes = np.ascontiguousarray(codes, np.int16)
        self.H, self.W, self.S = codes.shape
        self.k = k
        self.h = lib().ffo_sift_levels_create(_p(codes), self.W, self.H, self.S, k)
        if not self.h:
            raise ValueError("bad colour arguments")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().ffo_sift_levels_free(h)
            self.h = None

    def level(self, lev):
        """S x H x W int16."""
        out = np.empty((self.S, self.H, self.W), np.int16)
        assert lib().ffo_sift_levels_get(self.h, lev, _p(out)) == 0
        return out


def sift_cost(src: SiftLevels, dst: SiftLevels, Q: int, lev: int, r: int, S: int, px: int, py: int, fx: int,
              fy: int) -> int:
    return lib().ffo_sift_cost(src.h, dst.h, Q, lev, r, S, px, py, fx, fy)


def match_field_sift(src: Desc, dst: Desc, ssrc: SiftLevels, sdst: SiftLevels, r: int, S: int, k: int = 3,
                     R: int = 1, leaf: int = 8, n_prop: int = 4, n_rs: int = 3, skip_dup: bool = True,
                     max_steps: int = -1, seed: int = 0, field_id: int = 0, pair_id: int = 0,
                     counters: bool = False):
    """One Flow Field src -> dst with the SIFT-flow data term on the first S
    colours (kd-tree seeds from the CIELab WHTs of src / dst)."""
    params = np.array([k, R, leaf, n_prop, n_rs, 1, int(skip_dup), max_steps,
                       seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF, field_id, pair_id], np.int64)
    flow = np.empty((src.H, src.W), np.int32)
    cst = np.empty((src.H, src.W), np.int32)
    cnt = np.zeros(8, np.int64)
    rc = lib().ffo_match_field_sift(src.h, dst.h, ssrc.h, sdst.h, r, S, _p(params), _p(flow), _p(cst), _p(cnt))
    if rc < 0:
        raise ValueError(f"ffo_match_field_sift failed ({rc})")
    if counters:
        return flow, cst, cnt
    return flow, cst


def match_pair_sift(img1, img2, r: int = 3, r2: int = 2, S: int = 12, S2: int = 18, k: int = 3, Q: int = 4,
                    eps: int = 1, seed: int = 0, pair_id: int = 0, region_s=150, sparse_e=9, **kw):
    """The hot path with the SIFT-flow data term on one pair, with the
    paper's KITTI settings by default (r = 3, r2 = 2, S = 12 for F and B1,
    S2 = 18 for B2, epsilon = 1, s = 150, e = 9).  Returns a dict of arrays."""
    codes1, codes2, pca = sift_colors(img1, img2, max(S, S2))
    radii = (r, r2) if r2 != r else (r,)
    d1 = Desc(img1, k, Q, radii)
    d2 = Desc(img2, k, Q, radii)
    c1 = SiftLevels(codes1, k)
    c2 = SiftLevels(codes2, k)
    F, CF = match_field_sift(d1, d2, c1, c2, r, S, k=k, seed=seed, field_id=0, pair_id=pair_id, **kw)
    B1, CB1 = match_field_sift(d2, d1, c2, c1, r, S, k=k, seed=seed, field_id=1, pair_id=pair_id, **kw)
    B2, CB2 = match_field_sift(d2, d1, c2, c1, r2, S2, k=k, seed=seed, field_id=2, pair_id=pair_id, **kw)
    out = dict(codes1=codes1, codes2=codes2, eig=pca[1], F=F, CF=CF, B1=B1, CB1=CB1, B2=B2, CB2=CB2)
    keep, filt = consistency(F, [B1, B2], Q, eps * Q)
    out.update(keep=keep, filtered=filt)
    if region_s is not None:
        lab, kr, fr = region_filter(F, keep, Q, region_s)
        out.update(region_label=lab, keep_region=kr, filtered_region=fr)
        if sparse_e is not None:
            pick, sp = sparsify(fr, [B1, B2], Q, sparse_e)
            out.update(pick=pick, sparse=sp)
    return out
