"""Pins of the region-based outlier filter that follows the consistency check
(section 3.4, second paragraph).  Expected values come from a hand-worked
example, closed forms, and an independent formulation whose connected
components come from scipy.sparse.csgraph -- never from the oracle itself."""
import json
import os

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from oracle import ffo

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    g = json.load(open(os.path.join(GOLD, "region_filter_tiny.json")))
    Q = g["Q"]
    H, W = g["H"], g["W"]
    F = np.zeros((H, W), np.int32)
    keep = np.zeros((H, W), np.uint8)
    for y, row in enumerate(g["map"]):
        for x, ch in enumerate(row):
            fx, fy, k = g["legend_px"][ch]
            F[y, x] = ffo.pack(int(round(fx * Q)), int(round(fy * Q)))
            keep[y, x] = k
    return g, F, keep


def test_hand_worked_example():
    g, F, keep = _golden()
    label, ko, out = ffo.region_filter(F, keep, g["Q"], g["s"])
    assert np.array_equal(label, np.array(g["label"], np.int32))
    assert np.array_equal(ko, np.array(g["keep_out"], np.uint8))
    assert np.array_equal(out, np.where(ko == 1, F, ffo.EMPTY))


def _random_field(seed, H=23, W=31, Q=4, p_drop=0.25):
    """Piecewise flows (a few constant patches plus jitter) so that regions of
    many sizes occur, some flows on the 3 px boundary."""
    rng = np.random.default_rng(seed)
    base = rng.integers(-6, 7, (4, 2)) * Q
    idx = rng.integers(0, 4, (H // 4 + 1, W // 4 + 1)).repeat(4, 0).repeat(4, 1)[:H, :W]
    fx = base[idx, 0] + rng.choice([0, 0, 0, Q, 3 * Q, -2 * Q, 5], (H, W))
    fy = base[idx, 1] + rng.choice([0, 0, 0, -Q, 2 * Q, 3], (H, W))
    F = ffo.pack(fx, fy)
    F[rng.random((H, W)) < 0.02] = ffo.EMPTY
    keep = ((rng.random((H, W)) >= p_drop) & (F != ffo.EMPTY)).astype(np.uint8)
    return F, keep


def _independent(F, keep, Q, s):
    """The same definition from scratch: a graph of 4-neighbour pairs of
    field pixels whose flows differ by less than 3 px, its connected
    components from scipy, then the size and joinable rules."""
    H, W = F.shape
    dx, dy = ffo.unpack(F)
    field = (keep != 0) & (F != ffo.EMPTY)
    deleted = (keep == 0) & (F != ffo.EMPTY)
    idx = np.arange(H * W).reshape(H, W)
    rows, cols = [], []
    joinable_px = np.zeros((H, W), bool)
    for (ay, ax, by, bx) in ((slice(None), slice(0, -1), slice(None), slice(1, None)),
                             (slice(0, -1), slice(None), slice(1, None), slice(None))):
        d2 = (dx[ay, ax].astype(np.int64) - dx[by, bx]) ** 2 + (dy[ay, ax].astype(np.int64) - dy[by, bx]) ** 2
        sim = d2 < 9 * Q * Q
        e = field[ay, ax] & field[by, bx] & sim
        rows += list(idx[ay, ax][e])
        cols += list(idx[by, bx][e])
        # a deleted neighbour on either side of the pair
        joinable_px[ay, ax] |= field[ay, ax] & deleted[by, bx] & sim
        joinable_px[by, bx] |= field[by, bx] & deleted[ay, ax] & sim
    n = H * W
    g = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    comp = comp.reshape(H, W)
    label = np.full((H, W), -1, np.int64)
    keep_out = np.zeros((H, W), np.uint8)
    for c in np.unique(comp[field]):
        m = field & (comp == c)
        label[m] = idx[m].min()
        removed = m.sum() < s and joinable_px[m].any()
        keep_out[m] = 0 if removed else 1
    return label, keep_out


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("s", [0, 1, 3, 8, 50])
def test_equals_independent_formulation(seed, s):
    Q = 4
    F, keep = _random_field(seed, Q=Q)
    label, ko, out = ffo.region_filter(F, keep, Q, s)
    rl, rk = _independent(F, keep, Q, s)
    assert np.array_equal(label, rl)
    assert np.array_equal(ko, rk)
    assert np.array_equal(out, np.where(ko == 1, F, ffo.EMPTY))


def test_closed_forms():
    Q = 4
    for seed in range(4):
        F, keep = _random_field(10 + seed, Q=Q)
        field = (keep != 0) & (F != ffo.EMPTY)
        # nothing was deleted with a flow: no region can take in an outlier
        F0 = np.where(keep == 1, F, ffo.EMPTY).astype(np.int32)
        _, ko, out = ffo.region_filter(F0, keep, Q, 10 ** 6)
        assert np.array_equal(ko.astype(bool), field)
        assert np.array_equal(out, F0)
        # s <= 1: no region has fewer than one pixel
        for s in (0, 1):
            _, ko, _ = ffo.region_filter(F, keep, Q, s)
            assert np.array_equal(ko.astype(bool), field)
        # only removes, whole regions, and more for larger s
        label, k8, _ = ffo.region_filter(F, keep, Q, 8)
        _, k50, _ = ffo.region_filter(F, keep, Q, 50)
        assert not (k8.astype(bool) & ~field).any()
        assert not (k50.astype(bool) & ~k8.astype(bool)).any()
        for name in np.unique(label[label >= 0]):
            vals = k8[label == name]
            assert vals.min() == vals.max()


def test_constant_field_is_one_region():
    H, W, Q = 12, 17, 4
    F = np.full((H, W), ffo.pack(9, -5), np.int32)
    keep = np.ones((H, W), np.uint8)
    keep[3, 4] = 0            # a deleted pixel with the same flow
    label, ko, _ = ffo.region_filter(F, keep, Q, H * W)
    assert set(np.unique(label)) == {-1, 0}
    assert ko.sum() == 0      # fewer than H W pixels and joinable: removed
    label, ko, _ = ffo.region_filter(F, keep, Q, H * W - 1)
    assert ko.sum() == H * W - 1
