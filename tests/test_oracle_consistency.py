"""Pins of the forward/backward consistency filter (Eq. 5, section 3.4)."""
import json
import os

import numpy as np

from oracle import ffo

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _field(a):
    a = np.asarray(a)
    return ffo.pack(a[..., 0], a[..., 1])


def test_hand_worked_example():
    g = json.load(open(os.path.join(GOLD, "consistency_tiny.json")))
    F = _field(g["F"])
    B = _field(g["B1"])
    keep, filt = ffo.consistency(F, [B], g["Q"], g["eps_q"])
    assert np.array_equal(keep, np.array(g["keep"], np.uint8))
    assert np.array_equal(filt, np.where(keep == 1, F, ffo.EMPTY))


def test_perfect_inverse_keeps_everything_inside():
    H, W, Q = 30, 40, 4
    tx, ty = 13, -6  # quarter pixels
    F = np.full((H, W), ffo.pack(tx, ty), np.int32)
    B = np.full((H, W), ffo.pack(-tx, -ty), np.int32)
    keep, _ = ffo.consistency(F, [B, B], Q, 1)
    ys, xs = np.mgrid[0:H, 0:W]
    mx = (xs * Q + tx + Q // 2) // Q
    my = (ys * Q + ty + Q // 2) // Q
    inside = (mx >= 0) & (mx < W) & (my >= 0) & (my < H)
    assert np.array_equal(keep.astype(bool), inside)


def test_two_way_check_deletes_if_either_fails():
    """Eq. 5: a pixel is deleted if it is inconsistent with either backward
    field."""
    H, W, Q, eps_q = 10, 12, 4, 20
    rng = np.random.default_rng(1)
    F = np.zeros((H, W), np.int32)
    B1 = np.zeros((H, W), np.int32)
    B2 = np.zeros((H, W), np.int32)
    bad1 = rng.random((H, W)) < 0.2
    bad2 = rng.random((H, W)) < 0.2
    B1[bad1] = ffo.pack(20, 0)   # |error| = 20 = eps -> fails (strict)
    B2[bad2] = ffo.pack(0, -25)
    B1[~bad1 & (rng.random((H, W)) < 0.5)] = ffo.pack(19, 0)  # passes
    keep, _ = ffo.consistency(F, [B1, B2], Q, eps_q)
    assert np.array_equal(keep.astype(bool), ~(bad1 | bad2))
    k1, _ = ffo.consistency(F, [B1], Q, eps_q)
    assert np.array_equal(k1.astype(bool), ~bad1)


def test_empty_backward_and_empty_forward_dropped():
    H, W, Q = 4, 5, 4
    F = np.zeros((H, W), np.int32)
    F[0, 0] = ffo.EMPTY
    B = np.zeros((H, W), np.int32)
    B[2, 3] = ffo.EMPTY
    keep, filt = ffo.consistency(F, [B], Q, 4)
    assert keep[0, 0] == 0 and keep[2, 3] == 0 and keep.sum() == H * W - 2
    assert filt[0, 0] == ffo.EMPTY and filt[2, 3] == ffo.EMPTY
