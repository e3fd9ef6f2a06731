"""Pins of the sparsification of section 3.5 (one sample per 3x3 region with
at least e samples: the smallest summed consistency error).  Expected values
come from a hand-worked example, the integer square root of the Python
library, real-valued error sums and closed forms."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ffo

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    g = json.load(open(os.path.join(GOLD, "sparsify_tiny.json")))
    H, W = g["H"], g["W"]
    F = np.full((H, W), ffo.pack(*g["F_default"]), np.int32)
    for x, y in g["F_empty"]:
        F[y, x] = ffo.EMPTY
    for k, v in g["F_set"].items():
        x, y = map(int, k.split(","))
        F[y, x] = ffo.pack(*v)
    Bs = []
    for name in ("B1", "B2"):
        B = np.full((H, W), ffo.pack(*g["B_default"]), np.int32)
        for k, v in g[name].items():
            x, y = map(int, k.split(","))
            B[y, x] = ffo.EMPTY if v == "empty" else ffo.pack(*v)
        Bs.append(B)
    return g, F, Bs


def test_hand_worked_example():
    g, F, Bs = _golden()
    pick, sparse = ffo.sparsify(F, Bs, g["Q"], g["e"])
    assert np.array_equal(pick, np.array(g["pick"], np.int32))
    want = np.full(F.shape, ffo.EMPTY, np.int32)
    for i in pick[pick >= 0]:
        want.flat[i] = F.flat[i]
    assert np.array_equal(sparse, want)


def test_integer_square_root_matches_library():
    rng = np.random.default_rng(0)
    vals = [0, 1, 2, 3, 4, 8, 9, 15, 16, 17, 2 ** 28, 2 ** 28 - 1, 2 ** 62 - 1, (2 ** 31 - 1) ** 2,
            (2 ** 31 - 1) ** 2 - 1]
    vals += [int(v) for v in rng.integers(0, 2 ** 62, 2000, dtype=np.int64)]
    vals += [int(v) ** 2 + d for v in rng.integers(0, 2 ** 31 - 1, 500) for d in (-1, 0, 1) if int(v) ** 2 + d >= 0]
    for v in vals:
        assert ffo.isqrt64(v) == math.isqrt(v), v


def _random(seed, H, W, Q=4):
    rng = np.random.default_rng(seed)
    fx = rng.integers(-3 * Q, 3 * Q + 1, (H, W))
    fy = rng.integers(-3 * Q, 3 * Q + 1, (H, W))
    F = ffo.pack(fx, fy)
    F[rng.random((H, W)) < 0.4] = ffo.EMPTY
    Bs = []
    for _ in range(2):
        B = ffo.pack(-fx + rng.integers(-6, 7, (H, W)), -fy + rng.integers(-6, 7, (H, W)))
        B[rng.random((H, W)) < 0.05] = ffo.EMPTY
        Bs.append(B)
    return F, Bs


@pytest.mark.parametrize("seed", range(5))
def test_pick_minimises_real_error_sum(seed):
    """The chosen sample's real-valued error sum is within the fixed-point
    resolution of its block's minimum; blocks with fewer than e samples pick
    nothing; the sparse field holds exactly the picks."""
    H, W, Q, e = 26, 31, 4, 4
    F, Bs = _random(seed, H, W, Q)
    pick, sparse = ffo.sparsify(F, Bs, Q, e)
    dx, dy = ffo.unpack(F)
    for by in range((H + 2) // 3):
        for bx in range((W + 2) // 3):
            errs = {}
            for y in range(3 * by, min(3 * by + 3, H)):
                for x in range(3 * bx, min(3 * bx + 3, W)):
                    if F[y, x] == ffo.EMPTY:
                        continue
                    mx = (x * Q + int(dx[y, x]) + Q // 2) // Q
                    my = (y * Q + int(dy[y, x]) + Q // 2) // Q
                    tot = 0.0
                    for B in Bs:
                        if not (0 <= mx < W and 0 <= my < H) or B[my, mx] == ffo.EMPTY:
                            tot = math.inf
                            break
                        bx_, by_ = ffo.unpack(B[my, mx])
                        tot += math.hypot(int(dx[y, x]) + int(bx_), int(dy[y, x]) + int(by_))
                    errs[y * W + x] = tot
            p = int(pick[by, bx])
            if len(errs) < e:
                assert p == -1
                continue
            assert p in errs
            best = min(errs.values())
            assert errs[p] <= best + 2 * 2 ** -14 or (math.isinf(best) and math.isinf(errs[p]))
            # no earlier sample is strictly better beyond the resolution
            for i, v in errs.items():
                if i < p:
                    assert v >= errs[p] - 2 * 2 ** -14 or math.isinf(errs[p])
    want = np.full(F.shape, ffo.EMPTY, np.int32)
    for i in pick[pick >= 0]:
        want.flat[i] = F.flat[i]
    assert np.array_equal(sparse, want)


def test_closed_forms():
    H, W, Q = 13, 20, 4
    F, Bs = _random(9, H, W, Q)
    # e above 9: no 3x3 region holds that many samples
    pick, sparse = ffo.sparsify(F, Bs, Q, 10)
    assert (pick == -1).all() and (sparse == ffo.EMPTY).all()
    # e <= 1: every region with a sample keeps one
    pick, _ = ffo.sparsify(F, Bs, Q, 1)
    has = np.zeros(pick.shape, bool)
    for i in np.flatnonzero(F != ffo.EMPTY):
        y, x = divmod(int(i), W)
        has[y // 3, x // 3] = True
    assert np.array_equal(pick >= 0, has)
    # perfect inverse fields, every pixel a sample: all errors 0, first pixel wins
    F = np.full((H, W), ffo.pack(0, 0), np.int32)
    pick, _ = ffo.sparsify(F, [F, F], Q, 9)
    full = [(by, bx) for by in range(pick.shape[0]) for bx in range(pick.shape[1])
            if 3 * by + 3 <= H and 3 * bx + 3 <= W]
    for by, bx in full:
        assert pick[by, bx] == 3 * by * W + 3 * bx
    assert (pick[4, :] == -1).all() and (pick[:, 6] == -1).all()   # clipped blocks hold 3 or 6 pixels < 9
