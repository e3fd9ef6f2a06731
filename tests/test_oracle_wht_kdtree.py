"""Pins of the WHT patch vectors and of the kd-tree (section 3.1)."""
import json
import os

import numpy as np
import pytest

from oracle import ffo

GOLD = os.path.join(os.path.dirname(__file__), "golden")
BASES = [(0, 0), (0, 1), (1, 0), (1, 1), (0, 2), (2, 0), (1, 2), (2, 1), (2, 2)]


def test_walsh_signs_golden():
    ref = json.load(open(os.path.join(GOLD, "walsh_signs.json")))["rho"]
    for rho, fns in ref.items():
        rho = int(rho)
        for s in range(3):
            got = "".join("+" if ffo.walsh(s, t, rho) > 0 else "-" for t in range(-rho, rho + 1))
            assert got == fns[f"w{s}"], (rho, s, got)


def _sign_runs(rho, s):
    """Runs (t_lo, t_hi, sign) of the 1-D Walsh function from the golden
    strings (so the integral-image formulation below does not reuse the
    oracle's basis code)."""
    ref = json.load(open(os.path.join(GOLD, "walsh_signs.json")))["rho"]
    if str(rho) in ref:
        string = ref[str(rho)][f"w{s}"]
    else:
        raise KeyError(rho)
    runs = []
    t = -rho
    i = 0
    while i < len(string):
        j = i
        while j < len(string) and string[j] == string[i]:
            j += 1
        runs.append((t + i, t + j - 1, 1 if string[i] == "+" else -1))
        i = j
    return runs


def _wht_integral(lab, rho):
    """WHT vectors as signed box sums over a padded integral image."""
    C, H, W = lab.shape
    out = np.zeros((H, W, 9 * C), np.int64)
    for c in range(C):
        P = np.pad(lab[c].astype(np.int64), rho, mode="edge")
        I = np.zeros((P.shape[0] + 1, P.shape[1] + 1), np.int64)
        I[1:, 1:] = P.cumsum(0).cumsum(1)

        def box(y0, y1, x0, x1):  # inclusive offsets relative to the pixel
            ys = np.arange(H)[:, None] + rho
            xs = np.arange(W)[None, :] + rho
            return (I[ys + y1 + 1, xs + x1 + 1] - I[ys + y0, xs + x1 + 1] -
                    I[ys + y1 + 1, xs + x0] + I[ys + y0, xs + x0])

        for j, (u, v) in enumerate(BASES):
            acc = np.zeros((H, W), np.int64)
            for (y0, y1, sy) in _sign_runs(rho, u):
                for (x0, x1, sx) in _sign_runs(rho, v):
                    acc += sy * sx * box(y0, y1, x0, x1)
            out[:, :, c * 9 + j] = acc
    return out


@pytest.mark.parametrize("rho", [2, 3, 6, 8])
def test_wht_equals_integral_image_box_sums(rho):
    rng = np.random.default_rng(rho)
    lab = rng.integers(0, 256, (3, 23, 29)).astype(np.uint8)
    got = ffo.wht(lab, rho)
    ref = _wht_integral(lab, rho)
    assert np.array_equal(got, ref)


def test_wht_dc_is_patch_sum():
    lab = np.full((1, 12, 15), 9, np.uint8)
    v = ffo.wht(lab, 3)
    assert np.all(v[:, :, 0] == 49 * 9)
    # w1 and w2 have one more minus than plus tap: sum = -1 * 7 * 9 etc.
    assert np.all(v[:, :, 1] == -7 * 9)


# ---------------------------------------------------------------- kd-tree

def _tree_numpy(V, leaf):
    """Independent recursive build with NumPy lexsort (same reading)."""
    N, D = V.shape
    depth = 0
    while -(-N // (1 << depth)) > leaf:
        depth += 1
    nn = (2 << depth) - 1
    nd = np.full(nn, -1, np.int64)
    ns = np.zeros(nn, np.int64)
    perm = np.zeros(N, np.int64)
    stack = [(0, 0, np.arange(N))]
    while stack:
        node, start, ids = stack.pop()
        cnt = len(ids)
        if cnt <= leaf:
            perm[start:start + cnt] = np.sort(ids)
            continue
        sub = V[ids]
        spread = sub.max(0).astype(np.int64) - sub.min(0)
        dim = int(np.argmax(spread))  # first maximum = lowest dimension
        order = np.lexsort((ids, sub[:, dim]))
        ids = ids[order]
        h = cnt // 2
        nd[node] = dim
        ns[node] = V[ids[h], dim]
        stack.append((2 * node + 1, start, ids[:h]))
        stack.append((2 * node + 2, start + h, ids[h:]))
    return nd, ns, perm


@pytest.mark.parametrize("N,D,leaf,vals", [(1000, 27, 8, 50), (777, 9, 8, 4), (3000, 5, 3, 1000), (8, 4, 8, 10),
                                           (9, 4, 8, 10)])
def test_kdtree_equals_independent_build(N, D, leaf, vals):
    rng = np.random.default_rng(N)
    V = rng.integers(-vals, vals, (N, D)).astype(np.int32)
    nd, ns, perm = ffo.kdtree_build(V, leaf)
    rnd, rns, rperm = _tree_numpy(V, leaf)
    assert np.array_equal(nd, rnd)
    internal = nd >= 0
    assert np.array_equal(ns[internal], rns[internal])
    assert np.array_equal(perm, rperm)


def test_kdtree_invariants_and_self_query():
    rng = np.random.default_rng(5)
    N, D, leaf = 2500, 27, 8
    # distinct values in every dimension: no key ever ties with a split
    V = np.stack([rng.permutation(N) * 3 - 4000 for _ in range(D)], 1).astype(np.int32)
    nd, ns, perm = ffo.kdtree_build(V, leaf)
    assert np.array_equal(np.sort(perm), np.arange(N))
    # walk: ranges, leaf sizes, split ordering
    stack = [(0, 0, N)]
    leaves = []
    while stack:
        node, st, c = stack.pop()
        if nd[node] < 0:
            assert 1 <= c <= leaf
            seg = perm[st:st + c]
            assert np.all(np.diff(seg) > 0)
            leaves.append((st, c))
            continue
        h = c // 2
        d = nd[node]
        left = perm[st:st + h]
        right = perm[st + h:st + c]
        assert V[left, d].max() <= ns[node] <= V[right, d].min()
        stack.append((2 * node + 1, st, h))
        stack.append((2 * node + 2, st + h, c - h))
    assert sum(c for _, c in leaves) == N
    # a query with a point's own (unique) vector reaches the leaf holding it
    for i in rng.integers(0, N, 50):
        node, st, c = 0, 0, N
        while nd[node] >= 0:
            h = c // 2
            if V[i, nd[node]] >= ns[node]:
                node, st, c = 2 * node + 2, st + h, c - h
            else:
                node, c = 2 * node + 1, h
        assert i in perm[st:st + c]
