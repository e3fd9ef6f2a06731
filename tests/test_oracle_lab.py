"""Pins of the oracle's 8-bit CIELab conversion (section 3.3 computes the
census data term in CIELab).  Expected values come from textbook colour
coordinates and from a float64 formulation written here, never from the
oracle itself."""
import json
import os

import numpy as np
import pytest

from oracle import ffo

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _lab_float(rgb):
    """CIE L*a*b* (D65) of sRGB values in float64, straight from the sRGB and
    CIE definitions: linearise, XYZ / white point, cube-root compression."""
    v = rgb.astype(np.float64) / 255.0
    lin = np.where(v <= 0.04045, v / 12.92, ((v + 0.055) / 1.055) ** 2.4)
    Mx = np.array([[0.4124564, 0.3575761, 0.1804375],
                   [0.2126729, 0.7151522, 0.0721750],
                   [0.0193339, 0.1191920, 0.9503041]])
    white = Mx.sum(1)
    xyz = lin @ Mx.T / white
    d = 6.0 / 29.0
    f = np.where(xyz > d ** 3, np.cbrt(xyz), xyz / (3 * d * d) + 4.0 / 29.0)
    L = 116 * f[..., 1] - 16
    a = 500 * (f[..., 0] - f[..., 1])
    b = 200 * (f[..., 1] - f[..., 2])
    return np.stack([L, a, b], -1)


def test_textbook_colours():
    ref = json.load(open(os.path.join(GOLD, "lab_srgb_reference.json")))
    rgb = np.array([c["rgb"] for c in ref["colors"]], np.uint8)[None]
    lab = ffo.lab8(rgb)[:, 0, :].T.astype(np.int64)
    exp = np.array([c["lab"] for c in ref["colors"]])
    exp8 = np.stack([2.55 * exp[:, 0], exp[:, 1] + 128, exp[:, 2] + 128], 1)
    exp8 = np.clip(exp8, 0, 255)
    assert np.all(np.abs(lab - exp8) <= 1.0 + 1e-9), (lab, exp8)


def test_white_black_gray_exact():
    g = np.arange(256, dtype=np.uint8)
    rgb = np.stack([g, g, g], -1)[None]
    lab = ffo.lab8(rgb)[:, 0, :]
    # rows of the XYZ matrix sum to exactly 2^14, so every gray has a = b = 0
    assert np.all(lab[1] == 128) and np.all(lab[2] == 128)
    assert lab[0, 0] == 0 and lab[0, 255] == 255
    assert np.all(np.diff(lab[0].astype(int)) >= 0)


def test_tables_closed_form():
    gamma, mat, f = ffo.lab_tables()
    assert gamma[0] == 0 and gamma[255] == 65536
    assert np.all(np.diff(gamma) > 0)
    assert np.all(mat.sum(1) == 16384)
    assert f[0] == round(4 / 29 * 32768) and f[65536] == 32768
    assert np.all(np.diff(f) >= 0)


@pytest.mark.slow
def test_exhaustive_all_24bit_colours():
    """Every one of the 2^24 colours within one code of round(float Lab)."""
    v = np.arange(1 << 24, dtype=np.uint32)
    rgb = np.stack([(v >> 16) & 255, (v >> 8) & 255, v & 255], -1).astype(np.uint8)
    lab8 = ffo.lab8(rgb.reshape(4096, 4096, 3)).reshape(3, -1)
    for lo in range(0, 1 << 24, 1 << 22):
        sl = slice(lo, lo + (1 << 22))
        lab = _lab_float(rgb[sl])
        ref = np.stack([np.floor(2.55 * lab[:, 0] + 0.5), np.floor(lab[:, 1] + 0.5) + 128,
                        np.floor(lab[:, 2] + 0.5) + 128], 0)
        ref = np.clip(ref, 0, 255)
        d = np.abs(lab8[:, sl].astype(np.int64) - ref)
        assert d.max() <= 1, d.max()
