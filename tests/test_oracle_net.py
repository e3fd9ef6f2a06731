"""Pins of the proposal-network oracle: a library correlation for the plain
convolution, output sizes of the strided layers, and central finite
differences in float64 for every layer's gradient."""
import numpy as np
import pytest
from scipy import signal

from oracle import net_oracle as N


def test_param_count_and_split():
    assert N.param_count() == 6 * 32 * 9 + 32 + 4 * (32 * 32 * 9 + 32) + 32 * 2 * 9 + 2
    th = N.init_params(1)
    parts = N.split_params(th)
    assert [p[0].shape for p in parts][0] == (32, 6, 3, 3) and parts[-1][1].shape == (2,)


def test_conv_stride1_equals_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 11, 13, 3))
    W = rng.standard_normal((2, 3, 3, 3))
    b = np.array([0.5, -1.0])
    y = N.conv(x, W, b, 1, 1)
    for co in range(2):
        ref = sum(signal.correlate2d(x[0, :, :, ci], W[co, ci], mode="same", boundary="fill") for ci in range(3))
        assert np.allclose(y[0, :, :, co], ref + b[co])


def test_dilated_and_strided_sizes():
    x = np.zeros((2, 436, 1024, 6))
    th = N.init_params(0)
    out = N.forward(th, x, exact=True)
    assert out.shape == (2, 55, 128, 2)   # ceil(436/8) x ceil(1024/8): the seed grid
    y = N.conv(np.ones((1, 9, 9, 1)), np.ones((1, 1, 3, 3)), np.zeros(1), 1, 4)
    # centre tap only inside the image at dilation 4 for the corner pixel
    assert y[0, 0, 0, 0] == 4 and y[0, 4, 4, 0] == 9


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_central_differences(seed):
    rng = np.random.default_rng(seed)
    H, W = 19, 23
    x = rng.uniform(-0.5, 0.5, (2, H, W, 6))
    th = N.init_params(seed).astype(np.float64) * 0.7 + rng.standard_normal(N.param_count()) * 0.02
    out, acts = N.forward(th, x, exact=True, keep=True)
    # smooth loss (squared error) so that central differences are exact to O(h^2)
    tgt = rng.standard_normal(out.shape)
    def loss(t):
        o = N.forward(t, x, exact=True)
        return 0.5 * ((o - tgt) ** 2).sum()
    g = N.backward(th, acts, out - tgt, exact=True)
    idx = np.concatenate([rng.choice(np.arange(o0, o1), 6, replace=False) for o0, o1 in _layer_ranges()])
    h = 1e-6
    for i in idx:
        tp = th.copy(); tp[i] += h
        tm = th.copy(); tm[i] -= h
        fd = (loss(tp) - loss(tm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(fd)), (i, fd, g[i])


def _layer_ranges():
    o = 0
    out = []
    for ci, co, _, _, _ in N.LAYERS:
        out.append((o, o + co * ci * 9 + co))
        o += co * ci * 9 + co
    return out


def test_masked_l1_and_rounding():
    out = np.zeros((1, 2, 2, 2))
    lab = np.full((1, 2, 2, 2), np.nan)
    lab[0, 0, 0] = [32.0, -64.0]
    loss, g = N.masked_l1(out, lab)
    assert loss == pytest.approx(3.0)
    assert g[0, 0, 0, 0] == -1.0 and g[0, 0, 0, 1] == 1.0 and g[0, 1, 1].sum() == 0
    q = N.proposal_q(np.array([[[[0.5 / 32, -1.0 / 32]]]]), 4)
    assert q[0, 0, 0] == ((((-4) & 0xFFFF) << 16) | 2) - (1 << 32)
    assert N.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0 and N.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6
