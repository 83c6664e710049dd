"""Pins of the oracle's convolution primitives and GELU (CPU only)."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import conv as oc


def _ref_conv(x, w):
    """Stride-1 multi-channel correlation through scipy.ndimage.correlate."""
    D = x.ndim - 1
    out = np.zeros((w.shape[0],) + x.shape[1:])
    for o in range(w.shape[0]):
        for c in range(w.shape[1]):
            out[o] += ndi.correlate(x[c], w[o, c].reshape((3,) * D), mode="constant")
    return out


@pytest.mark.parametrize("shape", [(3, 9, 7), (2, 5, 6, 4)])
def test_conv_matches_library_correlate(shape):
    rng = np.random.default_rng(0)
    D = len(shape) - 1
    x = rng.standard_normal(shape)
    w = rng.standard_normal((4, shape[0], 3 ** D))
    assert np.abs(oc.conv(x, w) - _ref_conv(x, w)).max() < 1e-12


@pytest.mark.parametrize("shape", [(3, 9, 7), (3, 8, 8), (2, 5, 6, 7)])
def test_stride2_is_subsampled_conv(shape):
    """A stride-2, pad-1 convolution equals the stride-1 one read at even
    nodes, giving ceil(n/2) coarse nodes."""
    rng = np.random.default_rng(1)
    D = len(shape) - 1
    x = rng.standard_normal(shape)
    w = rng.standard_normal((5, shape[0], 3 ** D))
    full = _ref_conv(x, w)
    sub = full[(slice(None),) + (slice(None, None, 2),) * D]
    got = oc.conv_stride2(x, w)
    assert got.shape[1:] == tuple((n + 1) // 2 for n in shape[1:])
    assert np.abs(got - sub).max() < 1e-12


@pytest.mark.parametrize("shape", [(3, 9, 7), (3, 8, 8), (2, 5, 6, 7)])
def test_transpose_is_adjoint_of_restriction(shape):
    """With R's own tensor the prolongation is exactly R^T:
    <R x, y> = <x, P y> (real inner product over channels x nodes)."""
    rng = np.random.default_rng(2)
    D = len(shape) - 1
    x = rng.standard_normal(shape)
    w = rng.standard_normal((5, shape[0], 3 ** D))
    cs = tuple((n + 1) // 2 for n in shape[1:])
    y = rng.standard_normal((5,) + cs)
    lhs = np.sum(oc.conv_stride2(x, w) * y)
    rhs = np.sum(x * oc.conv_transpose2(y, w, shape[1:]))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_transpose_one_hot():
    """A coarse unit impulse at X spreads to fine nodes 2X + off with the
    tap weights (bilinear-like footprint of a transposed convolution)."""
    w = np.zeros((1, 1, 9))
    w[0, 0] = np.arange(1, 10)
    e = np.zeros((1, 4, 4))
    e[0, 1, 2] = 1.0
    y = oc.conv_transpose2(e, w, (7, 7))
    expect = np.zeros((7, 7))
    for t, (a, b) in enumerate(oc.taps(2)):
        expect[2 + a, 4 + b] = t + 1
    assert np.array_equal(y[0], expect)


def test_gelu_against_erf():
    xs = np.linspace(-6, 6, 97)
    ref = np.array([0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in xs])
    assert np.abs(oc.gelu(xs) - ref).max() < 1e-15
    assert oc.gelu(np.array([0.0]))[0] == 0.0
