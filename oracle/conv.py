"""Multi-channel 3^D convolutions and GELU (oracle, test infrastructure).

Fields are channel-first float64 arrays [C, n_0, ..., n_{D-1}].  Weights are
[d0][d1][3^D] with taps in row-major order (tap offset d_a - 1 per axis).

Readings where the paper is silent (it only says 3x3 kernels, strided
convolution for restriction and transposed convolution for prolongation,
Sec. 3.2): cross-correlation, zero padding of one cell, no bias (a bias would
make the V-cycle affine, against the linearity the paper requires), restriction
with stride 2 giving ceil(n/2) coarse nodes (coarse node X sits at fine node
2X), prolongation as the exact transpose structure of that restriction with
its own weight tensor and output size forced to the fine size.

Parity pins (tests/test_oracle_conv.py): stride-1 and strided convolution
against scipy.ndimage.correlate, transposed convolution as the adjoint of the
strided one, GELU against math.erf.
"""
import itertools
import math
import numpy as np
from scipy.special import erf


def taps(dim):
    """Tap offsets in row-major order: tuples in {-1, 0, 1}^dim."""
    return [tuple(d - 1 for d in t) for t in itertools.product(range(3), repeat=dim)]


def conv(x, w):
    """Stride-1 convolution: y[o, p] = sum_c sum_t w[o, c, t] x[c, p + off_t]."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    D = x.ndim - 1
    spatial = x.shape[1:]
    xp = np.pad(x, [(0, 0)] + [(1, 1)] * D)
    y = np.zeros((w.shape[0],) + spatial)
    for t, off in enumerate(taps(D)):
        sl = (slice(None),) + tuple(slice(1 + o, 1 + o + n) for o, n in zip(off, spatial))
        y += np.tensordot(w[:, :, t], xp[sl], axes=([1], [0]))
    return y


def coarse_shape(spatial):
    return tuple((n + 1) // 2 for n in spatial)


def conv_stride2(x, w):
    """Restriction: y[o, X] = sum_c sum_t w[o, c, t] x[c, 2X + off_t], zero padded."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    D = x.ndim - 1
    spatial = x.shape[1:]
    cs = coarse_shape(spatial)
    xp = np.pad(x, [(0, 0)] + [(1, 2)] * D)
    y = np.zeros((w.shape[0],) + cs)
    for t, off in enumerate(taps(D)):
        sl = (slice(None),) + tuple(slice(1 + o, 1 + o + 2 * m, 2) for o, m in zip(off, cs))
        y += np.tensordot(w[:, :, t], xp[sl], axes=([1], [0]))
    return y


def conv_transpose2(e, w, fine_shape):
    """Prolongation: y[c, 2X + off_t] += w[o, c, t] e[o, X], cropped to fine_shape.

    w has shape [C_coarse][C_fine][3^D]."""
    e = np.asarray(e, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    D = e.ndim - 1
    cs = e.shape[1:]
    ypad = np.zeros((w.shape[1],) + tuple(2 * m + 2 for m in cs))
    for t, off in enumerate(taps(D)):
        sl = (slice(None),) + tuple(slice(1 + o, 1 + o + 2 * m, 2) for o, m in zip(off, cs))
        ypad[sl] += np.tensordot(w[:, :, t], e, axes=([0], [0]))
    crop = (slice(None),) + tuple(slice(1, 1 + n) for n in fine_shape)
    return ypad[crop]


def gelu(x):
    """GELU in its exact form x * Phi(x), Phi the standard normal CDF."""
    return 0.5 * x * (1.0 + erf(np.asarray(x) / math.sqrt(2.0)))
