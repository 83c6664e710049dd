"""McMg setup (Alg. 1) and V-cycle MG(r) (Alg. 2) in FP64 (oracle, test
infrastructure).

Sec. 3.1: a physical feature is a nonlinear convolution of the medium,
c = GELU(K_m * m) (Eq. phys_feature); it modulates a linear convolution of
the field, c (.) (K_x * x) (Eq. pyhs_conv).  Alg. 1 builds a_1 = f_lift(k),
s_l = f_s^l(a_l), a_{l+1} = f_a^l(a_l).  Sec. 3.2 defines the smoother
S_l^(i)(x) = W^(i) * (s_l (.) (K_x * x)), the level operator
A_l(x) = W_l * x + a_l (.) (K_x * x), the update e += S^(i)(r - A_l e),
restriction r_{l+1} = R(r_l - A_l e_l), prolongation e_l += P(e_{l+1}) and the
linear lift/projection g_lift, g_proj; Alg. 2 orders them into the V-cycle.

Readings where the paper is silent:
  * the medium input m is the dimensionless k h (the (k h) of Eq.
    FDM_stencil), one channel on the extended grid;
  * f_lift, f_s^l, f_a^l are one convolution + GELU each (the minimal reading
    of Eq. phys_feature); f_a^l has stride 2, like the restriction it mirrors;
  * the K_x inside A_l (KA_l) and inside S_l (KS_l) are distinct tensors, each
    shared by all steps of its level; W^(i) is distinct per step;
  * C_1 = 2: the complex residual enters as (Re, Im) channels and g_lift,
    g_proj are 3^D convolutions 2 -> C_1 and C_1 -> 2;
  * at the coarsest level only the nu1^L pre-smoothing steps run (Alg. 2 has
    no up-cycle step at l = L); the first pre-smoothing step starts from e = 0;
  * no bias anywhere.

Parity pins (tests/test_oracle_mcmg.py): linearity in r for real scalars and
MG(0) = 0 (Sec. 3.2), exact locality against the receptive field, adjointness
of R and P when P carries R's tensor, reduction to a textbook geometric
multigrid V-cycle with hand-set weights (Sec. 2.2, App. A.3 smoother), the
order of feature modulation of Eq. pyhs_conv (the feature multiplies the
convolution's output, in A_l and in S_l) by a closed form with spatially
varying features and one-hot off-centre kernels, and closed-form setup features for one-hot kernels in each step of Alg. 1 (the
paper prints no feature values to compare against).
"""
import numpy as np

from .conv import conv, conv_stride2, conv_transpose2, gelu


class Weights:
    """Weights indexed by (kind, level, step), promoted exactly to float64."""

    def __init__(self, dim, channels, nu1, nu2, tensors):
        self.dim = dim
        self.channels = list(channels)
        self.nu1 = list(nu1)
        self.nu2 = list(nu2)
        self.L = len(channels)
        self._t = {}
        for t in tensors:
            self._t[(t["kind"], t["level"], t["step"])] = np.asarray(t["w"], dtype=np.float64)

    def __call__(self, kind, level=0, step=0):
        return self._t[(kind, level, step)]


def setup(wts, k, h):
    """Alg. 1: per-level cached features a_l, s_l (channel-first float64)."""
    m = (np.asarray(k, dtype=np.float64) * h)[None]
    a = [None] * (wts.L + 1)
    s = [None] * (wts.L + 1)
    a[1] = gelu(conv(m, wts("f_lift")))
    for l in range(1, wts.L + 1):
        s[l] = gelu(conv(a[l], wts("f_s", l)))
        if l < wts.L:
            a[l + 1] = gelu(conv_stride2(a[l], wts("f_a", l)))
    return {"a": a, "s": s}


def level_op(wts, feats, l, e):
    """A_l(e) = W_l * e + a_l (.) (KA_l * e)."""
    return conv(e, wts("W", l)) + feats["a"][l] * conv(e, wts("KA", l))


def smoother(wts, feats, l, i, x):
    """S_l^(i)(x) = Wsm_l^(i) * (s_l (.) (KS_l * x))."""
    return conv(feats["s"][l] * conv(x, wts("KS", l)), wts("Wsm", l, i))


def vcycle(wts, feats, r):
    """Alg. 2: e = MG(r) for a complex residual r on the extended grid."""
    L = wts.L
    r = np.asarray(r, dtype=np.complex128)
    r2 = np.stack([r.real, r.imag])
    rl = [None] * (L + 1)
    el = [None] * (L + 1)
    rl[1] = conv(r2, wts("g_lift"))
    for l in range(1, L + 1):
        e = np.zeros_like(rl[l])
        for i in range(1, wts.nu1[l - 1] + 1):
            e = e + smoother(wts, feats, l, i, rl[l] - level_op(wts, feats, l, e))
        el[l] = e
        if l < L:
            rl[l + 1] = conv_stride2(rl[l] - level_op(wts, feats, l, e), wts("R", l))
    for l in range(L - 1, 0, -1):
        e = el[l] + conv_transpose2(el[l + 1], wts("P", l), el[l].shape[1:])
        for i in range(1, wts.nu2[l - 1] + 1):
            e = e + smoother(wts, feats, l, wts.nu1[l - 1] + i, rl[l] - level_op(wts, feats, l, e))
        el[l] = e
    out = conv(el[1], wts("g_proj"))
    return out[0] + 1j * out[1]


class Preconditioner:
    """MG(.) bound to one medium: setup once, apply many times."""

    def __init__(self, wts, k, h):
        self.wts = wts
        self.feats = setup(wts, k, h)

    def __call__(self, r):
        return vcycle(self.wts, self.feats, r)
