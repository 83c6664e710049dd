"""Pins of the oracle's setup (Alg. 1) and V-cycle (Alg. 2) (CPU only)."""
import math

import numpy as np
import pytest

import synth
from oracle import conv as oc
from oracle import helmholtz, mcmg


def _small(dim=2, n=20, npml=4, channels=(2, 4, 6), nu=2, seed=3):
    L = len(channels)
    tens = synth.make_weights(dim, channels, (nu,) * L, (nu,) * L, seed)
    W = mcmg.Weights(dim, channels, (nu,) * L, (nu,) * L, tens)
    c = synth.medium_bump(n, dim)
    h = 1.0 / n
    omega = synth.omega_for_ppw(c, 10.0, h)
    op = helmholtz.setup_operator(c, omega, h, npml)
    return W, op, h


@pytest.mark.parametrize("dim", [2, 3])
def test_vcycle_linear_over_reals(dim):
    """Sec. 3.2: for a fixed medium MG is linear in the residual; the lift and
    projection carry no activation.  MG(0) = 0 exactly."""
    W, op, h = _small(dim=dim, n=12 if dim == 3 else 20, npml=2 if dim == 3 else 4,
                      channels=(2, 3) if dim == 3 else (2, 4, 6))
    M = mcmg.Preconditioner(W, np.sqrt(op["k2"]), h)
    shp = op["k2"].shape
    r1 = synth.random_rhs(shp, 1)
    r2 = synth.random_rhs(shp, 2)
    a, b = 0.7, -1.9
    lhs = M(a * r1 + b * r2)
    rhs = a * M(r1) + b * M(r2)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)
    z0 = M(np.zeros(shp, dtype=complex))
    assert np.all(z0 == 0)
    # real-linear only: multiplying by i does not commute with MG
    zi = M(1j * r1)
    assert np.linalg.norm(zi - 1j * M(r1)) > 1e-3 * np.linalg.norm(zi)


def _dilate(mask):
    D = mask.ndim
    out = mask.copy()
    for off in oc.taps(D):
        out |= np.roll(np.pad(mask, 1), off, axis=tuple(range(D)))[tuple(slice(1, -1) for _ in range(D))]
    return out


def test_vcycle_locality():
    """MG(delta_x) is exactly zero outside the receptive field obtained by
    propagating the support through the operation sequence of Alg. 2 (exact
    zeros survive floating point)."""
    dim, n, npml = 2, 40, 0
    channels, nu = (2, 3), 1
    tens = synth.make_weights(dim, channels, (nu, nu), (nu, nu), 4)
    W = mcmg.Weights(dim, channels, (nu, nu), (nu, nu), tens)
    c = np.ones((n, n))
    op = helmholtz.setup_operator(c, 10.0, 1.0 / n, npml)
    M = mcmg.Preconditioner(W, np.sqrt(op["k2"]), 1.0 / n)
    r = np.zeros((n, n), dtype=complex)
    r[20, 13] = 1.0
    z = M(r)
    # support propagation
    supp_r1 = _dilate(r != 0)                      # g_lift
    # level 1 pre-smoothing: one step from e = 0 -> S(r1): two convs
    e1 = _dilate(_dilate(supp_r1))
    # restriction of r1 - A e1
    t = supp_r1 | _dilate(e1)
    tc = _dilate(t)[::2, ::2]                      # stride-2 conv support
    # coarse level: one step from 0
    e2 = _dilate(_dilate(tc))
    # prolongation: coarse node X reaches fine 2X + {-1,0,1}
    up = np.zeros((n, n), dtype=bool)
    for X, Y in zip(*np.nonzero(e2)):
        up[max(2 * X - 1, 0):2 * X + 2, max(2 * Y - 1, 0):2 * Y + 2] = True
    e1b = e1 | up
    # post-smoothing: e += S(r1 - A e)
    e1c = e1b | _dilate(_dilate(supp_r1 | _dilate(e1b)))
    supp_z = _dilate(e1c)                          # g_proj
    assert not supp_z.all(), "test grid too small to exercise locality"
    assert np.all(z[~supp_z] == 0)
    assert np.count_nonzero(z[supp_z]) > 0.9 * supp_z.sum()


def _textbook_vcycle(r, kappa, h, L, nu1, nu2, omega_j):
    """Classical geometric multigrid V-cycle (Sec. 2.2) for (-Lap_h + kappa)
    with weighted Jacobi, full weighting and bilinear prolongation, coarse
    node I at fine node 2I, Dirichlet zero outside every level's grid."""
    def M(u, hl):
        up = np.pad(u, 1)
        return (4 * u - up[2:, 1:-1] - up[:-2, 1:-1] - up[1:-1, 2:] - up[1:-1, :-2]) / hl ** 2 + kappa * u

    def jacobi(u, f, hl, steps):
        dinv = omega_j / (4 / hl ** 2 + kappa)
        for _ in range(steps):
            u = u + dinv * (f - M(u, hl))
        return u

    def restrict(x):
        n0, n1 = x.shape
        m0, m1 = (n0 + 1) // 2, (n1 + 1) // 2
        xp = np.pad(x, 1)
        y = np.zeros((m0, m1), dtype=x.dtype)
        for I in range(m0):
            for J in range(m1):
                acc = 0
                for a, wa in ((-1, .25), (0, .5), (1, .25)):
                    for b, wb in ((-1, .25), (0, .5), (1, .25)):
                        acc += wa * wb * xp[2 * I + a + 1, 2 * J + b + 1]
                y[I, J] = acc
        return y

    def prolong(e, shape):
        y = np.zeros((shape[0] + 2, shape[1] + 2), dtype=e.dtype)
        for I in range(e.shape[0]):
            for J in range(e.shape[1]):
                for a, wa in ((-1, .5), (0, 1.), (1, .5)):
                    for b, wb in ((-1, .5), (0, 1.), (1, .5)):
                        y[2 * I + a + 1, 2 * J + b + 1] += wa * wb * e[I, J]
        return y[1:-1, 1:-1]

    def cycle(f, l, hl):
        u = jacobi(np.zeros_like(f), f, hl, nu1)
        if l == L:
            return u
        fc = restrict(f - M(u, hl))
        u = u + prolong(cycle(fc, l + 1, 2 * hl), f.shape)
        return jacobi(u, f, hl, nu2)

    return cycle(r, 1, h)


def _textbook_mcmg(n, L, kappa, h, omega_j, nu):
    """Weights and features that make McMg's V-cycle the textbook one."""
    dim = 2
    channels = (2,) * L
    eye = np.zeros((2, 2, 9))
    eye[0, 0, 4] = eye[1, 1, 4] = 1.0
    lap = np.array([0, -1, 0, -1, 4, -1, 0, -1, 0], dtype=float)
    fw = np.outer([.25, .5, .25], [.25, .5, .25]).reshape(-1)
    tens = [{"kind": "f_lift", "level": 0, "step": 0, "w": np.zeros((2, 1, 9))},
            {"kind": "g_lift", "level": 0, "step": 0, "w": eye},
            {"kind": "g_proj", "level": 0, "step": 0, "w": eye}]
    feats = {"a": [None], "s": [None]}
    side = n
    for l in range(1, L + 1):
        hl = h * 2 ** (l - 1)
        Wl = np.zeros((2, 2, 9))
        Wl[0, 0] = Wl[1, 1] = lap / hl ** 2
        tens += [{"kind": "f_s", "level": l, "step": 0, "w": np.zeros((2, 2, 9))},
                 {"kind": "W", "level": l, "step": 0, "w": Wl},
                 {"kind": "KA", "level": l, "step": 0, "w": eye},
                 {"kind": "KS", "level": l, "step": 0, "w": eye}]
        for i in range(1, 2 * nu + 1):
            tens.append({"kind": "Wsm", "level": l, "step": i, "w": eye})
        if l < L:
            R = np.zeros((2, 2, 9))
            R[0, 0] = R[1, 1] = fw
            tens += [{"kind": "f_a", "level": l, "step": 0, "w": np.zeros((2, 2, 9))},
                     {"kind": "R", "level": l, "step": 0, "w": R},
                     {"kind": "P", "level": l, "step": 0, "w": 4 * R}]
        feats["a"].append(np.full((2, side, side), kappa))
        feats["s"].append(np.full((2, side, side), omega_j / (4 / hl ** 2 + kappa)))
        side = (side + 1) // 2
    W = mcmg.Weights(dim, channels, (nu,) * L, (nu,) * L, tens)
    return W, feats


@pytest.mark.parametrize("n,kappa", [(33, 0.0), (24, 50.0)])
def test_textbook_reduction(n, kappa):
    """Hand-set channel-diagonal weights (W_l = 5-point Laplacian at h_l,
    KA = KS = Wsm = identity, a_l = kappa, s_l = omega_J / diag, R = full
    weighting, P = 4 R^T, identity lift/projection) turn Alg. 2 into a
    classical GMG V-cycle with weighted Jacobi (App. A.3's SL-style smoother,
    omega = 0.66, (2,2) sweeps, coarse level by the same smoother)."""
    L, nu, omega_j = 3, 2, 0.66
    h = 1.0 / n
    W, feats = _textbook_mcmg(n, L, kappa, h, omega_j, nu)
    rng = np.random.default_rng(7)
    r = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    got = mcmg.vcycle(W, feats, r)
    ref = _textbook_vcycle(r, kappa, h, L, nu, nu, omega_j)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_textbook_poisson_contracts():
    """Sanity band: the textbook V-cycle reduces the Poisson error."""
    n, L, nu, omega_j = 33, 4, 2, 0.66
    h = 1.0 / n
    W, feats = _textbook_mcmg(n, L, 0.0, h, omega_j, nu)
    rng = np.random.default_rng(8)
    u_true = rng.standard_normal((n, n)) + 0j

    def Apply(u):
        up = np.pad(u, 1)
        return (4 * u - up[2:, 1:-1] - up[:-2, 1:-1] - up[1:-1, 2:] - up[1:-1, :-2]) / h ** 2

    f = Apply(u_true)
    u = np.zeros_like(f)
    errs = []
    for _ in range(6):
        u = u + mcmg.vcycle(W, feats, f - Apply(u))
        errs.append(np.linalg.norm(u - u_true))
    rate = (errs[-1] / errs[1]) ** (1 / 4)
    assert rate < 0.5, rate


def test_setup_one_hot_closed_form():
    """Alg. 1 with one-hot kernels: a_1 = GELU(w m(x + off)), s_1 =
    GELU(v a_1(x + off')), a_2 = GELU(u a_1(2X + off'')) with zero values
    outside the grid, m = k h."""
    dim, n = 2, 9
    channels = (2, 2)
    tens = synth.make_weights(dim, channels, (1, 1), (1, 1), 0)
    for t in tens:
        t["w"] = np.zeros_like(t["w"])
    get = {(t["kind"], t["level"]): t for t in tens}
    get[("f_lift", 0)]["w"][0, 0, 1] = 2.0      # tap (-1, 0)
    get[("f_lift", 0)]["w"][1, 0, 5] = -1.0     # tap (0, +1)
    get[("f_s", 1)]["w"][0, 1, 8] = 0.5         # tap (+1, +1), channel 1 -> 0
    get[("f_a", 1)]["w"][1, 0, 0] = 3.0         # tap (-1, -1), channel 0 -> 1
    W = mcmg.Weights(dim, channels, (1, 1), (1, 1), tens)
    rng = np.random.default_rng(0)
    k = rng.uniform(5, 20, size=(n, n))
    h = 0.05
    m = k * h
    F = mcmg.setup(W, k, h)
    g = lambda v: 0.5 * v * (1 + np.vectorize(math.erf)(v / math.sqrt(2)))
    mp = np.pad(m, 1)
    a0 = g(2.0 * mp[0:n, 1:n + 1])
    a1 = g(-1.0 * mp[1:n + 1, 2:n + 2])
    assert np.allclose(F["a"][1][0], a0, atol=1e-15, rtol=1e-14)
    assert np.allclose(F["a"][1][1], a1, atol=1e-15, rtol=1e-14)
    a1p = np.pad(a1, 1)
    assert np.allclose(F["s"][1][0], g(0.5 * a1p[2:n + 2, 2:n + 2]), atol=1e-15, rtol=1e-14)
    assert np.allclose(F["s"][1][1], 0.0)
    a0p = np.pad(a0, 1)
    nc = (n + 1) // 2
    expect = g(3.0 * a0p[0:2 * nc:2, 0:2 * nc:2])
    assert F["a"][2].shape == (2, nc, nc)
    assert np.allclose(F["a"][2][1], expect, atol=1e-15, rtol=1e-14)
    assert np.allclose(F["a"][2][0], 0.0)


def _tap_index(off):
    """Row-major tap index of an offset in {-1, 0, 1}^D."""
    idx = 0
    for o in off:
        idx = 3 * idx + (o + 1)
    return idx


def _modulation_case(dim):
    """One level, nu1 = 2, spatially varying features, one-hot off-centre
    kernels on distinct channel pairs, identity lift/projection."""
    n = 11
    channels = (2,)
    tens = synth.make_weights(dim, channels, (2,), (0,), 0)
    for t in tens:
        t["w"] = np.zeros_like(t["w"])
    get = {(t["kind"], t["step"]): t for t in tens}
    ctr = _tap_index((0,) * dim)
    for kind in ("g_lift", "g_proj"):
        get[(kind, 0)]["w"][0, 0, ctr] = get[(kind, 0)]["w"][1, 1, ctr] = 1.0
    # offsets (the input a one-hot tap reads, relative to the output node)
    sS = (1, 0) if dim == 2 else (1, 0, -1)
    sA = (-1, -1) if dim == 2 else (-1, -1, 0)
    sW = (0, 1) if dim == 2 else (0, 1, 1)
    s1 = (0, -1) if dim == 2 else (0, -1, 1)
    s2 = (1, 1) if dim == 2 else (1, 1, -1)
    wW = 0.75
    get[("KS", 0)]["w"][1, 0, _tap_index(sS)] = 1.0    # channel 0 -> 1
    get[("KA", 0)]["w"][0, 1, _tap_index(sA)] = 1.0    # channel 1 -> 0
    get[("W", 0)]["w"][0, 1, _tap_index(sW)] = wW      # channel 1 -> 0
    get[("Wsm", 1)]["w"][1, 1, _tap_index(s1)] = 1.0
    get[("Wsm", 2)]["w"][1, 1, _tap_index(s2)] = 1.0
    W = mcmg.Weights(dim, channels, (2,), (0,), tens)
    rng = np.random.default_rng(11)
    shape = (n,) * dim
    a = rng.uniform(0.5, 2.0, size=(2,) + shape)
    s = rng.uniform(0.5, 2.0, size=(2,) + shape)
    feats = {"a": [None, a], "s": [None, s]}
    x0 = (5,) * dim
    return W, feats, shape, x0, dict(sS=sS, sA=sA, sW=sW, s1=s1, s2=s2, wW=wW)


def _modulation_expected(feats, shape, x0, o):
    """Closed form of Alg. 2 for the case above on an impulse r = delta_{x0}
    (real part), with Eq. pyhs_conv's order c (.) (K_x * x): a one-hot tap
    reading offset d moves an impulse at p to p - d, and the feature value
    that multiplies it is the one at the node where the convolution's output
    sits.  Only channel 1 of e is ever nonzero, so z = i e[1]."""
    a0 = feats["a"][1][0]
    s1 = feats["s"][1][1]
    sub = lambda p, *ds: tuple(pi - sum(d[i] for d in ds) for i, pi in enumerate(p))
    z = np.zeros(shape, dtype=complex)
    # step 1 from e = 0: e1 = Wsm1 * (s (.) (KS * r1))
    p1 = sub(x0, o["sS"])
    q1 = sub(p1, o["s1"])
    e1 = s1[p1]
    z[q1] += 1j * e1
    # step 2: t = r1 - W * e1 - a (.) (KA * e1) lives in channel 0
    t = {x0: 1.0}
    qa = sub(q1, o["sA"])
    qw = sub(q1, o["sW"])
    t[qa] = t.get(qa, 0.0) - a0[qa] * e1
    t[qw] = t.get(qw, 0.0) - o["wW"] * e1
    for p, v in t.items():
        pu = sub(p, o["sS"])
        z[sub(pu, o["s2"])] += 1j * s1[pu] * v
    return z


@pytest.mark.parametrize("dim", [2, 3])
def test_feature_modulation_order_closed_form(dim):
    """Eq. pyhs_conv: a physical feature modulates the OUTPUT of the linear
    convolution, Phi = c (.) (K_x * x), in both the level operator A_l and the
    smoother S_l (Sec. 3.2).  With spatially varying a_l, s_l and one-hot
    off-centre kernels on distinct channel pairs, an impulse's image carries
    the feature values at the convolutions' output nodes, not at their
    source nodes."""
    W, feats, shape, x0, o = _modulation_case(dim)
    r = np.zeros(shape, dtype=complex)
    r[x0] = 1.0
    got = mcmg.vcycle(W, feats, r)
    ref = _modulation_expected(feats, shape, x0, o)
    assert np.count_nonzero(ref) == 4
    assert np.abs(got - ref).max() <= 1e-15 * np.abs(ref).max()


@pytest.mark.parametrize("which", ["level_op", "smoother"])
def test_feature_modulation_order_rejects_swapped_oracle(which, monkeypatch):
    """The closed-form pin above fails when the oracle modulates the input of
    the convolution instead (K * (a (.) e) or K * (s (.) x)): planted in the
    oracle, on the CPU."""
    def level_op_swapped(wts, feats, l, e):
        return oc.conv(e, wts("W", l)) + oc.conv(feats["a"][l] * e, wts("KA", l))

    def smoother_swapped(wts, feats, l, i, x):
        return oc.conv(oc.conv(feats["s"][l] * x, wts("KS", l)), wts("Wsm", l, i))

    monkeypatch.setattr(mcmg, which, level_op_swapped if which == "level_op" else smoother_swapped)
    W, feats, shape, x0, o = _modulation_case(2)
    r = np.zeros(shape, dtype=complex)
    r[x0] = 1.0
    got = mcmg.vcycle(W, feats, r)
    ref = _modulation_expected(feats, shape, x0, o)
    assert np.abs(got - ref).max() > 1e-3 * np.abs(ref).max()
