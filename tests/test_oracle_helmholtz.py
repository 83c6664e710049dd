"""Pins of the oracle's Helmholtz + PML operator against what the paper and
the mathematics fix (CPU only)."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.sparse.linalg as spla
from scipy.special import hankel1

from oracle import helmholtz


def _const_op(shape, k, h, s=1.0 + 0j):
    """Operator with constant k and a constant stretch s on every axis."""
    return {"k2": np.full(shape, float(k) ** 2), "h": h,
            "stretch": [(np.full(n, s, dtype=complex), np.full(n + 1, s, dtype=complex))
                        for n in shape]}


@pytest.mark.parametrize("dim,n", [(2, 24), (3, 12)])
@pytest.mark.parametrize("s", [1.0 + 0j, 1.0 + 0.7j])
def test_plane_wave_symbol(dim, n, s):
    """Eq. discrete_symbol: the 5/7-point Laplacian has symbol
    -(4/h^2) sum sin^2(xi h / 2) on a discrete plane wave; with a constant
    stretch s each second difference is divided by s^2.  Away from the
    boundary A u = [(4/(h^2 s^2)) sum_a sin^2(xi_a h/2) - k^2] u."""
    h = 1.0 / n
    k = 7.3
    op = _const_op((n,) * dim, k, h, s)
    x = np.arange(n) * h
    X = np.meshgrid(*([x] * dim), indexing="ij")
    # several wave vectors, including near Nyquist and near the shell |xi| = k
    ps = [(1,) + (0,) * (dim - 1), (3,) + (2,) * (dim - 1), (n // 2 - 1,) * dim,
          (n // 2,) + (1,) * (dim - 1)]
    for p in ps:
        xi = [2 * math.pi * pa / (n * h) for pa in p]
        u = np.exp(1j * sum(xa * Xa for xa, Xa in zip(xi, X)))
        Au = helmholtz.apply(op, u)
        sym = 4.0 / (h * h * s * s) * sum(math.sin(xa * h / 2) ** 2 for xa in xi) - k * k
        inner = tuple(slice(1, n - 1) for _ in range(dim))
        err = np.abs(Au[inner] - sym * u[inner]).max() / (abs(sym) + k * k)
        assert err < 1e-13, (p, err)
    # near the shell |xi| ~ k
    xi = [k / math.sqrt(dim)] * dim
    u = np.exp(1j * sum(xa * Xa for xa, Xa in zip(xi, X)))
    sym = 4.0 / (h * h * s * s) * sum(math.sin(xa * h / 2) ** 2 for xa in xi) - k * k
    inner = tuple(slice(1, n - 1) for _ in range(dim))
    Au = helmholtz.apply(op, u)
    assert np.abs(Au[inner] - sym * u[inner]).max() < 1e-13 * (4 * dim / h ** 2)


def test_reduces_to_paper_stencil():
    """With no absorbing layer the operator is exactly Eq. FDM_stencil:
    (1/h^2) [[0,-1,0],[-1,4-(k h)^2,-1],[0,-1,0]] applied as a spatially
    varying correlation with zero values outside the grid."""
    rng = np.random.default_rng(5)
    n = 17
    h = 1.0 / n
    c = rng.uniform(1.0, 3.0, size=(n, n))
    omega = 20.0
    op = helmholtz.setup_operator(c, omega, h, npml=0)
    u = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    lap = np.array([[0, -1, 0], [-1, 4, -1], [0, -1, 0]], dtype=float) / h ** 2
    ref = (ndi.correlate(u.real, lap, mode="constant") + 1j * ndi.correlate(u.imag, lap, mode="constant"))
    ref -= (omega / c) ** 2 * u
    got = helmholtz.apply(op, u)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("dim,n,npml", [(2, 6, 4), (3, 3, 2)])
def test_stretched_operator_symmetry(dim, n, npml):
    """diag(prod_a s_a) A is complex symmetric: multiplying the stretched
    Laplacian by prod_a s_a gives the divergence form
    sum_a d_a((prod_{b != a} s_b / s_a) d_a), which is symmetric when
    discretised with face values (App. A.1.1)."""
    rng = np.random.default_rng(1)
    c = rng.uniform(1.0, 2.0, size=(n,) * dim)
    h = 1.0 / n
    op = helmholtz.setup_operator(c, 9.0, h, npml)
    A = helmholtz.assemble(op).toarray()
    shape = op["k2"].shape
    dvec = np.ones(shape, dtype=complex)
    for a in range(dim):
        sh = [1] * dim
        sh[a] = -1
        dvec = dvec * op["stretch"][a][0].reshape(sh)
    DA = dvec.reshape(-1)[:, None] * A
    assert np.abs(DA - DA.T).max() <= 1e-13 * np.abs(DA).max()
    assert np.abs(DA - DA.conj().T).max() > 1e-3 * np.abs(DA).max()   # not Hermitian
    # the vectorised operator and the entry-by-entry matrix agree
    u = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    assert np.abs(A @ u.reshape(-1) - helmholtz.apply(op, u).reshape(-1)).max() <= 1e-12 * np.abs(A).max()


def test_pml_profile_shape():
    """sigma vanishes on the interior nodes and grows quadratically into the layer."""
    s_node, s_half = helmholtz.pml_stretch(10, 4, 2.0)
    sig = s_node.imag
    assert np.all(sig[4:14] == 0.0)
    assert np.allclose(sig[:4], 2.0 * (np.arange(4, 0, -1) / 4.0) ** 2)
    assert np.allclose(sig[14:], 2.0 * (np.arange(1, 5) / 4.0) ** 2)
    assert np.allclose(s_half.imag[4], 2.0 * (0.5 / 4) ** 2)
    assert np.all(s_node.real == 1.0)


def _greens_error(sign=+1):
    n, npml = 160, 20
    h = 1.0 / n
    ppw = 30.0
    k = 2 * math.pi / (ppw * h)
    c = np.ones((n, n))
    op = helmholtz.setup_operator(c, k, h, npml)
    if sign < 0:   # planted mistake: stretching with the wrong sign
        op["stretch"] = [(s.conj(), t.conj()) for s, t in op["stretch"]]
    A = helmholtz.assemble(op).tocsc()
    ne = n + 2 * npml
    f = np.zeros((ne, ne), dtype=complex)
    ic = npml + n // 2
    f[ic, ic] = 1.0 / h ** 2
    u = spla.spsolve(A, f.reshape(-1)).reshape(ne, ne)
    idx = np.arange(ne) - ic
    R = np.hypot(*np.meshgrid(idx, idx, indexing="ij")) * h
    ring = (R > 8 * h) & (R < 60 * h)
    ref = 0.25j * hankel1(0, k * R[ring])
    return np.linalg.norm(u[ring] - ref) / np.linalg.norm(ref)


def test_outgoing_greens_function():
    """The operator with its PML reproduces the outgoing free-space Green's
    function (i/4) H_0^(1)(k r) of -Lap - k^2 in 2D (radiation condition of
    Eq. helm) up to discretisation error; a stretch with the opposite sign
    (incoming waves) does not."""
    err = _greens_error(+1)
    assert err < 0.05, err
    assert _greens_error(-1) > 0.3


def _sponge_1d(npml, flip=False):
    import scipy.sparse.linalg as spl
    n = 400
    h = 1.0 / n
    kh = 2 * math.pi / 20
    op = helmholtz.setup_operator(np.ones(n), kh / h, h, npml, absorber="sponge")
    if flip:                                   # the sign as printed: (1 - gamma i)
        op = dict(op)
        op["gamma"] = -op["gamma"]
    j0 = npml + n // 2
    f = np.zeros(n + 2 * npml, dtype=complex)
    f[j0] = 1.0
    u = spl.spsolve(helmholtz.assemble(op).tocsc(), f)
    # exact outgoing solution of the discrete free-space problem:
    # u_j = A e^{i xi h |j - j0|}, cos(xi h) = 1 - (k h)^2 / 2, A = i h^2 / (2 sin xi h)
    xh = math.acos(1 - kh * kh / 2)
    j = np.arange(n + 2 * npml)
    ex = 1j * h * h / (2 * math.sin(xh)) * np.exp(1j * xh * np.abs(j - j0))
    inner = slice(npml, npml + n)
    err = np.linalg.norm(u[inner] - ex[inner]) / np.linalg.norm(ex[inner])
    return u, err


def test_sponge_absorbs_outgoing_waves_in_1d():
    """Sponge layer (Sec. 2.1) with k^2 (1 + i gamma): the interior solution of
    a point source is the discrete outgoing (e^{+ikr}) Green's function up to
    the layer's small reflection, and the field decays through the layer.
    The printed factor (1 - gamma i) yields the incoming solution instead
    (the sign reading this pins)."""
    u, err = _sponge_1d(60)
    assert err < 3e-3, err
    assert abs(u[1]) < 1e-2 * abs(u[60])
    _, err_flip = _sponge_1d(60, flip=True)
    assert err_flip > 1.0, err_flip
    # a longer layer reflects less
    _, err_long = _sponge_1d(100)
    assert err_long < err


def test_sponge_profile_and_symmetry():
    """gamma vanishes in the physical domain, grows quadratically with the
    distance into the layer, saturates at gamma_max; without stretching the
    operator is complex symmetric (A = A^T) and npml = 0 is the paper's
    stencil."""
    n, npml = 12, 4
    c = np.ones((n, n))
    op = helmholtz.setup_operator(c, 10.0, 1.0 / n, npml, absorber="sponge", gamma_max=2.0)
    g = op["gamma"]
    assert np.all(g[npml:npml + n, npml:npml + n] == 0)
    mid = npml + n // 2
    assert np.allclose(g[npml - np.arange(1, npml + 1), mid], 2.0 * (np.arange(1, npml + 1) / npml) ** 2)
    assert g[0, 0] == 2.0 and g.max() == 2.0
    A = helmholtz.assemble(op)
    assert abs(A - A.T).max() == 0
    op0 = helmholtz.setup_operator(c, 10.0, 1.0 / n, 0, absorber="sponge")
    rng = np.random.default_rng(3)
    u = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    lap = np.array([[0, -1, 0], [-1, 4, -1], [0, -1, 0]], dtype=float) * n * n
    ref = ndi.correlate(u.real, lap, mode="constant") + 1j * ndi.correlate(u.imag, lap, mode="constant")
    ref -= op0["k2"] * u
    got = helmholtz.apply(op0, u)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
