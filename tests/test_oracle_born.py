"""Pins of the oracle's Born-series iterations and discrete Green operator
against what the paper and the mathematics fix (CPU only)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import born, helmholtz
import synth


def _sponge_problem(n, npml, dim, gamma_max, ppw=10.0, seed=0):
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    c = synth.medium_bump(n, dim)
    if seed:
        c = c * rng.uniform(0.9, 1.1, size=c.shape)
    omega = synth.omega_for_ppw(c, ppw, h)
    return born.sponge_operator(c, omega, h, npml, gamma_max=gamma_max)


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("shape", [(12, 18), (7, 9, 10)])
def test_periodic_operator_on_plane_waves(shape):
    """Eq. discrete_symbol: on the periodic grid every FFT mode is an exact
    eigenvector of the five-/seven-point Laplacian, eigenvalue
    -(4/h^2) sum_a sin^2(pi m_a / n_a), including modes above n/2 and
    uneven sides."""
    h = 0.37
    k = 2.1
    op = {"k2": np.full(shape, k * k), "h": h,
          "stretch": [(np.ones(n, complex), np.ones(n + 1, complex)) for n in shape]}
    idx = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    for m in [(1,) + (0,) * (len(shape) - 1), tuple(n - 1 for n in shape),
              tuple(n // 2 for n in shape), tuple(3 % n for n in shape)]:
        w = np.exp(2j * math.pi * sum(ma * Ia / n for ma, Ia, n in zip(m, idx, shape)))
        lam = sum(4.0 / h ** 2 * math.sin(math.pi * ma / n) ** 2 for ma, n in zip(m, shape))
        err = np.abs(born.apply_periodic(op, w) - (lam - k * k) * w).max()
        assert err < 1e-12 * (lam + k * k), (m, err)


@pytest.mark.parametrize("dim,n,npml", [(2, 16, 4), (3, 6, 2)])
def test_green_inverts_the_background_operator(dim, n, npml):
    """G x solves (-Lap_h^per - k0^2 - i eps) y = x: the sparse background
    operator is A_per + diag(V) - i eps I, assembled entry by entry and
    solved directly."""
    op = _sponge_problem(n, npml, dim, gamma_max=0.8, seed=3)
    bg = born.background(op)
    A = born.assemble_periodic(op)
    N = A.shape[0]
    B0 = A + sp.diags(bg["V"].ravel()) - 1j * bg["eps"] * sp.identity(N)
    x = _rand(op["k2"].shape, 1)
    y_lu = spla.spsolve(B0.tocsc(), x.ravel())
    y = born.green(bg, x).ravel()
    assert np.linalg.norm(y - y_lu) / np.linalg.norm(y_lu) < 1e-12


def test_born_residual_two_forms_and_fixed_point():
    """The Born-series residual G(V_eps u + f) - u equals G(f - A_per u), and
    the exact solution of A_per u = f is a fixed point of the Born iteration
    (the Lippmann-Schwinger equation)."""
    op = _sponge_problem(20, 4, 2, gamma_max=1.0, seed=5)
    bg = born.background(op)
    A = born.assemble_periodic(op)
    N = A.shape[0]
    B0 = (A + sp.diags(bg["V"].ravel()) - 1j * bg["eps"] * sp.identity(N)).tocsc()
    shape = op["k2"].shape
    u = _rand(shape, 2)
    f = _rand(shape, 3)
    Veps = (bg["V"] - 1j * bg["eps"]).ravel()
    lhs = spla.spsolve(B0, Veps * u.ravel() + f.ravel()) - u.ravel()
    rhs = born.born_residual(op, bg, f, u).ravel()
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(lhs) < 1e-11
    ustar = spla.spsolve(A.tocsc(), f.ravel()).reshape(shape)
    r = born.born_residual(op, bg, f, ustar)
    assert np.linalg.norm(r) / np.linalg.norm(ustar) < 1e-11


def test_assembly_matches_apply_and_dirichlet_interior():
    """The entry-by-entry matrix of A_per equals the rolled-stencil apply, and
    on fields supported away from the boundary A_per equals the Dirichlet
    operator of the other solvers (sponge layer, no stretching)."""
    op = _sponge_problem(12, 3, 2, gamma_max=2.0, seed=7)
    shape = op["k2"].shape
    u = _rand(shape, 4)
    A = born.assemble_periodic(op)
    assert np.abs(A @ u.ravel() - born.apply_periodic(op, u).ravel()).max() < 1e-10 * np.abs(u).max() * 4 / op["h"] ** 2
    v = np.zeros(shape, complex)
    v[2:-2, 2:-2] = u[2:-2, 2:-2]
    d = born.apply_periodic(op, v) - helmholtz.apply(op, v)
    assert np.abs(d).max() < 1e-9
    # ... and they differ on the boundary rows by the wrapped couplings
    w = np.zeros(shape, complex)
    w[0, 5] = 1.0
    d = born.apply_periodic(op, w) - helmholtz.apply(op, w)
    assert abs(d[-1, 5] + 1.0 / op["h"] ** 2) < 1e-9


def test_background_closed_form():
    """Two-valued medium without a layer: k0^2 is the midpoint of the two
    k^2, V = +-(k1^2 - k2^2)/2, eps = |k1^2 - k2^2| / 2, and gamma_cbs lies on
    the circle |gamma - 1| = 1 (here 1 +- i)."""
    c = np.ones((10, 10))
    c[:, 5:] = 2.0
    op = helmholtz.setup_operator(c, 30.0, 0.1, 0, absorber="sponge")
    bg = born.background(op)
    k1, k2 = 30.0 ** 2, (30.0 / 2.0) ** 2
    assert abs(bg["k0sq"] - 0.5 * (k1 + k2)) < 1e-9
    assert abs(bg["eps"] - 0.5 * (k1 - k2)) < 1e-9
    g = born.cbs_gamma(bg)
    assert np.allclose(np.sort(np.unique(np.round(g.imag, 12))), [-1.0, 1.0])
    assert np.allclose(g.real, 1.0)


def test_cbs_converges_to_the_direct_solution():
    """CBS (Eq. cbs_eq with Eq. cbs_gamma and eps = max |V|) is a convergent
    iteration: it reaches the sparse LU solution of A_per u = f."""
    op = _sponge_problem(24, 6, 2, gamma_max=0.5, seed=11)
    bg = born.background(op)
    f = synth.point_source(24, 6, (0.5, 0.25), 2)
    u, info = born.cbs(op, bg, f, tol=1e-9, maxit=20000)
    assert info["converged"], info["relres_true"]
    ustar = spla.spsolve(born.assemble_periodic(op).tocsc(), f.ravel()).reshape(f.shape)
    assert np.linalg.norm(u - ustar) / np.linalg.norm(ustar) < 1e-6
    assert info["iters"] > 10


def test_pml_is_rejected():
    op = helmholtz.setup_operator(np.ones((8, 8)), 10.0, 0.125, 2, absorber="pml")
    with pytest.raises(ValueError):
        born.background(op)


def test_born_mcmg_with_exact_inverse_preconditioner():
    """With P = (G A_per)^{-1}, the inverse of the Born-preconditioned
    operator that Born+McMg learns, one Born step gives the exact solution."""
    op = _sponge_problem(10, 3, 2, gamma_max=1.0, seed=13)
    bg = born.background(op)
    A = born.assemble_periodic(op).toarray()
    N = A.shape[0]
    shape = op["k2"].shape
    G = np.stack([born.green(bg, e.reshape(shape)).ravel() for e in np.eye(N)], axis=1)
    P = np.linalg.inv(G @ A)
    f = _rand(shape, 6)
    u, info = born.born_mcmg(op, bg, lambda r: (P @ r.ravel()).reshape(shape), f, tol=1e-10, maxit=3)
    assert info["iters"] == 1 and info["converged"]
