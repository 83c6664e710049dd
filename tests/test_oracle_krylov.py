"""Pins of the oracle's FGMRES and stationary iteration (CPU only)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import helmholtz, krylov, mcmg


def _pml16():
    """16 x 16 interior + 4-cell PML = 24 x 24 = 576 unknowns."""
    n, npml = 16, 4
    c = synth.medium_bump(n, 2)
    h = 1.0 / n
    omega = synth.omega_for_ppw(c, 6.0, h)
    op = helmholtz.setup_operator(c, omega, h, npml)
    f = synth.point_source(n, npml, (0.5, 0.25), 2)
    return op, f, h


def test_fgmres_matches_dense_lu():
    """Random-init McMg preconditioner, no restart (m >= 576), tol 1e-12:
    the FGMRES solution matches LAPACK's dense solve to 1e-10 (a random
    preconditioner needs the full 576 steps: finite termination)."""
    op, f, h = _pml16()
    channels = (2, 4, 8)
    tens = synth.make_weights(2, channels, (2, 2, 2), (2, 2, 2), 0)
    W = mcmg.Weights(2, channels, (2, 2, 2), (2, 2, 2), tens)
    M = mcmg.Preconditioner(W, np.sqrt(op["k2"]), h)
    A = helmholtz.assemble(op).toarray()
    u_lu = np.linalg.solve(A, f.reshape(-1)).reshape(f.shape)
    u, info = krylov.fgmres(lambda x: helmholtz.apply(op, x), M, f, m=600, tol=1e-12, maxit=600)
    assert info["converged"], info["relres_true"]
    err = np.linalg.norm(u - u_lu) / np.linalg.norm(u_lu)
    assert err <= 1e-10, err


def test_identity_preconditioner_matches_scipy_gmres():
    """With M = I, FGMRES(m) is GMRES(m): its residual estimate at every
    inner step equals SciPy's GMRES residual history."""
    op, f, h = _pml16()
    A = helmholtz.assemble(op).tocsr()
    m = 20
    hist_ref = []
    spla.gmres(A, f.reshape(-1), rtol=1e-9, restart=m, maxiter=3,
               callback=lambda pr: hist_ref.append(pr), callback_type="pr_norm")
    _, info = krylov.fgmres(lambda x: helmholtz.apply(op, x), lambda r: r, f,
                            m=m, tol=1e-9, maxit=len(hist_ref))
    ours = np.array(info["hist"][:len(hist_ref)])
    ref = np.array(hist_ref)
    assert len(ours) == len(ref) and len(ref) >= 3 * m - 1
    assert np.max(np.abs(ours - ref) / ref) < 1e-8


def test_exact_inverse_one_iteration():
    op, f, h = _pml16()
    lu = spla.splu(helmholtz.assemble(op).tocsc())
    Minv = lambda r: lu.solve(r.reshape(-1)).reshape(r.shape)
    u, info = krylov.fgmres(lambda x: helmholtz.apply(op, x), Minv, f, m=30, tol=1e-10)
    assert info["iters"] == 1 and info["converged"]
    u2, info2 = krylov.stationary(lambda x: helmholtz.apply(op, x), Minv, f, tol=1e-10)
    assert info2["iters"] == 1 and info2["converged"]


def test_ls_estimate_equals_true_residual():
    """A Z_j = V_{j+1} Hbar_j makes the Givens estimate |g_{j+1}| the exact
    residual of u_j = Z_j y_j; it is non-increasing within a cycle."""
    op, f, h = _pml16()
    channels = (2, 4)
    tens = synth.make_weights(2, channels, (1, 1), (1, 1), 5)
    W = mcmg.Weights(2, channels, (1, 1), (1, 1), tens)
    M = mcmg.Preconditioner(W, np.sqrt(op["k2"]), h)
    Aop = lambda x: helmholtz.apply(op, x)
    _, full = krylov.fgmres(Aop, M, f, m=50, tol=1e-14, maxit=12)
    hist = np.array(full["hist"])
    assert np.all(np.diff(hist) <= 1e-15)
    for j in (1, 4, 8, 12):
        _, info = krylov.fgmres(Aop, M, f, m=50, tol=1e-14, maxit=j)
        assert abs(info["relres_true"] - hist[j - 1]) <= 1e-10 * hist[j - 1]


def test_restart_and_initial_guess():
    """A restarted run resumes from its returned iterate (warm start)."""
    op, f, h = _pml16()
    Aop = lambda x: helmholtz.apply(op, x)
    u1, i1 = krylov.fgmres(Aop, lambda r: r, f, m=10, tol=1e-8, maxit=40)
    u2, i2 = krylov.fgmres(Aop, lambda r: r, f, u0=u1, m=10, tol=1e-8, maxit=40)
    r2 = np.linalg.norm(f - Aop(u2)) / np.linalg.norm(f)
    assert r2 < i1["relres_true"]
    assert abs(r2 - i2["relres_true"]) < 1e-12
