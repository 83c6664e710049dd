"""Right-preconditioned restarted FGMRES(m) and the stationary McMg iteration
(oracle, test infrastructure).

The paper uses McMg as a GMRES preconditioner (Sec. 3.3, Sec. 4.1 "GMRES+McMg")
without giving the Krylov details, and as a stationary correction
u <- u + MG(f - A u) (Sec. 3.3, Eq. mcmg_iteration); tolerance is a relative
residual of 1e-6 (Sec. 4.1, evaluation protocol).

Reading: MG is linear over the reals only (it acts on (Re, Im) channels with
real weights), so MG(i r) != i MG(r) in general.  Flexible GMRES (Saad 1993)
stores z_j = MG(v_j) and forms u = u_0 + Z y, which is exact for any
preconditioner, so it is the variant used.  Here: modified Gram-Schmidt,
Givens rotations on the Hessenberg matrix, restart from the true residual
f - A u; iteration count = number of preconditioner applications.

Parity pins (tests/test_oracle_krylov.py): solve of a 576-unknown PML problem
against LAPACK (numpy.linalg.solve) to 1e-10, identity preconditioner against
scipy.sparse.linalg.gmres residual history, exact inverse converging in one
step, and the least-squares estimate equal to the explicit residual at every
inner step.
"""
import numpy as np


def _dot(a, b):
    return np.vdot(a, b)              # sum conj(a) * b


def _norm(a):
    return float(np.sqrt(np.vdot(a, a).real))


def fgmres(apply_A, apply_M, f, u0=None, m=30, tol=1e-6, maxit=500, callback=None):
    """Solve A u = f.  Returns (u, info) with info = {iters, converged,
    relres_true, hist (LS residual estimate / |f| per inner step), restarts}."""
    f = np.asarray(f, dtype=np.complex128)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.complex128)
    fnorm = _norm(f)
    if fnorm == 0.0:
        return np.zeros_like(f), {"iters": 0, "converged": True, "relres_true": 0.0,
                                  "hist": [], "restarts": 0}
    target = tol * fnorm
    r = f - apply_A(u)
    beta = _norm(r)
    hist = []
    its = 0
    restarts = 0
    while True:
        if beta <= target:
            return u, {"iters": its, "converged": True, "relres_true": beta / fnorm,
                       "hist": hist, "restarts": restarts}
        if its >= maxit:
            return u, {"iters": its, "converged": False, "relres_true": beta / fnorm,
                       "hist": hist, "restarts": restarts}
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        j_done = 0
        for j in range(m):
            z = apply_M(V[j])
            Z.append(z)
            w = apply_A(z)
            its += 1
            for i in range(j + 1):
                H[i, j] = _dot(V[i], w)
                w = w - H[i, j] * V[i]
            hn = _norm(w)
            H[j + 1, j] = hn
            colnorm = _norm(H[: j + 2, j])
            # earlier rotations on column j
            for i in range(j):
                x, y = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * x + np.conj(sn[i]) * y
                H[i + 1, j] = -sn[i] * x + cs[i] * y
            # new rotation zeroing H[j+1, j] (real, >= 0)
            a, b = H[j, j], H[j + 1, j].real
            t = np.hypot(abs(a), b)
            if abs(a) == 0.0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / t
                sn[j] = (np.conj(a) / abs(a)) * (b / t)
            H[j, j] = cs[j] * a + np.conj(sn[j]) * b
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            rho = abs(g[j + 1])
            hist.append(rho / fnorm)
            j_done = j + 1
            if callback is not None:
                callback(j, rho)
            if rho <= target or hn <= 1e-14 * colnorm or its >= maxit:
                break
            V.append(w / hn)
        # back-substitution H[:j,:j] y = g[:j]
        k = j_done
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        for i in range(k):
            u = u + y[i] * Z[i]
        r = f - apply_A(u)
        beta = _norm(r)
        restarts += 1


def stationary(apply_A, apply_M, f, u0=None, tol=1e-6, maxit=500):
    """u <- u + MG(f - A u) until |f - A u| <= tol |f| (Eq. mcmg_iteration)."""
    f = np.asarray(f, dtype=np.complex128)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.complex128)
    fnorm = _norm(f)
    hist = []
    its = 0
    r = f - apply_A(u)
    while True:
        rel = _norm(r) / fnorm if fnorm > 0 else 0.0
        hist.append(rel)
        if rel <= tol or its >= maxit or not np.isfinite(rel):
            return u, {"iters": its, "converged": rel <= tol, "relres_true": rel, "hist": hist}
        u = u + apply_M(r)
        its += 1
        r = f - apply_A(u)
