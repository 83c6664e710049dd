"""Born-series outer iterations with the discrete Green operator (oracle,
test infrastructure).

Follows the appendix on the Born-series variant: the scattering potential,
the Lippmann-Schwinger equation, the Born-series residual, the convergent
Born series (Eq. cbs_eq) and its learned replacement by MG.  It also follows
the appendix on the discrete Green operator (Eq. discrete_symbol) and the CBS
parameters of the baseline-configuration appendix (Eq. cbs_gamma).

Readings where the paper is silent or leaves a choice:
  * The FFT diagonalises the PERIODIC five-/seven-point Laplacian on the
    extended grid.  Its eigenvalue at the FFT frequency xi_a = 2 pi m_a /
    (n_a h) is Eq. discrete_symbol, -sum_a (4/h^2) sin^2(pi m_a / n_a).  The
    Born-series solvers therefore act on the periodic operator
        A_per u = -Lap_h^per u - k^2 (1 + i gamma) u,
    where gamma is the sponge damping of Sec. 2.1; the layer absorbs what
    wraps around.  A PML changes the Laplacian itself, so it has no Born
    form here; only the sponge layer, or no layer at all, is accepted.
  * Background: k0^2 = (min k^2 + max k^2) / 2 over the extended grid, the
    CBS centring.
  * Potential and absorption: V = k^2 (1 + i gamma) - k0^2 and
    eps = max |V|.
  * The Green operator carries the CBS absorption,
        G = (-Lap_h^per - k0^2 - i eps)^{-1}.
    The Born residual is then G (f - A_per u) = G (V_eps u + f) - u, with
    V_eps = V - i eps.  Born+McMg runs the same Born iteration as CBS and
    differs only in the preconditioner, so it uses the same G.
  * CBS: u <- u + gamma_cbs (.) G (f - A_per u), with gamma_cbs = 1 + i V / eps.
  * Born+McMg: u <- u + MG(G (f - A_per u)).
  * Both stop when the true residual satisfies |f - A_per u| <= tol |f|,
    in FP64.

The FFT (numpy.fft) serves as a library primitive.

Parity pins (tests/test_oracle_born.py):
  * the periodic operator on discrete plane waves (Eq. discrete_symbol);
  * G against a sparse direct solve of the assembled background operator;
  * the two forms of the Born residual;
  * the exact solution as a fixed point;
  * CBS converging to the sparse LU solution of A_per;
  * the closed-form background of a two-valued medium;
  * agreement of A_per with the Dirichlet operator away from the boundary.
"""
import numpy as np
import scipy.sparse as sp

from . import helmholtz


def _check_unstretched(op):
    for s_node, s_half in op["stretch"]:
        if np.any(s_node != 1.0) or np.any(s_half != 1.0):
            raise ValueError("the Born form needs the sponge layer (a PML stretches the Laplacian)")


def _damped_k2(op):
    """k^2 (1 + i gamma) on the extended grid."""
    return op["k2"] * (1.0 + 1j * op.get("gamma", 0.0))


def apply_periodic(op, u):
    """A_per u with the five-/seven-point Laplacian wrapped around every axis."""
    _check_unstretched(op)
    u = np.asarray(u, dtype=np.complex128)
    h2 = op["h"] ** 2
    out = -_damped_k2(op) * u
    for a in range(u.ndim):
        out = out + (2.0 * u - np.roll(u, 1, axis=a) - np.roll(u, -1, axis=a)) / h2
    return out


def assemble_periodic(op):
    """Sparse matrix of A_per (row-major flattening), built entry by entry."""
    _check_unstretched(op)
    kd = _damped_k2(op)
    shape = kd.shape
    D = len(shape)
    N = kd.size
    h2 = op["h"] ** 2
    rows, cols, vals = [], [], []
    for flat in range(N):
        I = np.unravel_index(flat, shape)
        rows.append(flat); cols.append(flat); vals.append(2.0 * D / h2 - kd[I])
        for a in range(D):
            for step in (-1, 1):
                J = list(I)
                J[a] = (J[a] + step) % shape[a]
                rows.append(flat)
                cols.append(int(np.ravel_multi_index(tuple(J), shape)))
                vals.append(-1.0 / h2)
    return sp.csr_matrix((np.array(vals), (np.array(rows), np.array(cols))), shape=(N, N))


def laplacian_symbol(shape, h):
    """-lambda_h on the FFT grid (Eq. discrete_symbol with xi_a h / 2 = pi m_a / n_a)."""
    tot = np.zeros(shape)
    D = len(shape)
    for a, n in enumerate(shape):
        m = np.arange(n, dtype=np.float64)
        d = 4.0 / h ** 2 * np.sin(np.pi * m / n) ** 2
        shp = [1] * D
        shp[a] = -1
        tot = tot + d.reshape(shp)
    return tot


def background(op, k0sq=None, eps=None):
    """k0^2, V, eps and the Green symbol for the Born iteration."""
    _check_unstretched(op)
    k2 = op["k2"]
    if k0sq is None or k0sq <= 0:
        k0sq = 0.5 * (float(np.min(k2)) + float(np.max(k2)))
    V = _damped_k2(op) - k0sq
    if eps is None or eps <= 0:
        eps = float(np.max(np.abs(V)))
    if not eps > 0:
        raise ValueError("eps = 0: the Born background needs a scattering potential or a sponge")
    sym = laplacian_symbol(k2.shape, op["h"]) - k0sq - 1j * eps
    return {"k0sq": float(k0sq), "eps": float(eps), "V": V, "sym": sym}


def green(bg, x):
    """G x = F^{-1}[ F[x] / (-lambda_h - k0^2 - i eps) ]."""
    return np.fft.ifftn(np.fft.fftn(np.asarray(x, dtype=np.complex128)) / bg["sym"])


def born_residual(op, bg, f, u):
    """r_BS = G (f - A_per u)."""
    return green(bg, np.asarray(f, dtype=np.complex128) - apply_periodic(op, u))


def cbs_gamma(bg):
    """Eq. cbs_gamma: gamma = 1 + i V / eps."""
    return 1.0 + 1j * bg["V"] / bg["eps"]


def born_iterate(op, bg, apply_P, f, u0=None, tol=1e-6, maxit=1000):
    """u <- u + P(G (f - A_per u)) until |f - A_per u| <= tol |f|.

    P = gamma_cbs (.) gives CBS (Eq. cbs_eq); P = MG gives Born+McMg."""
    f = np.asarray(f, dtype=np.complex128)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.complex128)
    fnorm = float(np.linalg.norm(f))
    hist = []
    its = 0
    while True:
        r = f - apply_periodic(op, u)
        rel = float(np.linalg.norm(r)) / fnorm if fnorm > 0 else 0.0
        hist.append(rel)
        if rel <= tol or its >= maxit or not np.isfinite(rel):
            return u, {"iters": its, "converged": rel <= tol, "relres_true": rel, "hist": hist}
        u = u + apply_P(green(bg, r))
        its += 1


def cbs(op, bg, f, u0=None, tol=1e-6, maxit=5000):
    g = cbs_gamma(bg)
    return born_iterate(op, bg, lambda x: g * x, f, u0, tol, maxit)


def born_mcmg(op, bg, apply_MG, f, u0=None, tol=1e-6, maxit=1000):
    return born_iterate(op, bg, apply_MG, f, u0, tol, maxit)


def sponge_operator(c, omega, h, npml, gamma_max=None):
    """Operator description with the sponge layer (the Born solvers' setting)."""
    return helmholtz.setup_operator(c, omega, h, npml, absorber="sponge", gamma_max=gamma_max)
