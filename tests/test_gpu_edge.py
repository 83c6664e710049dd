"""Degenerate inputs through the C ABI: a zero right-hand side, maxit = 0,
an initial guess that already solves the system, a non-finite right-hand
side, and the V-cycle on a single-node impulse at a corner of the extended
grid (every level's zero padding on two sides at once)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from _gpu_common import handle, oracle_parts, problem, rel_l2, say, to_dev, to_host
from oracle import helmholtz

pytestmark = pytest.mark.gpu


def _small():
    p = problem(2, 32, 6, (2, 8, 16))
    op, W, M = oracle_parts(p)
    f = synth.point_source(32, 6, (0.5, 0.25), 2)
    return p, op, M, f


@pytest.mark.parametrize("method", ["solve", "stationary"])
def test_zero_rhs_gives_zero_at_once(method):
    """f = 0: status OK after zero iterations and u = 0, whatever u held."""
    say(f"[edge-zero-rhs] {method}")
    p, op, M, f = _small()
    H = handle(p)
    u = to_dev(synth.random_rhs(f.shape, 5))
    info = getattr(H, method)(to_dev(np.zeros_like(f)), u, tol=1e-6, maxit=50)
    H.close()
    assert info["status"] == 0 and info["converged"] and info["iters"] == 0
    assert np.all(to_host(u) == 0)


@pytest.mark.parametrize("method", ["solve", "stationary"])
def test_maxit_zero_reports_the_initial_residual(method):
    """maxit = 0: NOT_CONVERGED, no iteration, u untouched, and the reported
    true residual is the oracle's |f - A u0| / |f| for the initial guess."""
    say(f"[edge-maxit0] {method}")
    p, op, M, f = _small()
    H = handle(p)
    u0 = 1e-3 * synth.random_rhs(f.shape, 6)
    u = to_dev(u0)
    info = getattr(H, method)(to_dev(f), u, tol=1e-6, maxit=0)
    H.close()
    assert info["status"] == 1 and not info["converged"] and info["iters"] == 0
    assert np.array_equal(to_host(u), u0)
    true = np.linalg.norm(f - helmholtz.apply(op, u0)) / np.linalg.norm(f)
    assert abs(info["relres_true"] - true) <= 1e-12 * true


def test_exact_initial_guess_needs_no_iteration():
    """u0 = the sparse direct solution: converged after zero iterations with
    u unchanged."""
    say("[edge-exact-u0]")
    p, op, M, f = _small()
    A = helmholtz.assemble(op).tocsc()
    u0 = spla.spsolve(A, f.ravel()).reshape(f.shape)
    H = handle(p)
    u = to_dev(u0)
    info = H.solve(to_dev(f), u, tol=1e-6, maxit=50)
    H.close()
    say(f"  relres_true {info['relres_true']:.3e}")
    assert info["converged"] and info["iters"] == 0
    assert info["relres_true"] < 1e-10
    assert np.array_equal(to_host(u), u0)


def test_nonfinite_rhs_is_an_error():
    from paper_2606_30495_amd._lib import McmgError
    say("[edge-nan]")
    p, op, M, f = _small()
    bad = f.copy()
    bad[10, 10] = np.nan
    H = handle(p)
    u = to_dev(np.zeros_like(f))
    with pytest.raises(McmgError) as exc:
        H.solve(to_dev(bad), u, tol=1e-6, maxit=10)
    H.close()
    assert exc.value.status == -5          # MCMG_E_NONFINITE


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
@pytest.mark.parametrize("corner", [(0, 0), (-1, -1), (0, -1), (0, 0, 0), (-1, -1, -1), (-1, 0, -1)])
def test_vcycle_corner_impulse_matches_oracle(corner, precision, tol):
    """A unit impulse (real and imaginary parts) on a corner node of the
    extended grid against the FP64 oracle V-cycle: FP32 to 1e-5, BF16 to
    2e-2 relative L2 (2D: 44^2, 3D: 20^3 through the z-streaming sweep)."""
    say(f"[edge-corner] {corner} {precision}")
    if len(corner) == 2:
        p, op, M, f = _small()
    else:
        p = problem(3, 14, 3, (2, 4, 8))
        op, W, M = oracle_parts(p)
        f = np.zeros((20, 20, 20), dtype=np.complex128)
    r = np.zeros_like(f)
    r[corner] = 1.0 - 0.5j
    H = handle(p, precision)
    z = to_dev(np.zeros_like(r))
    H.apply(to_dev(r), z)
    H.close()
    err = rel_l2(to_host(z), M(r))
    say(f"  relL2 {err:.3e}")
    assert err <= tol, err


@pytest.mark.parametrize("method", ["mcmg", "cbs"])
def test_born_zero_rhs_and_maxit_zero(method):
    """The Born-series iteration: f = 0 returns u = 0 after no step; with
    maxit = 0 it reports the oracle's periodic residual |f - A_per u0| / |f|
    of the initial guess and leaves u untouched."""
    from oracle import born
    from paper_2606_30495_amd import Handle
    say(f"[edge-born] {method}")
    p = problem(2, 32, 6, (2, 8, 16))
    gm = helmholtz.default_gamma_max(p["omega"], p["c"], p["npml"], p["h"])
    H = Handle(p["c"], p["omega"], p["h"], p["npml"], p["blob"], precision="fp32", restart=4,
               sigma_max=gm, absorber="sponge")
    op = born.sponge_operator(p["c"], p["omega"], p["h"], p["npml"], gamma_max=gm)
    f = synth.point_source(32, 6, (0.5, 0.25), 2)
    u = to_dev(synth.random_rhs(f.shape, 9))
    info = H.born_solve(to_dev(np.zeros_like(f)), u, method=method, tol=1e-6, maxit=20)
    assert info["status"] == 0 and info["iters"] == 0 and np.all(to_host(u) == 0)
    u0 = 1e-3 * synth.random_rhs(f.shape, 10)
    u = to_dev(u0)
    info = H.born_solve(to_dev(f), u, method=method, tol=1e-6, maxit=0)
    H.close()
    assert info["status"] == 1 and info["iters"] == 0
    assert np.array_equal(to_host(u), u0)
    true = np.linalg.norm(f - born.apply_periodic(op, u0)) / np.linalg.norm(f)
    assert abs(info["relres_true"] - true) <= 1e-12 * true


def _zero_weight_problem():
    """bump 32^2 + 6-cell PML with every weight tensor zero: MG(r) = 0 for
    every r, so w = A MG(v_1) = 0 and the first Hessenberg column is zero."""
    p = problem(2, 32, 6, (2, 8, 16))
    L = len(p["channels"])
    tens = [dict(t, w=np.zeros_like(t["w"])) for t in p["tens"]]
    p["blob"] = synth.pack_blob(2, p["channels"], p["nu1"], p["nu2"], tens)
    f = synth.point_source(32, 6, (0.5, 0.25), 2)
    return p, f


def test_zero_preconditioner_column_leaves_u_unchanged():
    """A preconditioner that maps v_1 to zero gives a zero first column of H
    (its rotated diagonal is zero): the cycle has no usable direction, so the
    solve stops with NOT_CONVERGED after that one application, u unchanged
    and finite, and the reported residual that of the initial guess."""
    say("[edge-zero-mg]")
    p, f = _zero_weight_problem()
    op, _, _ = oracle_parts(p)
    u0 = 1e-3 * synth.random_rhs(f.shape, 14)
    H = handle(p)
    u = to_dev(u0)
    info = H.solve(to_dev(f), u, tol=1e-6, maxit=20)
    H.close()
    say(f"  status {info['status']} iters {info['iters']} relres {info['relres_true']:.3e}")
    assert info["status"] == 1 and info["iters"] == 1
    assert np.array_equal(to_host(u), u0)
    true = np.linalg.norm(f - helmholtz.apply(op, u0)) / np.linalg.norm(f)
    assert abs(info["relres_true"] - true) <= 1e-12 * true


def test_zero_preconditioner_column_in_a_batch():
    """The batched engine takes the same decision for a zero-MG problem
    while an ordinary problem in the same batch runs on and equals its
    single solve bitwise."""
    from paper_2606_30495_amd import solve_batch
    say("[edge-zero-mg-batch]")
    p0, f0 = _zero_weight_problem()
    p1 = problem(2, 32, 6, (2, 8, 16))
    f1 = synth.point_source(32, 6, (0.3, 0.6), 2)
    u0 = 1e-3 * synth.random_rhs(f0.shape, 15)
    h0, h1 = handle(p0), handle(p1)
    ua, ub = to_dev(u0), to_dev(np.zeros_like(f1))
    st, infos = solve_batch([h0, h1], [to_dev(f0), to_dev(f1)], [ua, ub], tol=1e-6, maxit=12)
    ref = to_dev(np.zeros_like(f1))
    info1 = h1.solve(to_dev(f1), ref, tol=1e-6, maxit=12)
    h0.close()
    h1.close()
    assert infos[0]["status"] == 1 and infos[0]["iters"] == 1
    assert np.array_equal(to_host(ua), u0)
    assert infos[1]["iters"] == info1["iters"] == 12
    assert np.array_equal(to_host(ub), to_host(ref))
