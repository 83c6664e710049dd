"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs.  Tolerances: FP64 operator 1e-13 relative; FP32
V-cycle 1e-5 relative L2 per application; FP32 setup features 1e-5."""
import numpy as np
import pytest

from _gpu_common import handle, oracle_parts, problem, rel_l2, say, to_dev, to_host
import synth
from oracle import helmholtz, krylov, mcmg

pytestmark = pytest.mark.gpu

CASES = {
    # name: (dim, n interior, npml, channels)
    "bump64": (2, 64, 8, (2, 8, 16)),
    "ragged2d": (2, 37, 5, (2, 8, 16, 32)),       # 47 -> 24 -> 12 -> 6: odd and even sides
    "small3d": (3, 14, 3, (2, 4, 8)),             # 20 -> 10 -> 5
    "ragged3d": (3, 11, 2, (2, 12, 24)),          # 15 -> 8 -> 4
    # 70^3: several z-chunks of the streaming level-1 sweep, ragged in z, y, x
    "chunked3d": (3, 64, 3, (2, 4, 8)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_matvec(name):
    dim, n, npml, ch = CASES[name]
    say(f"[matvec] {name}")
    p = problem(dim, n, npml, ch)
    op, _, _ = oracle_parts(p)
    H = handle(p)
    u = synth.random_rhs(H.ext_shape, 11)
    ud = to_dev(u)
    Au = to_dev(np.zeros_like(u))
    H.matvec(ud, Au)
    got = to_host(Au)
    ref = helmholtz.apply(op, u)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < 1e-13, err


@pytest.mark.parametrize("name", ["bump64", "ragged2d", "small3d", "chunked3d"])
def test_matvec_sponge(name):
    """Sponge absorbing layer (Sec. 2.1): FP64 matvec against the oracle."""
    from paper_2606_30495_amd import Handle
    dim, n, npml, ch = CASES[name]
    say(f"[matvec-sponge] {name}")
    p = problem(dim, n, npml, ch)
    op = helmholtz.setup_operator(p["c"], p["omega"], p["h"], npml, absorber="sponge")
    H = Handle(p["c"], p["omega"], p["h"], npml, p["blob"], absorber="sponge")
    u = synth.random_rhs(H.ext_shape, 12)
    Au = to_dev(np.zeros_like(u))
    H.matvec(to_dev(u), Au)
    ref = helmholtz.apply(op, u)
    err = np.abs(to_host(Au) - ref).max() / np.abs(ref).max()
    assert err < 1e-13, err


@pytest.mark.parametrize("dim,n", [(2, 40), (3, 16)])
def test_matvec_plane_wave_symbol(dim, n):
    """Eq. discrete_symbol on the GPU: constant medium, no layer."""
    say(f"[symbol] dim={dim}")
    from paper_2606_30495_amd import Handle
    tens = synth.make_weights(dim, (2, 4), (1, 1), (1, 1), 0)
    blob = synth.pack_blob(dim, (2, 4), (1, 1), (1, 1), tens)
    h = 1.0 / n
    k = 9.0
    H = Handle(np.ones((n,) * dim), k, h, 0, blob)
    x = np.arange(n) * h
    X = np.meshgrid(*([x] * dim), indexing="ij")
    for p in [(1,) * dim, (n // 2 - 1,) + (2,) * (dim - 1)]:
        xi = [2 * np.pi * pa for pa in p]
        u = np.exp(1j * sum(a * b for a, b in zip(xi, X)))
        Au = to_dev(np.zeros_like(u))
        H.matvec(to_dev(u), Au)
        got = to_host(Au)
        sym = 4.0 / h ** 2 * sum(np.sin(a * h / 2) ** 2 for a in xi) - k * k
        inner = tuple(slice(1, n - 1) for _ in range(dim))
        assert np.abs(got[inner] - sym * u[inner]).max() < 1e-12 * (4 * dim / h ** 2)


@pytest.mark.parametrize("name", list(CASES))
def test_setup_features(name):
    dim, n, npml, ch = CASES[name]
    say(f"[setup] {name}")
    p = problem(dim, n, npml, ch)
    op, W, M = oracle_parts(p)
    H = handle(p)
    import torch
    for l in range(1, len(ch) + 1):
        shape, C = H.level_shape(l)
        assert C == ch[l - 1]
        a = torch.zeros(shape + (C,), dtype=torch.float32, device="cuda")
        s = torch.zeros_like(a)
        H.get_features(l, a, s)
        ra = np.moveaxis(M.feats["a"][l], 0, -1)
        rs = np.moveaxis(M.feats["s"][l], 0, -1)
        assert ra.shape == tuple(a.shape)
        assert rel_l2(to_host(a), ra) < 1e-5
        assert rel_l2(to_host(s), rs) < 1e-5


@pytest.mark.parametrize("name", list(CASES))
def test_apply_matches_oracle(name):
    dim, n, npml, ch = CASES[name]
    say(f"[apply] {name}")
    p = problem(dim, n, npml, ch)
    op, W, M = oracle_parts(p)
    H = handle(p)
    r = synth.random_rhs(H.ext_shape, 3)
    z = to_dev(np.zeros_like(r))
    H.apply(to_dev(r), z)
    got = to_host(z)
    ref = M(r)
    err = rel_l2(got, ref)
    say(f"  relL2 = {err:.3e}")
    assert err <= 1e-5, err


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("name,tile", [("ragged2d", "1,1,2"), ("ragged2d", "2,2,2"),
                                       ("bump64", "4,1,2"), ("ragged3d", "1,1,2"),
                                       ("ragged3d", "2,1,4"), ("chunked3d", "1,1,4"),
                                       ("chunked3d", "4,2,2")])
def test_apply_every_tile_shape(name, tile, precision, monkeypatch):
    """Each matrix-core tile shape (16*mt nodes per wave row, ntw column
    tiles, rpw rows per wave), forced where it fits, against the oracle."""
    monkeypatch.setenv("MCMG_FORCE_TILE", tile)
    dim, n, npml, ch = CASES[name]
    say(f"[tile] {name} {tile} {precision}")
    p = problem(dim, n, npml, ch)
    _, _, M = oracle_parts(p)
    H = handle(p, precision)
    r = synth.random_rhs(H.ext_shape, 5)
    z = to_dev(np.zeros_like(r))
    H.apply(to_dev(r), z)
    err = rel_l2(to_host(z), M(r))
    say(f"  rel L2 {err:.3e}")
    assert err <= (1e-5 if precision == "fp32" else 2e-2), err


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("name", ["bump64", "ragged2d"])
def test_fused_step_bitwise_equals_three_launches(name, precision, monkeypatch):
    """The fused matrix-core smoothing step rounds t and u where the three
    separate convolutions do and sums K in the same order: same bits."""
    dim, n, npml, ch = CASES[name]
    say(f"[fused-step] {name} {precision}")
    p = problem(dim, n, npml, ch)
    r = synth.random_rhs((n + 2 * npml,) * dim, 9)
    out = []
    for fused in ("2", "0"):        # 2: fuse every C >= 8 level in both precisions
        monkeypatch.setenv("MCMG_FUSED_STEP", fused)
        H = handle(p, precision)
        z = to_dev(np.zeros_like(r))
        H.apply(to_dev(r), z)
        out.append(to_host(z))
        H.close()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("name", list(CASES))
def test_apply_bf16_within_budget(name):
    """bf16 matrix-core operands with float32 accumulation and float32 state:
    per-application error against the FP64 oracle within 2e-2."""
    dim, n, npml, ch = CASES[name]
    say(f"[apply-bf16] {name}")
    p = problem(dim, n, npml, ch)
    op, W, M = oracle_parts(p)
    H = handle(p, precision="bf16")
    r = synth.random_rhs(H.ext_shape, 3)
    z = to_dev(np.zeros_like(r))
    H.apply(to_dev(r), z)
    err = rel_l2(to_host(z), M(r))
    say(f"  relL2 = {err:.3e}")
    assert err <= 2e-2, err
    assert err > 1e-6      # the bf16 path really rounds


def test_apply_linear_and_deterministic():
    """Linearity in r over the reals (Sec. 3.2) survives FP32 to rounding
    level; two runs give bitwise identical output."""
    say("[linear]")
    p = problem(2, 64, 8, (2, 8, 16))
    H = handle(p)
    r1 = synth.random_rhs(H.ext_shape, 1)
    r2 = synth.random_rhs(H.ext_shape, 2)
    outs = []
    for r in (r1, r2, 0.7 * r1 - 1.9 * r2, r1):
        z = to_dev(np.zeros_like(r))
        H.apply(to_dev(r), z)
        outs.append(to_host(z))
    assert rel_l2(outs[2], 0.7 * outs[0] - 1.9 * outs[1]) < 1e-5
    assert np.array_equal(outs[0], outs[3])
    z0 = to_dev(np.zeros_like(r1))
    H.apply(to_dev(np.zeros_like(r1)), z0)
    assert np.all(to_host(z0) == 0)


def test_fgmres_history_matches_oracle():
    """Random-init weights (bump64): the GPU FGMRES residual history follows
    the oracle's for 60 iterations (two restart cycles)."""
    say("[fgmres-hist]")
    p = problem(2, 64, 8, (2, 8, 16))
    op, W, M = oracle_parts(p)
    H = handle(p, restart=30)
    f = synth.point_source(64, 8, (0.5, 0.25), 2)
    u = to_dev(np.zeros_like(f))
    info = H.solve(to_dev(f), u, tol=1e-6, maxit=60)
    uo, io = krylov.fgmres(lambda x: helmholtz.apply(op, x), M, f, m=30, tol=1e-6, maxit=60)
    say(f"  gpu iters {info['iters']} rel {info['relres_true']:.6e}; oracle {io['iters']} {io['relres_true']:.6e}")
    assert info["iters"] == io["iters"] == 60
    hg, ho = np.array(info["hist"]), np.array(io["hist"])
    assert len(hg) == len(ho)
    assert np.max(np.abs(hg - ho) / ho) < 1e-5
    assert abs(info["relres_true"] - io["relres_true"]) / io["relres_true"] < 1e-5
    assert rel_l2(to_host(u), uo) < 1e-3


def test_fgmres_longest_restart_history_matches_oracle():
    """Restart length 64, the longest the library takes (random-init weights,
    bump64): 66 iterations run a whole cycle, whose last Givens step works on
    column 63 and whose back substitution solves a 64 x 64 system, then two
    iterations of the next cycle.  The residual history and the iterate
    follow the oracle's FGMRES(64)."""
    say("[fgmres-m64]")
    p = problem(2, 64, 8, (2, 8, 16))
    op, W, M = oracle_parts(p)
    H = handle(p, restart=64)
    f = synth.point_source(64, 8, (0.5, 0.25), 2)
    u = to_dev(np.zeros_like(f))
    info = H.solve(to_dev(f), u, tol=1e-6, maxit=66)
    uo, io = krylov.fgmres(lambda x: helmholtz.apply(op, x), M, f, m=64, tol=1e-6, maxit=66)
    say(f"  gpu iters {info['iters']} rel {info['relres_true']:.6e}; oracle {io['iters']} {io['relres_true']:.6e}")
    assert info["iters"] == io["iters"] == 66
    hg, ho = np.array(info["hist"]), np.array(io["hist"])
    assert len(hg) == len(ho)
    assert np.max(np.abs(hg - ho) / ho) < 1e-5
    assert abs(info["relres_true"] - io["relres_true"]) / io["relres_true"] < 1e-5
    assert rel_l2(to_host(u), uo) < 1e-3


def test_fgmres_small_pml_vs_oracle():
    """16x16 + 4-cell PML with restart 64, 128 iterations: the residual
    history follows the oracle's FGMRES(64) and the two iterates agree."""
    say("[fgmres-16]")
    p = problem(2, 16, 4, (2, 4, 8), ppw=6.0)
    op, W, M = oracle_parts(p)
    H = handle(p, restart=64)
    f = synth.point_source(16, 4, (0.5, 0.25), 2)
    u = to_dev(np.zeros_like(f))
    info = H.solve(to_dev(f), u, tol=1e-10, maxit=128)
    uo, io = krylov.fgmres(lambda x: helmholtz.apply(op, x), M, f, m=64, tol=1e-10, maxit=128)
    say(f"  gpu {info['relres_true']:.3e} oracle {io['relres_true']:.3e}")
    assert info["iters"] == io["iters"] == 128
    hg, ho = np.array(info["hist"]), np.array(io["hist"])
    assert np.max(np.abs(hg - ho) / ho) < 1e-4
    assert abs(info["relres_true"] - io["relres_true"]) / io["relres_true"] < 1e-4
    assert rel_l2(to_host(u), uo) < 1e-3


def test_fgmres_full_krylov_space_matches_dense_lu():
    """O8(i) through the C ABI: 16x16 + 4-cell PML (576 unknowns), random-init
    McMg preconditioner (FP32 V-cycle), no restart (m = 600 >= 576),
    tol 1e-12.  FGMRES converges within its one cycle (in exact arithmetic
    by the dimension of the space, 576; FP64 loss of orthogonality adds a
    few steps), and its FP64 solution equals LAPACK's dense solve of the
    assembled A to 1e-10, as the oracle's does."""
    say("[fgmres-lu]")
    p = problem(2, 16, 4, (2, 4, 8), ppw=6.0)
    op, W, M = oracle_parts(p)
    f = synth.point_source(16, 4, (0.5, 0.25), 2)
    A = helmholtz.assemble(op).toarray()
    u_lu = np.linalg.solve(A, f.reshape(-1)).reshape(f.shape)
    H = handle(p, restart=600)
    u = to_dev(np.zeros_like(f))
    info = H.solve(to_dev(f), u, tol=1e-12, maxit=600)
    H.close()
    err = rel_l2(to_host(u), u_lu)
    say(f"  iters {info['iters']} relres {info['relres_true']:.3e} |u - u_LU|/|u_LU| {err:.3e}")
    assert info["converged"] and info["iters"] < 600
    assert err <= 1e-10, err


def test_stationary_matches_oracle():
    say("[stationary]")
    p = problem(2, 64, 8, (2, 8, 16))
    op, W, M = oracle_parts(p)
    H = handle(p)
    f = synth.point_source(64, 8, (0.5, 0.25), 2)
    u = to_dev(np.zeros_like(f))
    info = H.stationary(to_dev(f), u, tol=1e-6, maxit=3)
    uo, io = krylov.stationary(lambda x: helmholtz.apply(op, x), M, f, tol=1e-6, maxit=3)
    assert info["iters"] == io["iters"] == 3
    assert np.max(np.abs(np.array(info["hist"]) - np.array(io["hist"])) / np.array(io["hist"])) < 1e-4
    # the iterate after three V-cycle updates: FP32 MG error per application
    # is below 1e-5 relative, so three summed corrections stay near it
    assert rel_l2(to_host(u), uo) < 1e-4
