"""Batched FGMRES (mcmg_solve_batch): uneven grid sizes and several RHS per
medium in one launch per operation.  Each problem's result must be the same
alone and in the mix: the batched kernels share their bodies and per-problem
fixed-order reductions with the single-problem path, so results are compared
bitwise (and iteration counts exactly)."""
import numpy as np
import pytest

import synth
from _gpu_common import say, to_dev, to_host
from test_gpu_solve import classical_problem, gpu_handle

pytestmark = pytest.mark.gpu


def _problems(precision, ortho=0):
    sides = [(48, 6), (64, 8), (40, 4)]
    probs, handles = [], []
    for n, npml in sides:
        p = classical_problem(n=n, npml=npml)
        probs.append(p)
        handles.append(gpu_handle(p, precision, ortho=ortho))
    # a second right-hand side for the 64^2 medium (same handle twice)
    rng = np.random.default_rng(9)
    f2 = synth.point_source(64, 8, tuple(rng.uniform(0.2, 0.8, 2)), 2)
    items = [(handles[0], probs[0]["f"]), (handles[1], probs[1]["f"]), (handles[2], probs[2]["f"]),
             (handles[1], f2)]
    return handles, items


@pytest.mark.parametrize("precision,ortho", [("fp32", 0), ("bf16", 0), ("fp32", 1)])
def test_batch_matches_single_solves(precision, ortho):
    """ortho = 1 forces the second Gram-Schmidt pass on every column, so the
    pass's norm reduce inside the Givens launch runs for every problem."""
    from paper_2606_30495_amd import solve_batch
    say(f"[batch] {precision} ortho {ortho}")
    handles, items = _problems(precision, ortho)
    singles = []
    for H, f in items:
        u = to_dev(np.zeros_like(f))
        info = H.solve(to_dev(f), u, tol=1e-6, maxit=500)
        singles.append((to_host(u), info))
    fs = [to_dev(f) for _, f in items]
    us = [to_dev(np.zeros_like(f)) for _, f in items]
    st, infos = solve_batch([H for H, _ in items], fs, us, tol=1e-6, maxit=500, hist_cap=600)
    assert st == 0
    for k, ((us_single, i1), ub, i2) in enumerate(zip(singles, us, infos)):
        say(f"  problem {k}: single {i1['iters']} it, batch {i2['iters']} it, relres {i2['relres_true']:.3e}")
        assert i2["converged"] and i2["relres_true"] <= 1e-6
        assert i2["iters"] == i1["iters"]
        assert np.array_equal(to_host(ub), us_single)
        assert np.array_equal(np.array(i2["hist"]), np.array(i1["hist"]))


def test_batch_zero_rhs_and_solved_guess_in_a_mix():
    """One batch holding a zero right-hand side (u set to zero at once, from
    a nonzero guess), a right-hand side whose initial guess is the sparse
    direct solution (no iteration, u untouched) and two ordinary problems:
    each result is bitwise equal to its single solve."""
    import scipy.sparse.linalg as spla
    from oracle import helmholtz
    from paper_2606_30495_amd import solve_batch
    say("[batch-edge]")
    handles, items = _problems("fp32")
    fs = [f for _, f in items]
    fs[0] = np.zeros_like(fs[0])
    p2 = classical_problem(n=40, npml=4)
    op2 = helmholtz.setup_operator(p2["c"], p2["omega"], p2["h"], p2["npml"])
    exact = spla.spsolve(helmholtz.assemble(op2).tocsc(), fs[2].ravel()).reshape(fs[2].shape)
    u0s = [synth.random_rhs(fs[0].shape, 8), np.zeros_like(fs[1]), exact, np.zeros_like(fs[3])]
    singles = []
    for (H, _), f, u0 in zip(items, fs, u0s):
        u = to_dev(u0)
        info = H.solve(to_dev(f), u, tol=1e-6, maxit=500)
        singles.append((to_host(u), info))
    us = [to_dev(u0) for u0 in u0s]
    st, infos = solve_batch([H for H, _ in items], [to_dev(f) for f in fs], us, tol=1e-6,
                            maxit=500, hist_cap=600)
    assert st == 0
    for k, ((u1, i1), ub, i2) in enumerate(zip(singles, us, infos)):
        say(f"  problem {k}: single {i1['iters']} it, batch {i2['iters']} it")
        assert i2["converged"] and i2["iters"] == i1["iters"]
        assert np.array_equal(to_host(ub), u1)
    assert infos[0]["iters"] == 0 and np.all(to_host(us[0]) == 0)
    assert infos[2]["iters"] == 0 and np.array_equal(to_host(us[2]), exact)
    assert infos[1]["iters"] > 0 and infos[3]["iters"] > 0


def test_batch_alone_equals_in_mix():
    """The same problem alone in a batch of one and inside a larger batch."""
    from paper_2606_30495_amd import solve_batch
    say("[batch-mix]")
    handles, items = _problems("bf16")
    H, f = items[1]
    u_alone = to_dev(np.zeros_like(f))
    solve_batch([H], [to_dev(f)], [u_alone], tol=1e-6, maxit=500)
    fs = [to_dev(x) for _, x in items]
    us = [to_dev(np.zeros_like(x)) for _, x in items]
    solve_batch([h for h, _ in items], fs, us, tol=1e-6, maxit=500)
    assert np.array_equal(to_host(us[1]), to_host(u_alone))


def test_batch_random_weights_partial_cycles():
    """Random-init weights (no convergence): maxit cuts every problem in the
    middle of a cycle; the partial iterates still match the single solves."""
    from paper_2606_30495_amd import Handle, solve_batch
    say("[batch-random]")
    ch, nu = (2, 8, 16), (2, 2, 2)
    blob = synth.pack_blob(2, ch, nu, nu, synth.make_weights(2, ch, nu, nu, 0))
    hs, fs = [], []
    for n in (64, 37):
        c = synth.medium_bump(n, 2)
        h = 1.0 / n
        hs.append(Handle(c, synth.omega_for_ppw(c, 10.0, h), h, 8, blob, restart=30))
        fs.append(synth.point_source(n, 8, (0.5, 0.25), 2))
    singles = []
    for H, f in zip(hs, fs):
        u = to_dev(np.zeros_like(f))
        singles.append((H.solve(to_dev(f), u, tol=1e-6, maxit=45), u))
    us = [to_dev(np.zeros_like(f)) for f in fs]
    st, infos = solve_batch(hs, [to_dev(f) for f in fs], us, tol=1e-6, maxit=45)
    assert st == 1
    for (i1, u1), u2, i2 in zip(singles, us, infos):
        assert i2["iters"] == i1["iters"] == 45 and not i2["converged"]
        assert np.array_equal(to_host(u2), to_host(u1))


def test_batch_rejects_mixed_precision():
    from paper_2606_30495_amd import McmgError, solve_batch
    p = classical_problem(n=32, npml=4)
    h1, h2 = gpu_handle(p, "fp32"), gpu_handle(p, "bf16")
    f = to_dev(p["f"])
    with pytest.raises(McmgError):
        solve_batch([h1, h2], [f, f.clone()], [f.clone() * 0, f.clone() * 0])


def test_batch_graph_replay_equals_plain_launches(monkeypatch):
    """Iterations replayed from captured graphs give the same bits as plain
    launches; the batch is run twice with unrelated eager device work between
    the calls, so later replays are checked as well as the first."""
    import torch
    from paper_2606_30495_amd import solve_batch
    say("[batch-graphs]")
    handles, items = _problems("bf16")
    hl = [H for H, _ in items]

    def run():
        fs = [to_dev(x) for _, x in items]
        us = [to_dev(np.zeros_like(x)) for _, x in items]
        st, infos = solve_batch(hl, fs, us, tol=1e-6, maxit=500)
        assert st == 0
        return [to_host(u) for u in us], [i["iters"] for i in infos]

    monkeypatch.setenv("MCMG_GRAPHS", "0")
    u_plain, it_plain = run()
    monkeypatch.setenv("MCMG_GRAPHS", "1")
    for rep in range(2):
        x = torch.randn(1 << 20, device="cuda")
        torch.cuda.synchronize()
        assert torch.isfinite((x * 2.0).sum()).item()
        u_g, it_g = run()
        say(f"  replay {rep}: iters {it_g} (plain {it_plain})")
        assert it_g == it_plain
        for a, b in zip(u_g, u_plain):
            assert np.array_equal(a, b)
