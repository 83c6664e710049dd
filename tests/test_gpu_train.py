"""GPU training (L_H, its gradient, Adam, LLPF, commit) against the float64
training oracle."""
import numpy as np
import pytest

import synth
from oracle import helmholtz, krylov, mcmg
from tests._gpu_common import rel_l2, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _model(dim, channels, nu, seed=0):
    L = len(channels)
    nu1 = nu2 = (nu,) * L
    tens = synth.make_weights(dim, channels, nu1, nu2, seed)
    return tens, nu1, nu2, synth.pack_blob(dim, channels, nu1, nu2, tens)


def _medium(n, dim, seed):
    c = synth.medium_bump(n, dim)
    if seed:
        c = c * np.random.default_rng(seed).uniform(0.9, 1.1, size=c.shape)
    return c


def _handles(media, npml, blob, absorber, precision="fp32", gamma_max=1.0):
    from paper_2606_30495_amd import Handle
    out = []
    for c in media:
        h = 1.0 / c.shape[0]
        om = synth.omega_for_ppw(c, 10.0, h)
        out.append(Handle(c, om, h, npml, blob, precision=precision, restart=30,
                          sigma_max=gamma_max if absorber == "sponge" else 0.0, absorber=absorber))
    return out


def _samples(media, npml, absorber, gamma_max=1.0):
    from oracle import train
    out = []
    for c in media:
        h = 1.0 / c.shape[0]
        om = synth.omega_for_ppw(c, 10.0, h)
        out.append(train.Sample(c, om, h, npml, absorber=absorber,
                                gamma_max=gamma_max if absorber == "sponge" else None))
    return out


CASES = {
    # name: (dim, interior side, npml, channels, nu, absorber)
    "2d-pml": (2, 24, 4, (2, 4, 8), 2, "pml"),
    "2d-sponge": (2, 21, 4, (2, 8, 16), 1, "sponge"),
    "3d-pml": (3, 8, 2, (2, 3, 4), 1, "pml"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_loss_and_gradient_match_oracle(name):
    """L_H over a batch of two media and its gradient for every tensor, GPU
    float32 against the float64 reverse-mode oracle."""
    from oracle import train
    from paper_2606_30495_amd import train_loss_grad
    dim, n, npml, ch, nu, ab = CASES[name]
    say(f"[train-grad] {name}")
    tens, nu1, nu2, blob = _model(dim, ch, nu)
    media = [_medium(n, dim, 0), _medium(n, dim, 7)]
    H = _handles(media, npml, blob, ab)
    res = [train.random_residuals(H[0].ext_shape, 1, 20 + i)[0] for i in range(2)]
    loss, g = train_loss_grad(H, [to_dev(r) for r in res])
    lo, go = train.loss_and_grads(tens, dim, nu1, nu2, _samples(media, npml, ab), res)
    say(f"  loss gpu {loss:.8f} oracle {lo:.8f}")
    assert abs(loss - lo) <= 1e-5 * lo
    off = 0
    worst = 0.0
    for t, gt in zip(tens, go):
        k = gt.size
        gg = g[off:off + k].reshape(gt.shape)
        off += k
        if not np.any(gt):
            assert not np.any(gg), (t["kind"], t["level"], t["step"])
            continue
        e = rel_l2(gg, gt)
        worst = max(worst, e)
        assert e < 2e-3, (t["kind"], t["level"], t["step"], e)
    assert off == g.size
    say(f"  worst tensor gradient rel err {worst:.2e}")


def test_adam_step_matches_oracle():
    """One mcmg_train_step: the update equals the oracle's Adam step on the
    oracle gradient (entries whose gradient is not at round-off level)."""
    from oracle import train
    from paper_2606_30495_amd import train_step
    dim, n, npml, ch, nu, ab = CASES["2d-pml"]
    say("[train-adam]")
    tens, nu1, nu2, blob = _model(dim, ch, nu)
    media = [_medium(n, dim, 3)]
    H = _handles(media, npml, blob, ab)
    res = train.random_residuals(H[0].ext_shape, 1, 5)
    w0 = H[0].get_weights()
    lr = 1e-3
    loss = train_step(H, [to_dev(r) for r in res], lr=lr)
    w1 = H[0].get_weights()
    lo, go = train.loss_and_grads(tens, dim, nu1, nu2, _samples(media, npml, ab), res)
    new = train.adam_step(tens, go, {}, lr)
    d_gpu = (w1 - w0).astype(np.float64)
    d_or = np.concatenate([(t1["w"] - np.asarray(t0["w"], dtype=np.float64)).ravel() for t0, t1 in zip(tens, new)])
    gflat = np.concatenate([gt.ravel() for gt in go])
    big = np.abs(gflat) > 1e-3 * np.abs(gflat).max()
    say(f"  loss {loss:.6f} oracle {lo:.6f}; compared {big.sum()} of {big.size} entries")
    assert abs(loss - lo) <= 1e-5 * lo
    assert np.max(np.abs(d_gpu[big] - d_or[big])) <= 1e-2 * lr
    assert np.all(d_gpu[gflat == 0] == 0)


def test_commit_gives_fast_path_parity_with_trained_weights():
    """After a few steps and mcmg_train_commit, the fast V-cycle (matrix-core
    and fused level-1 kernels) applies the trained weights: it matches the
    oracle V-cycle built from the exported blob."""
    from oracle import train
    from paper_2606_30495_amd import train_step
    dim, n, npml, ch, nu, ab = CASES["2d-pml"]
    say("[train-commit]")
    _, nu1, nu2, blob = _model(dim, ch, nu)
    media = [_medium(n, dim, 0)]
    H = _handles(media, npml, blob, ab)
    for it in range(5):
        res = train.random_residuals(H[0].ext_shape, 1, 40 + it)
        train_step(H, [to_dev(r) for r in res], lr=3e-3)
    H[0].commit()
    from paper_2606_30495_amd.weights import parse_blob
    _, trained = parse_blob(H[0].export_blob())
    smp = _samples(media, npml, ab)[0]
    W = mcmg.Weights(dim, ch, nu1, nu2, trained)
    M = mcmg.Preconditioner(W, smp.k, smp.h)
    r = train.random_residuals(H[0].ext_shape, 1, 99)[0]
    z = to_dev(np.zeros_like(r))
    H[0].apply(to_dev(r), z)
    e = rel_l2(to_host(z), M(r))
    say(f"  apply after commit rel err {e:.2e}")
    assert e < 1e-5


def test_llpf_growth_freezes_old_levels():
    """Sec. llpf: grow a trained 2-level model to 3 levels, freeze the old
    tensors, train: only the new level's tensors (and the new post-smoothing
    weights of level 2) change."""
    from oracle import train
    from paper_2606_30495_amd import Handle, train_step
    from paper_2606_30495_amd.weights import grow, parse_blob
    say("[train-llpf]")
    dim = 2
    _, _, _, blob2 = _model(dim, (2, 6), 1)
    _, _, _, fresh3 = _model(dim, (2, 6, 12), 1, seed=11)
    grown, mask = grow(blob2, fresh3)
    c = _medium(32, dim, 0)
    h = 1.0 / 32
    H = Handle(c, synth.omega_for_ppw(c, 10.0, h), h, 4, grown)
    H.set_trainable(mask)
    _, before = parse_blob(H.export_blob())
    for it in range(3):
        res = train.random_residuals(H.ext_shape, 1, 60 + it)
        train_step([H], [to_dev(r) for r in res], lr=1e-2)
    _, after = parse_blob(H.export_blob())
    moved = [not np.array_equal(a["w"], b["w"]) for a, b in zip(before, after)]
    for t, m, mv in zip(before, mask, moved):
        if not m:
            assert not mv, (t["kind"], t["level"], t["step"])
    names = {(t["kind"], t["level"], t["step"]) for t, mv in zip(before, moved) if mv}
    say(f"  trained tensors {sorted(names)}")
    assert {("f_a", 2, 0), ("R", 2, 0), ("P", 2, 0), ("Wsm", 2, 2), ("f_s", 3, 0),
            ("KS", 3, 0), ("Wsm", 3, 1)} <= names
    assert names <= {(t["kind"], t["level"], t["step"]) for t, m in zip(before, mask) if m}


def test_training_lowers_fgmres_iterations():
    """Training on N(0, I) residuals (Eq. loss_fun) on two media makes the
    learned preconditioner effective on a third medium of the same family:
    with the random initialisation FGMRES(30) does not reach 1e-6 in 1000
    iterations, after 2000 Adam steps it does, in well under that."""
    from oracle import train
    from paper_2606_30495_amd import Handle, train_step
    say("[train-iters]")
    dim, n, npml, ch = 2, 32, 6, (2, 8, 16)
    _, nu1, nu2, blob = _model(dim, ch, 2)
    H = _handles([_medium(n, dim, 1), _medium(n, dim, 2)], npml, blob, "sponge", gamma_max=2.0)
    h = 1.0 / n
    c3 = _medium(n, dim, 99)
    f = synth.point_source(n, npml, (0.5, 0.25), dim)

    def iters(b):
        T = Handle(c3, synth.omega_for_ppw(c3, 10.0, h), h, npml, b, sigma_max=2.0, absorber="sponge")
        u = to_dev(np.zeros_like(f))
        info = T.solve(to_dev(f), u, tol=1e-6, maxit=1000)
        T.close()
        return info["iters"], info["converged"]

    it0, ok0 = iters(blob)
    losses, k = [], 0
    for lr, steps in ((3e-2, 300), (1e-2, 700), (3e-3, 1000)):
        for _ in range(steps):
            res = [train.random_residuals(H[0].ext_shape, 1, 10000 + 2 * k + j)[0] for j in range(2)]
            losses.append(train_step(H, [to_dev(r) for r in res], lr=lr))
            k += 1
    it1, ok1 = iters(H[0].export_blob())
    say(f"  loss {np.mean(losses[:20]):.4f} -> {np.mean(losses[-20:]):.4f}; "
        f"FGMRES iterations {it0} ({ok0}) -> {it1} ({ok1})")
    assert np.mean(losses[-20:]) < 0.5
    assert not ok0 and ok1 and it1 < 600
