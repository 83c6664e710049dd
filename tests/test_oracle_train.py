"""Pins of the training oracle (L_H, its gradient, Adam, LLPF) against what
the paper and the mathematics fix (CPU only)."""
import numpy as np
import pytest
import torch

import synth
from oracle import mcmg, train


def _small(dim, n, npml, channels, absorber="pml", seed=0, nu=1):
    L = len(channels)
    nu1 = nu2 = (nu,) * L
    tens = synth.make_weights(dim, channels, nu1, nu2, seed)
    c = synth.medium_bump(n, dim)
    h = 1.0 / n
    omega = synth.omega_for_ppw(c, 10.0, h)
    smp = train.Sample(c, omega, h, npml, absorber=absorber, gamma_max=1.0 if absorber == "sponge" else None)
    return tens, nu1, nu2, smp


@pytest.mark.parametrize("dim,n,npml,channels", [(2, 13, 2, (2, 4, 6)), (3, 6, 1, (2, 3))])
def test_torch_forward_matches_numpy_oracle(dim, n, npml, channels):
    """The torch forward (Alg. 1 + Alg. 2 via library convolutions) and the
    NumPy oracle are two implementations of the same V-cycle."""
    tens, nu1, nu2, smp = _small(dim, n, npml, channels, nu=2)
    W = mcmg.Weights(dim, channels, nu1, nu2, tens)
    Mnp = mcmg.Preconditioner(W, smp.k, smp.h)
    r = train.random_residuals(smp.k.shape, 1, 3)[0]
    P = train.params_from(tens, requires_grad=False)
    a, s = train.setup(P, dim, len(channels), smp.k, smp.h)
    z = train.vcycle(P, dim, nu1, nu2, a, s, torch.tensor(r)).numpy()
    zn = Mnp(r)
    assert np.linalg.norm(z - zn) / np.linalg.norm(zn) < 1e-12
    # and apply_A equals the oracle's operator
    from oracle import helmholtz
    Az = train.apply_A(smp.op, torch.tensor(zn)).numpy()
    assert np.linalg.norm(Az - helmholtz.apply(smp.op, zn)) / np.linalg.norm(Az) < 1e-13


@pytest.mark.parametrize("absorber", ["pml", "sponge"])
def test_gradient_matches_finite_differences(absorber):
    """dL_H/dw from reverse mode against central differences along random
    directions, one tensor of every kind (setup nets, lift/projection, level
    operator, smoother, transfers)."""
    dim, channels = 2, (2, 3, 4)
    tens, nu1, nu2, smp = _small(dim, 11, 2, channels, absorber=absorber, nu=1)
    res = train.random_residuals(smp.k.shape, 2, 5)
    samples = [smp, smp]
    loss, grads = train.loss_and_grads(tens, dim, nu1, nu2, samples, res)
    rng = np.random.default_rng(7)
    kinds = {}
    for i, t in enumerate(tens):
        kinds.setdefault(t["kind"], i)
    for kind, i in kinds.items():
        d = rng.standard_normal(np.shape(tens[i]["w"]))
        eps = 1e-6

        def L_at(sign):
            tt = [dict(t) for t in tens]
            tt[i] = dict(tens[i], w=np.asarray(tens[i]["w"], dtype=np.float64) + sign * eps * d)
            P = train.params_from(tt, requires_grad=False)
            return float(train.loss_H(P, dim, nu1, nu2, samples, res))

        fd = (L_at(1) - L_at(-1)) / (2 * eps)
        an = float(np.sum(grads[i] * d))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (kind, fd, an)


def test_adam_first_two_steps_closed_form():
    """Adam with bias correction: after one step the update is
    -lr g / (|g| + eps); after two steps with gradients g1, g2 it is
    -lr mh / (sqrt(vh) + eps) with mh = (0.1 (0.9 g1 + g2)) / (1 - 0.81)
    and vh = (0.001 (0.999 g1^2 + g2^2)) / (1 - 0.998001)."""
    w0 = np.array([[[1.0, -2.0, 0.5]]])
    g1 = np.array([[[0.3, -1e-3, 2.0]]])
    g2 = np.array([[[-0.1, 4e-3, 1.0]]])
    tens = [{"kind": "W", "level": 1, "step": 0, "w": w0}]
    st = {}
    lr = 0.01
    t1 = train.adam_step(tens, [g1], st, lr)
    assert np.allclose(t1[0]["w"], w0 - lr * g1 / (np.abs(g1) + 1e-8), rtol=0, atol=1e-15)
    t2 = train.adam_step(t1, [g2], st, lr)
    mh = 0.1 * (0.9 * g1 + g2) / (1 - 0.9 ** 2)
    vh = 0.001 * (0.999 * g1 ** 2 + g2 ** 2) / (1 - 0.999 ** 2)
    assert np.allclose(t2[0]["w"], t1[0]["w"] - lr * mh / (np.sqrt(vh) + 1e-8), rtol=0, atol=1e-14)


def test_training_decreases_the_loss():
    """A few Adam steps on fresh N(0, I) residuals lower L_H (Eq. loss_fun)."""
    dim, channels = 2, (2, 4)
    tens, nu1, nu2, smp = _small(dim, 12, 2, channels, nu=1)
    st = {}
    hist = []
    for it in range(25):
        res = train.random_residuals(smp.k.shape, 2, 100 + it)
        loss, g = train.loss_and_grads(tens, dim, nu1, nu2, [smp, smp], res)
        hist.append(loss)
        tens = train.adam_step(tens, g, st, 3e-3)
    assert np.mean(hist[-5:]) < 0.9 * np.mean(hist[:5]), hist


def test_llpf_growth_trains_only_the_new_level():
    """Sec. llpf: growing (2, 4) -> (2, 4, 6) marks as trainable exactly the
    tensors of level 3, f_a/R/P of level 2 and level 2's post-smoothing
    weights; a training step leaves every other tensor unchanged."""
    dim = 2
    old = synth.make_weights(dim, (2, 4), (1, 1), (1, 1), 0)
    fresh = synth.make_weights(dim, (2, 4, 6), (1, 1, 1), (1, 1, 1), 9)
    grown, mask = train.grow(old, fresh, (1, 1))
    names = [(t["kind"], t["level"], t["step"]) for t in grown]
    expect = {("f_a", 2, 0), ("R", 2, 0), ("P", 2, 0), ("Wsm", 2, 2),
              ("f_s", 3, 0), ("W", 3, 0), ("KA", 3, 0), ("KS", 3, 0), ("Wsm", 3, 1)}
    assert {n for n, m in zip(names, mask) if m} == expect
    c = synth.medium_bump(16, 2)
    smp = train.Sample(c, synth.omega_for_ppw(c, 10.0, 1 / 16), 1 / 16, 2)
    res = train.random_residuals(smp.k.shape, 1, 4)
    _, g = train.loss_and_grads(grown, dim, (1, 1, 1), (1, 1, 1), [smp], res)
    new = train.adam_step(grown, g, {}, 1e-2, trainable=mask)
    for t0, t1, m, gi in zip(grown, new, mask, g):
        same = np.array_equal(np.asarray(t0["w"], dtype=np.float64), t1["w"])
        # frozen tensors never move; trainable ones move unless unused (with
        # nu1 = 1 at the coarsest level, W_L and KA_L never act: zero gradient)
        assert same == (not m or not np.any(gi)), (t0["kind"], t0["level"], t0["step"])
    unused = {(t["kind"], t["level"]) for t, gi in zip(grown, g) if not np.any(gi)}
    assert unused == {("W", 3), ("KA", 3)}
