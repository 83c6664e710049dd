"""Training McMg with the residual loss L_H, plus LLPF level growth (oracle,
test infrastructure).

Follows:
  * the training section: random residuals r ~ N(0, I) and the batch loss
    L_H = (1/B) sum_i |A_i MG(k_i, r_i) - r_i| / |r_i|  (Eq. loss_fun);
  * the optimiser the experiments name (Adam);
  * Sec. llpf: append a coarser level, freeze the levels trained before,
    and optimise only the parameters of the new level.

The forward here is a second, independent implementation of Alg. 1 and
Alg. 2.  It uses torch's float64 convolutions (conv{2,3}d with padding 1,
stride 2 for the restriction, conv_transpose{2,3}d for the prolongation)
instead of the NumPy loops of oracle.mcmg.  Torch's reverse-mode
differentiation then supplies dL_H/dw for every weight tensor: the library
primitive stands in for the chain rule.  A central finite-difference pin
checks the resulting gradient.

Readings where the paper is silent:
  * r ~ N(0, I) on the extended grid: real and imaginary parts are i.i.d.
    standard normal at every node;
  * Adam uses the constants of Kingma and Ba (beta1 = 0.9, beta2 = 0.999,
    eps = 1e-8) with bias correction, and one learning rate for every
    tensor;
  * LLPF trains the tensors that appending level L+1 creates, and freezes
    every other tensor.  The created tensors are:
      - every tensor of level L+1;
      - the transfer tensors f_a^L, R_L and P_L;
      - the post-smoothing weights Wsm_L^(nu1+i) of the old coarsest level,
        which had no up-cycle steps before the growth.
    The new tensors start from the seeded random initialisation of the
    grown configuration.

Parity pins (tests/test_oracle_train.py):
  * the torch forward against oracle.mcmg;
  * the gradient against central finite differences;
  * the first two Adam steps in closed form;
  * a decreasing loss;
  * the LLPF trainable set and frozen tensors left unchanged.
"""
import numpy as np
import torch
import torch.nn.functional as F

from . import helmholtz

B1, B2, EPS = 0.9, 0.999, 1e-8


def _key(t):
    return (t["kind"], int(t["level"]), int(t["step"]))


def params_from(tensors, requires_grad=True):
    """{(kind, level, step): float64 torch tensor [d0][d1][3^D]}."""
    return {_key(t): torch.tensor(np.asarray(t["w"], dtype=np.float64), requires_grad=requires_grad)
            for t in tensors}


def _k(w, dim):
    return w.reshape(w.shape[0], w.shape[1], *([3] * dim))


def _conv(x, w, dim):
    f = F.conv2d if dim == 2 else F.conv3d
    return f(x[None], _k(w, dim), padding=1)[0]


def _conv_s2(x, w, dim):
    f = F.conv2d if dim == 2 else F.conv3d
    return f(x[None], _k(w, dim), stride=2, padding=1)[0]


def _conv_t2(x, w, dim, fine):
    f = F.conv_transpose2d if dim == 2 else F.conv_transpose3d
    op = tuple(n - (2 * m - 1) for n, m in zip(fine, x.shape[1:]))
    return f(x[None], _k(w, dim), stride=2, padding=1, output_padding=op)[0]


def _gelu(x):
    return F.gelu(x)   # exact erf form


def setup(P, dim, L, k, h):
    """Alg. 1 with float64 torch tensors: features a_l, s_l (channel-first)."""
    m = torch.tensor(np.asarray(k, dtype=np.float64) * h)[None]
    a, s = [None] * (L + 1), [None] * (L + 1)
    a[1] = _gelu(_conv(m, P[("f_lift", 0, 0)], dim))
    for l in range(1, L + 1):
        s[l] = _gelu(_conv(a[l], P[("f_s", l, 0)], dim))
        if l < L:
            a[l + 1] = _gelu(_conv_s2(a[l], P[("f_a", l, 0)], dim))
    return a, s


def vcycle(P, dim, nu1, nu2, a, s, r):
    """Alg. 2 on a complex residual r (torch complex128); returns complex MG(r)."""
    L = len(nu1)

    def A(l, e):
        return _conv(e, P[("W", l, 0)], dim) + a[l] * _conv(e, P[("KA", l, 0)], dim)

    def S(l, i, x):
        return _conv(s[l] * _conv(x, P[("KS", l, 0)], dim), P[("Wsm", l, i)], dim)

    rl, el = [None] * (L + 1), [None] * (L + 1)
    rl[1] = _conv(torch.stack([r.real, r.imag]), P[("g_lift", 0, 0)], dim)
    for l in range(1, L + 1):
        e = torch.zeros_like(rl[l])
        for i in range(1, nu1[l - 1] + 1):
            e = e + S(l, i, rl[l] - A(l, e))
        el[l] = e
        if l < L:
            rl[l + 1] = _conv_s2(rl[l] - A(l, e), P[("R", l, 0)], dim)
    for l in range(L - 1, 0, -1):
        e = el[l] + _conv_t2(el[l + 1], P[("P", l, 0)], dim, el[l].shape[1:])
        for i in range(1, nu2[l - 1] + 1):
            e = e + S(l, nu1[l - 1] + i, rl[l] - A(l, e))
        el[l] = e
    out = _conv(el[1], P[("g_proj", 0, 0)], dim)
    return torch.complex(out[0], out[1])


def apply_A(op, u):
    """The Helmholtz operator of oracle.helmholtz on a torch complex field."""
    D = u.dim()
    h2 = op["h"] ** 2
    gamma = np.broadcast_to(np.asarray(op.get("gamma", 0.0), dtype=np.float64), op["k2"].shape)
    k2 = torch.tensor(op["k2"]) * (1.0 + 1j * torch.tensor(np.ascontiguousarray(gamma)))
    out = -k2 * u
    for a_ in range(D):
        s_node, s_half = op["stretch"][a_]
        shp = [1] * D
        shp[a_] = -1
        sn = torch.tensor(s_node).reshape(shp)
        sl = torch.tensor(s_half[:-1]).reshape(shp)
        sr = torch.tensor(s_half[1:]).reshape(shp)
        pad = [0, 0] * D
        pad[2 * (D - 1 - a_)] = 1
        pad[2 * (D - 1 - a_) + 1] = 1
        up = F.pad(u[None], pad)[0]
        idx_p = [slice(None)] * D
        idx_m = [slice(None)] * D
        idx_p[a_] = slice(2, None)
        idx_m[a_] = slice(0, -2)
        flux = (up[tuple(idx_p)] - u) / sr - (u - up[tuple(idx_m)]) / sl
        out = out - flux / (h2 * sn)
    return out


class Sample:
    """One training medium: its operator and the oracle's grid data."""

    def __init__(self, c, omega, h, npml, absorber="pml", gamma_max=None):
        self.op = helmholtz.setup_operator(c, omega, h, npml, absorber=absorber, gamma_max=gamma_max)
        self.k = np.sqrt(self.op["k2"])
        self.h = h


def loss_H(P, dim, nu1, nu2, samples, residuals):
    """Eq. loss_fun over a batch: samples[i] with residual residuals[i]."""
    L = len(nu1)
    tot = 0.0
    for smp, r in zip(samples, residuals):
        a, s = setup(P, dim, L, smp.k, smp.h)
        rt = torch.tensor(np.asarray(r, dtype=np.complex128))
        z = vcycle(P, dim, nu1, nu2, a, s, rt)
        w = apply_A(smp.op, z) - rt
        tot = tot + torch.linalg.vector_norm(w) / torch.linalg.vector_norm(rt)
    return tot / len(samples)


def loss_and_grads(tensors, dim, nu1, nu2, samples, residuals):
    """L_H and dL_H/dw for every tensor (NumPy float64, canonical order)."""
    P = params_from(tensors)
    loss = loss_H(P, dim, nu1, nu2, samples, residuals)
    loss.backward()
    return float(loss.detach()), [P[_key(t)].grad.numpy().copy() for t in tensors]


def adam_step(tensors, grads, state, lr, trainable=None):
    """One Adam update in place on float64 copies of the tensors.

    state: {"t": step count, "m": [...], "v": [...]} (created on first call)."""
    if "m" not in state:
        state["t"] = 0
        state["m"] = [np.zeros_like(np.asarray(t["w"], dtype=np.float64)) for t in tensors]
        state["v"] = [np.zeros_like(np.asarray(t["w"], dtype=np.float64)) for t in tensors]
    state["t"] += 1
    t = state["t"]
    out = []
    for i, (tt, g) in enumerate(zip(tensors, grads)):
        w = np.asarray(tt["w"], dtype=np.float64).copy()
        if trainable is None or trainable[i]:
            state["m"][i] = B1 * state["m"][i] + (1 - B1) * g
            state["v"][i] = B2 * state["v"][i] + (1 - B2) * g * g
            mh = state["m"][i] / (1 - B1 ** t)
            vh = state["v"][i] / (1 - B2 ** t)
            w = w - lr * mh / (np.sqrt(vh) + EPS)
        out.append(dict(tt, w=w))
    return out


def random_residuals(shape, n, seed):
    """r ~ N(0, I): i.i.d. standard normal real and imaginary parts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.standard_normal(shape) + 1j * rng.standard_normal(shape) for _ in range(n)]


def grow(old, new_fresh, nu1_old):
    """LLPF architecture growth: the grown configuration's seeded init
    (`new_fresh`, canonical order) with every tensor the old model has copied
    over.  Returns (tensors, trainable mask)."""
    have = {_key(t): t for t in old}
    L_new = max(int(t["level"]) for t in new_fresh)
    out, mask = [], []
    for t in new_fresh:
        k = _key(t)
        if k in have:
            out.append(dict(t, w=np.asarray(have[k]["w"]).copy()))
            mask.append(False)
        else:
            out.append(dict(t))
            mask.append(True)
    # the tensors the old model lacks are exactly the LLPF trainable set
    if not (sum(mask) > 0 and L_new == len(nu1_old) + 1):
        raise ValueError("the grown configuration must add exactly one level")
    return out, mask
