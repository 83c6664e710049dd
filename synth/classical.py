"""Hand-set classical coefficients for the McMg tensor set: a shifted-Laplacian
geometric multigrid V-cycle written in McMg's own structure.

Random-init weights make MG a structureless preconditioner (FGMRES(30) then
stalls near relative residual 1); these coefficients make the same V-cycle
(same kernels, shapes and channel counts) a classical preconditioner that
converges on small problems, so solve-to-tolerance behaviour (iteration
counts, solves/s, latency) can be measured and compared with the oracle.

Recipe (real 2-channel form of complex arithmetic; channels 0, 1 carry
(Re, Im), every other channel stays zero):
  * level operator M_l = -Lap_{h_l} - (1 + i beta) k_l^2:
      W_l = 5/7-point Laplacian / h_l^2 on channels 0 and 1,
      KA_l = centre tap [[-1, beta], [-beta, -1]], feature a_l = k_l^2;
  * smoother: weighted Jacobi e += omega_J M_diag^{-1} (r - M e), the complex
    multiplication by 1/diag done with four channels where C_l >= 4
    (KS copies (Re, Im, Im, Re), s_l = (Re, Im, Re, Im) of 1/diag, Wsm
    recombines), and on the 2-channel finest level as |1/diag| times the
    phase of 1/diag at the mean wavenumber;
  * restriction R = full weighting ([1,2,1]/4)^D, prolongation P = 2^D R^T;
  * lift / projection = identity, setup networks zero;
  * k_l^2 on a coarse level = k^2 injected at the coarse nodes 2X.
Features are returned for injection through the library's feature hook
(the setup networks cannot produce k^2 exactly).
"""
import itertools
import math

import numpy as np


def _taps(dim):
    return [tuple(d - 1 for d in t) for t in itertools.product(range(3), repeat=dim)]


def shifted_laplacian(c, omega, h, npml, channels, nu1, nu2, beta=1.0, omega_j=0.66):
    """Return (tensors, feats) for the medium c (interior speed).

    tensors: canonical list of {kind, level, step, w float32 [d0][d1][3^D]};
    feats: list over levels l = 1..L of (a, s), float32 channel-last
    [nodes...][C_l] (the library's feature layout)."""
    c = np.asarray(c, dtype=np.float64)
    dim = c.ndim
    T = 3 ** dim
    taps = _taps(dim)
    ctr = taps.index((0,) * dim)
    lap = np.zeros(T)
    for t, off in enumerate(taps):
        s = sum(abs(o) for o in off)
        if s == 0:
            lap[t] = 2 * dim
        elif s == 1:
            lap[t] = -1.0
    fw1 = np.array([0.25, 0.5, 0.25])
    fw = fw1
    for _ in range(dim - 1):
        fw = np.multiply.outer(fw, fw1)
    fw = fw.reshape(-1)
    L = len(channels)

    def z(a, b):
        return np.zeros((a, b, T))

    def eye2(C):
        w = z(C, C)
        w[0, 0, ctr] = w[1, 1, ctr] = 1.0
        return w

    k2 = (omega / np.pad(c, npml, mode="edge")) ** 2
    tens = [{"kind": "f_lift", "level": 0, "step": 0, "w": z(channels[0], 1)},
            {"kind": "g_lift", "level": 0, "step": 0, "w": eye2(2)},
            {"kind": "g_proj", "level": 0, "step": 0, "w": eye2(2)}]
    feats = []
    k2l = k2
    for l in range(1, L + 1):
        C = channels[l - 1]
        hl = h * 2 ** (l - 1)
        W = z(C, C)
        W[0, 0] = W[1, 1] = lap / hl ** 2
        KA = z(C, C)
        KA[0, 0, ctr], KA[0, 1, ctr], KA[1, 0, ctr], KA[1, 1, ctr] = -1.0, beta, -beta, -1.0
        dr = 2 * dim / hl ** 2 - k2l
        di = -beta * k2l
        mag2 = dr ** 2 + di ** 2
        ir, ii = dr / mag2, -di / mag2            # 1 / diag
        a = np.zeros(k2l.shape + (C,))
        a[..., 0] = a[..., 1] = k2l
        s = np.zeros(k2l.shape + (C,))
        KS = z(C, C)
        Wsm = z(C, C)
        if C >= 4:
            KS[0, 0, ctr] = KS[1, 1, ctr] = KS[2, 1, ctr] = KS[3, 0, ctr] = 1.0
            s[..., 0], s[..., 1], s[..., 2], s[..., 3] = ir, ii, ir, ii
            Wsm[0, 0, ctr], Wsm[0, 1, ctr] = omega_j, -omega_j
            Wsm[1, 2, ctr], Wsm[1, 3, ctr] = omega_j, omega_j
        else:
            ph = math.atan2(float(ii.mean()), float(ir.mean()))
            KS[0, 0, ctr], KS[0, 1, ctr] = math.cos(ph), -math.sin(ph)
            KS[1, 0, ctr], KS[1, 1, ctr] = math.sin(ph), math.cos(ph)
            s[..., 0] = s[..., 1] = 1.0 / np.sqrt(mag2)
            Wsm[0, 0, ctr] = Wsm[1, 1, ctr] = omega_j
        feats.append((a.astype(np.float32), s.astype(np.float32)))
        tens += [{"kind": "f_s", "level": l, "step": 0, "w": z(C, C)},
                 {"kind": "W", "level": l, "step": 0, "w": W},
                 {"kind": "KA", "level": l, "step": 0, "w": KA},
                 {"kind": "KS", "level": l, "step": 0, "w": KS}]
        ns = nu1[l - 1] + (nu2[l - 1] if l < L else 0)
        for i in range(1, ns + 1):
            tens.append({"kind": "Wsm", "level": l, "step": i, "w": Wsm})
        if l < L:
            Cn = channels[l]
            R = z(Cn, C)
            R[0, 0] = R[1, 1] = fw
            tens += [{"kind": "f_a", "level": l, "step": 0, "w": z(Cn, C)},
                     {"kind": "R", "level": l, "step": 0, "w": R},
                     {"kind": "P", "level": l, "step": 0, "w": (2 ** dim) * R}]
            k2l = k2l[(slice(None, None, 2),) * dim]
    for t in tens:
        t["w"] = t["w"].astype(np.float32)
    return tens, feats
