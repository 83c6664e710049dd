"""Helpers shared by the GPU parity tests: seeded problems, handles, and the
oracle on the same inputs."""
import sys

import numpy as np

import synth
from oracle import helmholtz, krylov, mcmg


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def problem(dim, n, npml, channels, nu=2, ppw=10.0, seed=0, medium="bump"):
    L = len(channels)
    nu1 = nu2 = (nu,) * L
    tens = synth.make_weights(dim, channels, nu1, nu2, seed)
    blob = synth.pack_blob(dim, channels, nu1, nu2, tens)
    if medium == "bump":
        c = synth.medium_bump(n, dim)
    elif medium == "grf":
        c = synth.medium_grf(n, 1)
    elif medium == "layered":
        c = synth.medium_layered_sphere(n, 4)
    else:
        raise ValueError(medium)
    h = 1.0 / n
    omega = synth.omega_for_ppw(c, ppw, h)
    return {"dim": dim, "n": n, "npml": npml, "channels": channels, "nu1": nu1, "nu2": nu2,
            "tens": tens, "blob": blob, "c": c, "h": h, "omega": omega}


def oracle_parts(p):
    op = helmholtz.setup_operator(p["c"], p["omega"], p["h"], p["npml"])
    W = mcmg.Weights(p["dim"], p["channels"], p["nu1"], p["nu2"], p["tens"])
    M = mcmg.Preconditioner(W, np.sqrt(op["k2"]), p["h"])
    return op, W, M


def handle(p, precision="fp32", restart=30, ortho=0):
    from paper_2606_30495_amd import Handle
    return Handle(p["c"], p["omega"], p["h"], p["npml"], p["blob"], precision=precision,
                  restart=restart, ortho=ortho)


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
