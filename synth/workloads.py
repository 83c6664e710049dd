"""Multi-problem workloads: the batched set of uneven 2D problems and the
serving trace (media cache + Poisson request arrivals).  Seeded draws only."""
import math

import numpy as np

from .configs import CONFIGS, Config
from .media import (gaussian_source, medium_bump, medium_ellipses, medium_grf,
                    medium_layered_sphere, omega_for_ppw, point_source)


def make_batch(cfg: Config = CONFIGS["ellipses64"]):
    """The batched workload: `count` independent 2D problems (PCG64 seed
    cfg.medium_seed).  Per problem, drawn in this order: side s uniform over
    cfg.extra['sides']; a high-contrast ellipse medium of side s (background
    2, 5-20 ellipses with speed in [1, 10]); a Gaussian source (sigma 2h,
    truncated at 4 sigma) centred on an interior node drawn uniformly from
    [0.1, 0.9]^2.  omega gives cfg.ppw points per wavelength at the
    problem's slowest speed.  Returns a list of dicts (n, c, h, omega, f)."""
    rng = np.random.Generator(np.random.PCG64(cfg.medium_seed))
    sides = cfg.extra["sides"]
    out = []
    for _ in range(cfg.extra["count"]):
        s = int(sides[int(rng.integers(0, len(sides)))])
        c = medium_ellipses(s, rng)
        h = 1.0 / s
        lo, hi = int(math.ceil(0.1 * s)), int(math.floor(0.9 * s))
        node = rng.integers(lo, hi + 1, size=2)
        pos = tuple(float(i) / s for i in node)
        out.append({"n": s, "c": c, "h": h, "omega": omega_for_ppw(c, cfg.ppw, h),
                    "f": gaussian_source(s, cfg.npml, pos, 2)})
    return out


def serve_media(seed=3, sides2d=(64, 96, 128), sides3d=(24, 32), n2d=12, n3d=4,
                npml2d=16, npml3d=12, ppw2d=10.0, ppw3d=8.0):
    """The media cache of the serving workload: n2d 2D media whose types
    cycle bump / Gaussian random field / ellipses and n3d 3D layered media
    with a spherical inclusion; sides drawn uniformly from the given sets
    (PCG64 seed).  Returns a list of dicts (dim, n, npml, c, h, omega)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    media = []
    for i in range(n2d):
        s = int(sides2d[int(rng.integers(0, len(sides2d)))])
        kind = ("bump", "grf", "ellipses")[i % 3]
        if kind == "bump":
            c = medium_bump(s, 2)
        elif kind == "grf":
            c = medium_grf(s, int(rng.integers(0, 1 << 30)), corr=0.05, cmin=1.5, cmax=4.5)
        else:
            c = medium_ellipses(s, rng)
        h = 1.0 / s
        media.append({"dim": 2, "n": s, "npml": npml2d, "c": c, "h": h, "kind": kind,
                      "omega": omega_for_ppw(c, ppw2d, h)})
    for _ in range(n3d):
        s = int(sides3d[int(rng.integers(0, len(sides3d)))])
        c = medium_layered_sphere(s, int(rng.integers(0, 1 << 30)))
        h = 1.0 / s
        media.append({"dim": 3, "n": s, "npml": npml3d, "c": c, "h": h, "kind": "layered",
                      "omega": omega_for_ppw(c, ppw3d, h)})
    return media


def serve_trace(media, nreq, rate, seed=3, p2d=0.8, nrhs_max=8):
    """Poisson arrivals at `rate` requests/s (exponential gaps, PCG64 seed):
    each request picks a 2D medium with probability p2d (uniform over the 2D
    media) else a 3D one, carries 1..nrhs_max point sources at interior
    nodes drawn uniformly from [0.1, 0.9]^D.  Returns a list of dicts
    (t arrival seconds, medium index, fs list of extended-grid sources)."""
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    idx2 = [i for i, m in enumerate(media) if m["dim"] == 2]
    idx3 = [i for i, m in enumerate(media) if m["dim"] == 3]
    t = 0.0
    out = []
    for _ in range(nreq):
        t += float(rng.exponential(1.0 / rate))
        pool = idx2 if (rng.uniform() < p2d or not idx3) else idx3
        mi = pool[int(rng.integers(0, len(pool)))]
        m = media[mi]
        k = int(rng.integers(1, nrhs_max + 1))
        fs = []
        for _ in range(k):
            lo, hi = int(math.ceil(0.1 * m["n"])), int(math.floor(0.9 * m["n"]))
            node = rng.integers(lo, hi + 1, size=m["dim"])
            fs.append(point_source(m["n"], m["npml"], tuple(float(i) / m["n"] for i in node), m["dim"]))
        out.append({"t": t, "medium": mi, "fs": fs})
    return out
