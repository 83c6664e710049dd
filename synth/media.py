"""Seeded synthetic media and right-hand sides.

Node i of an interior axis of n nodes sits at x = i*h with h = 1/n (unit
box).  Arrays are row-major with axis 0 slowest; in 3D axis 0 is depth.
Right-hand sides live on the extended grid (interior + PML on every side) and
are zero inside the PML.
"""
import math
import numpy as np

from .configs import Config


def _coords(n, dim):
    h = 1.0 / n
    x = np.arange(n) * h
    return np.meshgrid(*([x] * dim), indexing="ij")


def medium_bump(n, dim=2, amp=0.5, width=0.15):
    """c = 1 + amp * exp(-|x - centre|^2 / (2 width^2)), centre (0.5, ...)."""
    xs = _coords(n, dim)
    r2 = sum((x - 0.5) ** 2 for x in xs)
    return 1.0 + amp * np.exp(-r2 / (2.0 * width * width))


def medium_grf(n, seed, corr=0.05, cmin=1.5, cmax=4.5):
    """Periodic Gaussian random field with covariance exp(-d^2 / (2 corr^2)),
    affinely mapped so that its minimum is cmin and its maximum cmax.

    White noise N(0,1) on the n x n grid (PCG64(seed)) is filtered in Fourier
    space by a Gaussian of standard deviation corr/sqrt(2); convolving that
    filter with itself gives the stated covariance."""
    rng = np.random.Generator(np.random.PCG64(seed))
    white = rng.standard_normal((n, n))
    h = 1.0 / n
    f = np.fft.fftfreq(n, d=h)                      # cycles per unit length
    fx, fy = np.meshgrid(f, f, indexing="ij")
    sf = corr / math.sqrt(2.0)
    filt = np.exp(-2.0 * (math.pi ** 2) * (sf ** 2) * (fx ** 2 + fy ** 2))
    field = np.real(np.fft.ifft2(np.fft.fft2(white) * filt))
    lo, hi = field.min(), field.max()
    return cmin + (field - lo) * (cmax - cmin) / (hi - lo)


def medium_ellipses(n, rng, background=2.0, nmin=5, nmax=20, cmin=1.0, cmax=10.0):
    """Piecewise-constant high-contrast medium: background speed with n_e
    random ellipses (painter's order; later ellipses overwrite earlier ones)."""
    xs = _coords(n, 2)
    c = np.full((n, n), background)
    ne = int(rng.integers(nmin, nmax + 1))
    for _ in range(ne):
        cx, cy = rng.uniform(0.1, 0.9, size=2)
        a, b = rng.uniform(0.03, 0.2, size=2)
        th = rng.uniform(0.0, math.pi)
        val = rng.uniform(cmin, cmax)
        dx, dy = xs[0] - cx, xs[1] - cy
        u = dx * math.cos(th) + dy * math.sin(th)
        v = -dx * math.sin(th) + dy * math.cos(th)
        c[(u / a) ** 2 + (v / b) ** 2 <= 1.0] = val
    return c


def medium_layered_sphere(n, seed, nlayers=6, cmin=1.5, cmax=5.0):
    """3D layered medium (axis 0 = depth) with a spherical inclusion at half
    the local layer speed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    depths = np.sort(rng.uniform(0.0, 1.0, size=nlayers - 1))
    speeds = rng.uniform(cmin, cmax, size=nlayers)
    centre = rng.uniform(0.3, 0.7, size=3)
    radius = rng.uniform(0.08, 0.15)
    z, y, x = _coords(n, 3)
    layer = np.searchsorted(depths, z, side="right")
    c = speeds[layer]
    inside = (z - centre[0]) ** 2 + (y - centre[1]) ** 2 + (x - centre[2]) ** 2 <= radius ** 2
    c = np.where(inside, 0.5 * c, c)
    return c


def omega_for_ppw(c, ppw, h):
    """Angular frequency giving `ppw` grid points per wavelength at min(c):
    wavelength = 2 pi c_min / omega = ppw * h."""
    return 2.0 * math.pi * float(np.min(c)) / (ppw * h)


def point_source(n, npml, pos, dim):
    """Unit point source at the interior node nearest to `pos` (round half
    up), placed on the extended grid (zero inside the PML)."""
    ne = n + 2 * npml
    f = np.zeros((ne,) * dim, dtype=np.complex128)
    idx = tuple(int(math.floor(p * n + 0.5)) + npml for p in pos)
    f[idx] = 1.0
    return f


def gaussian_source(n, npml, pos, dim, width_cells=2.0):
    """exp(-|x - pos|^2 / (2 (width h)^2)) truncated at 4 sigma, on the
    extended grid."""
    h = 1.0 / n
    xs = _coords(n, dim)
    r2 = sum((x - p) ** 2 for x, p in zip(xs, pos))
    s = width_cells * h
    g = np.exp(-r2 / (2 * s * s))
    g[r2 > (4 * s) ** 2] = 0.0
    f = np.zeros((n + 2 * npml,) * dim, dtype=np.complex128)
    sl = tuple(slice(npml, npml + n) for _ in range(dim))
    f[sl] = g
    return f


def random_rhs(shape, seed):
    """Complex N(0,1) field (real and imaginary parts independent)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def make_problem(cfg: Config):
    """Return (c_interior, omega, h, f_ext) for a single-problem config."""
    if cfg.medium == "bump":
        c = medium_bump(cfg.n, cfg.dim)
    elif cfg.medium == "grf":
        c = medium_grf(cfg.n, cfg.medium_seed, **cfg.extra)
    elif cfg.medium == "layered":
        c = medium_layered_sphere(cfg.n, cfg.medium_seed)
    else:
        raise ValueError(f"config {cfg.name} is not a single-problem workload")
    h = cfg.h
    omega = omega_for_ppw(c, cfg.ppw, h)
    f = point_source(cfg.n, cfg.npml, cfg.source, cfg.dim)
    return c, omega, h, f
