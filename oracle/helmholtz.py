"""Helmholtz operator with an absorbing layer (PML or sponge) on the extended
grid (oracle, test infrastructure).

Follows Sec. 2.1 (Eq. helm, the sponge-layer equation, Eq. discrete_fdm,
Eq. FDM_stencil) and App. A.1.1 (complex coordinate stretching, Laplacian in
stretched form).

Readings where the paper is silent:
  * the absorbing layer sits outside the physical grid (as in the 3D
    benchmark of Sec. 4.1: interior plus a layer on every side);
  * the wave speed inside the layer is the nearest interior value (edge
    replication); k = omega / c;
  * homogeneous Dirichlet values outside the extended grid;
  * stretching s(x) = 1 + i sigma(x), sigma = sigma_max (d / npml)^2, d the
    distance into the layer in cells, evaluated at nodes and half-nodes;
  * default sigma_max = 3 ln(10^6) / (2 k_ref npml h), k_ref = omega / max(c):
    a round-trip amplitude factor 1e-6 for the slowest-decaying wave;
  * the stretched operator is discretised in divergence form
      (A u)_I = - sum_a 1/(h^2 s_a(I)) [ (u_{I+e_a} - u_I)/s_a(I+1/2)
                                          - (u_I - u_{I-e_a})/s_a(I-1/2) ] - k_I^2 u_I,
    which is the paper's 5-point (2D) / 7-point (3D) stencil when s = 1.

Sponge layer (Sec. 2.1): -Lap u - k^2 (1 + i gamma) u = f with the plain
5/7-point Laplacian.  Readings:
  * sign: the paper prints (1 - gamma i), but under its own radiation
    condition (outgoing waves e^{+ikr}, the convention the PML's s = 1 + i
    sigma also follows) that factor amplifies waves entering the layer; the
    absorbing factor is (1 + i gamma) (pinned by a 1D decay test);
  * gamma = gamma_max min(1, sum_a (d_a / npml)^2), d_a the distance into the
    layer along axis a in cells (quadratic in the Euclidean distance to the
    physical domain, constant gamma_max beyond it);
  * default gamma_max = 3 ln(10^6) / (k_ref npml h): for small gamma the
    wave decays like exp(-k gamma x / 2), so the round trip through the
    layer attenuates the slowest wave by 1e-6.

Parity pins (tests/test_oracle_helmholtz.py): discrete plane-wave symbol
(Eq. discrete_symbol) with and without a constant stretching, complex
symmetry of diag(prod_a s_a) A, reduction to Eq. FDM_stencil, and the
outgoing free-space Green's function of the 2D Helmholtz equation.
"""
import math
import numpy as np
import scipy.sparse as sp


def extend_medium(c, npml):
    """Edge-replicate the interior speed c into a layer of npml cells."""
    return np.pad(np.asarray(c, dtype=np.float64), npml, mode="edge")


def default_sigma_max(omega, c, npml, h):
    if npml == 0:
        return 0.0
    k_ref = omega / float(np.max(c))
    return 3.0 * math.log(1e6) / (2.0 * k_ref * npml * h)


def pml_stretch(n, npml, sigma_max):
    """Stretch factors along one axis of the extended grid (n interior nodes).

    Returns (s_node[n_ext], s_half[n_ext + 1]) with s_half[j] = s(j - 1/2),
    i.e. s_half[I] is the face between node I-1 and node I."""
    ne = n + 2 * npml
    lo, hi = npml, npml + n - 1        # first and last interior node

    def sig(x):
        d = np.maximum(0.0, np.maximum(lo - x, x - hi))
        if npml == 0:
            return np.zeros_like(x)
        return sigma_max * (d / npml) ** 2

    xn = np.arange(ne, dtype=np.float64)
    xh = np.arange(ne + 1, dtype=np.float64) - 0.5
    return 1.0 + 1j * sig(xn), 1.0 + 1j * sig(xh)


def default_gamma_max(omega, c, npml, h):
    if npml == 0:
        return 0.0
    k_ref = omega / float(np.max(c))
    return 3.0 * math.log(1e6) / (k_ref * npml * h)


def sponge_gamma(shape_int, npml, gamma_max):
    """Damping gamma on the extended grid: gamma_max min(1, sum_a (d_a/npml)^2)."""
    if npml == 0:
        return np.zeros(tuple(n for n in shape_int))
    D = len(shape_int)
    tot = np.zeros(tuple(n + 2 * npml for n in shape_int))
    for a, n in enumerate(shape_int):
        x = np.arange(n + 2 * npml, dtype=np.float64)
        d = np.maximum(0.0, np.maximum(npml - x, x - (npml + n - 1)))
        shp = [1] * D
        shp[a] = -1
        tot = tot + ((d / npml) ** 2).reshape(shp)
    return gamma_max * np.minimum(1.0, tot)


def setup_operator(c, omega, h, npml, sigma_max=None, absorber="pml", gamma_max=None):
    """Return the operator description (k^2 on the extended grid, per-axis
    stretch factors, sponge damping) for an interior speed field c."""
    c = np.asarray(c, dtype=np.float64)
    cext = extend_medium(c, npml)
    k2 = (omega / cext) ** 2
    if absorber == "pml":
        if sigma_max is None or sigma_max <= 0:
            sigma_max = default_sigma_max(omega, c, npml, h)
        gamma = np.zeros_like(k2)
        gamma_max = 0.0
    elif absorber == "sponge":
        sigma_max = 0.0
        if gamma_max is None or gamma_max <= 0:
            gamma_max = default_gamma_max(omega, c, npml, h)
        gamma = sponge_gamma(c.shape, npml, gamma_max)
    else:
        raise ValueError(absorber)
    stretch = [pml_stretch(c.shape[a], npml, sigma_max) for a in range(c.ndim)]
    return {"k2": k2, "h": float(h), "stretch": stretch, "npml": npml,
            "sigma_max": sigma_max, "omega": float(omega), "absorber": absorber,
            "gamma": gamma, "gamma_max": gamma_max}


def apply(op, u):
    """A u for a complex field u on the extended grid (Dirichlet ghosts)."""
    u = np.asarray(u, dtype=np.complex128)
    h2 = op["h"] ** 2
    out = -op["k2"] * (1.0 + 1j * op.get("gamma", 0.0)) * u
    D = u.ndim
    for a in range(D):
        s_node, s_half = op["stretch"][a]
        shp = [1] * D
        shp[a] = -1
        sn = s_node.reshape(shp)
        sl = s_half[:-1].reshape(shp)      # face I - 1/2
        sr = s_half[1:].reshape(shp)       # face I + 1/2
        pad = [(0, 0)] * D
        pad[a] = (1, 1)
        up = np.pad(u, pad)
        idx_p = [slice(None)] * D
        idx_m = [slice(None)] * D
        idx_p[a] = slice(2, None)
        idx_m[a] = slice(0, -2)
        u_p = up[tuple(idx_p)]
        u_m = up[tuple(idx_m)]
        flux = (u_p - u) / sr - (u - u_m) / sl
        out = out - flux / (h2 * sn)
    return out


def assemble(op):
    """Sparse matrix of A (row-major flattening), built entry by entry."""
    k2 = op["k2"]
    shape = k2.shape
    D = len(shape)
    N = k2.size
    h2 = op["h"] ** 2
    rows, cols, vals = [], [], []
    strides = [int(np.prod(shape[a + 1:])) for a in range(D)]
    for flat in range(N):
        I = np.unravel_index(flat, shape)
        diag = -k2[I] * (1.0 + 1j * (op["gamma"][I] if "gamma" in op else 0.0))
        for a in range(D):
            s_node, s_half = op["stretch"][a]
            i = I[a]
            cm = 1.0 / (h2 * s_node[i] * s_half[i])
            cp = 1.0 / (h2 * s_node[i] * s_half[i + 1])
            diag += cm + cp
            if i > 0:
                rows.append(flat); cols.append(flat - strides[a]); vals.append(-cm)
            if i < shape[a] - 1:
                rows.append(flat); cols.append(flat + strides[a]); vals.append(-cp)
        rows.append(flat); cols.append(flat); vals.append(diag)
    return sp.csr_matrix((np.array(vals), (np.array(rows), np.array(cols))), shape=(N, N))


def residual(op, f, u):
    return np.asarray(f, dtype=np.complex128) - apply(op, u)
