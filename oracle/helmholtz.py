"""Helmholtz + PML operator on the extended grid (oracle, test infrastructure).

Follows Sec. 2.1 (Eq. helm, Eq. discrete_fdm, Eq. FDM_stencil) and App. A.1.1
(complex coordinate stretching, Laplacian in stretched form).

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


def setup_operator(c, omega, h, npml, sigma_max=None):
    """Return the operator description (k^2 on the extended grid, per-axis
    stretch factors) for an interior speed field c."""
    c = np.asarray(c, dtype=np.float64)
    if sigma_max is None or sigma_max <= 0:
        sigma_max = default_sigma_max(omega, c, npml, h)
    cext = extend_medium(c, npml)
    k2 = (omega / cext) ** 2
    stretch = [pml_stretch(c.shape[a], npml, sigma_max) for a in range(c.ndim)]
    return {"k2": k2, "h": float(h), "stretch": stretch, "npml": npml,
            "sigma_max": sigma_max, "omega": float(omega)}


def apply(op, u):
    """A u for a complex field u on the extended grid (Dirichlet ghosts)."""
    u = np.asarray(u, dtype=np.complex128)
    h2 = op["h"] ** 2
    out = -op["k2"] * u
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
        diag = -k2[I]
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
