"""Seeded random-init weights and the self-describing weight blob.

Canonical tensor order (the order weights are drawn and stored):

    f_lift [C_1][1][T], g_lift [C_1][2][T], g_proj [2][C_1][T],
    then for each level l = 1..L:
        f_s^l [C_l][C_l][T], W_l [C_l][C_l][T], KA_l [C_l][C_l][T], KS_l [C_l][C_l][T],
        Wsm_l^(i) [C_l][C_l][T] for i = 1..(nu1_l + nu2_l) (only nu1_L at l = L),
        and, if l < L: f_a^l [C_{l+1}][C_l][T], R_l [C_{l+1}][C_l][T], P_l [C_{l+1}][C_l][T].

T = 3^D taps in row-major tap order (tap offset d_a - 1 per axis).  Every
tensor except P is a convolution weight [out][in][T]; P is a transposed
convolution weight [in = C_{l+1}][out = C_l][T].  Values are drawn in this
order from one PCG64(seed) stream as standard normals times sqrt(1/fan_in),
fan_in = (input channels of the op) * T, and stored as float32.

Blob layout (little endian):
    header (256 bytes): magic "MCMGWB01", u32 version=1, u32 dim, u32 levels,
        u32 ksize=3, u32 channels[8], u32 nu1[8], u32 nu2[8], u32 ntensors,
        zero padding to 256 bytes;
    tensor table: ntensors records of {u32 kind, u32 level (1-based; 0 for
        the global tensors), u32 step (1-based for Wsm, else 0), u32 d0,
        u32 d1, u32 taps, u64 offset}, 32 bytes each;
    data: float32 tensors [d0][d1][taps], each at its 64-byte aligned offset.
"""
import struct
import numpy as np

MAGIC = b"MCMGWB01"
KINDS = {"f_lift": 0, "g_lift": 1, "g_proj": 2, "f_s": 3, "W": 4, "KA": 5, "KS": 6,
         "Wsm": 7, "f_a": 8, "R": 9, "P": 10}


def weight_names(dim, channels, nu1, nu2):
    """Canonical (kind, level, step, d0, d1, fan_in_channels) list."""
    L = len(channels)
    out = [("f_lift", 0, 0, channels[0], 1, 1),
           ("g_lift", 0, 0, channels[0], 2, 2),
           ("g_proj", 0, 0, 2, channels[0], channels[0])]
    for l in range(1, L + 1):
        C = channels[l - 1]
        out.append(("f_s", l, 0, C, C, C))
        out.append(("W", l, 0, C, C, C))
        out.append(("KA", l, 0, C, C, C))
        out.append(("KS", l, 0, C, C, C))
        nsteps = nu1[l - 1] + (nu2[l - 1] if l < L else 0)
        for i in range(1, nsteps + 1):
            out.append(("Wsm", l, i, C, C, C))
        if l < L:
            Cn = channels[l]
            out.append(("f_a", l, 0, Cn, C, C))
            out.append(("R", l, 0, Cn, C, C))
            out.append(("P", l, 0, Cn, C, Cn))
    return out


def make_weights(dim, channels, nu1, nu2, seed):
    """Return a list of dicts {kind, level, step, w (float32 [d0][d1][3^D])}."""
    taps = 3 ** dim
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for kind, level, step, d0, d1, fin in weight_names(dim, channels, nu1, nu2):
        std = np.sqrt(1.0 / (fin * taps))
        w = (rng.standard_normal((d0, d1, taps)) * std).astype(np.float32)
        out.append({"kind": kind, "level": level, "step": step, "w": w})
    return out


def pack_blob(dim, channels, nu1, nu2, tensors):
    """Serialise tensors (canonical order) into the weight blob (bytes)."""
    L = len(channels)
    if L > 8:
        raise ValueError("at most 8 levels")
    pad8 = lambda v: list(v) + [0] * (8 - len(v))
    head = MAGIC + struct.pack("<4I", 1, dim, L, 3)
    head += struct.pack("<8I", *pad8(channels))
    head += struct.pack("<8I", *pad8(nu1))
    head += struct.pack("<8I", *pad8(nu2))
    head += struct.pack("<I", len(tensors))
    head += b"\0" * (256 - len(head))
    table_bytes = 32 * len(tensors)
    off = 256 + table_bytes
    off = (off + 63) // 64 * 64
    table = b""
    data = []
    for t in tensors:
        w = np.ascontiguousarray(t["w"], dtype=np.float32)
        d0, d1, taps = w.shape
        table += struct.pack("<6IQ", KINDS[t["kind"]], t["level"], t["step"], d0, d1, taps, off)
        data.append((off, w.tobytes()))
        off += w.nbytes
        off = (off + 63) // 64 * 64
    buf = bytearray(off)
    buf[:256] = head
    buf[256:256 + table_bytes] = table
    for o, b in data:
        buf[o:o + len(b)] = b
    return bytes(buf)
