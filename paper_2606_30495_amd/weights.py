"""Weight blob reading and writing on the host, and LLPF growth (Sec. llpf).

The blob is the self-describing format of include/mcmg.h: a 256-byte header
(magic, version, dim, levels, ksize, channels[8], nu1[8], nu2[8], tensor
count), a table of 32-byte records (kind, level, step, d0, d1, taps, offset)
and float32 tensors [d0][d1][taps] at 64-byte aligned offsets, in the
canonical order the library checks.
"""
import struct

import numpy as np

MAGIC = b"MCMGWB01"
KIND_NAMES = ["f_lift", "g_lift", "g_proj", "f_s", "W", "KA", "KS", "Wsm", "f_a", "R", "P"]


def parse_blob(blob):
    """(header dict, [tensor dict {kind, level, step, w}]) of a blob."""
    b = bytes(blob)
    if b[:8] != MAGIC:
        raise ValueError("not a weight blob")
    hdr = struct.unpack_from("<4I8I8I8II", b, 8)
    version, dim, L, ks = hdr[:4]
    if version != 1 or ks != 3:
        raise ValueError("unsupported blob version")
    head = {"dim": dim, "levels": L, "channels": list(hdr[4:12][:L]),
            "nu1": list(hdr[12:20][:L]), "nu2": list(hdr[20:28][:L])}
    nt = hdr[28]
    out = []
    for k in range(nt):
        kind, level, step, d0, d1, taps, off = struct.unpack_from("<6IQ", b, 256 + 32 * k)
        w = np.frombuffer(b, dtype=np.float32, count=d0 * d1 * taps, offset=off).reshape(d0, d1, taps)
        out.append({"kind": KIND_NAMES[kind], "level": level, "step": step, "w": w.copy()})
    return head, out


def build_blob(head, tensors):
    """Serialise a header dict and tensors (canonical order) into a blob."""
    L = head["levels"]
    pad8 = lambda v: list(v) + [0] * (8 - len(v))
    hdr = MAGIC + struct.pack("<4I8I8I8II", 1, head["dim"], L, 3, *pad8(head["channels"]),
                              *pad8(head["nu1"]), *pad8(head["nu2"]), len(tensors))
    hdr = hdr + b"\0" * (256 - len(hdr))
    off = 256 + 32 * len(tensors)
    off = (off + 63) // 64 * 64
    table, data, pos = b"", b"", off
    for t in tensors:
        w = np.ascontiguousarray(t["w"], dtype=np.float32)
        d0, d1, taps = w.shape
        table += struct.pack("<6IQ", KIND_NAMES.index(t["kind"]), t["level"], t["step"], d0, d1, taps, pos)
        raw = w.tobytes()
        raw += b"\0" * ((-len(raw)) % 64)
        data += raw
        pos += len(raw)
    body = hdr + table
    body += b"\0" * (off - len(body))
    return body + data


def split_flat(tensors, flat):
    """Canonical float32 vector -> tensors with the shapes of `tensors`."""
    out, o = [], 0
    for t in tensors:
        n = int(np.prod(t["w"].shape))
        out.append(dict(t, w=np.asarray(flat[o:o + n], dtype=np.float32).reshape(t["w"].shape)))
        o += n
    if o != len(flat):
        raise ValueError("vector length does not match the model")
    return out


def grow(old_blob, fresh_blob):
    """LLPF architecture growth.  fresh_blob: an initialisation of the grown
    model (one more level).  Every tensor the old model holds (same kind,
    level and step) is copied over; the rest are the new parameters.
    Returns (blob, trainable mask): the mask marks exactly the new tensors,
    i.e. the new level, the transfers to it and the old coarsest level's
    post-smoothing weights."""
    ho, to = parse_blob(old_blob)
    hf, tf = parse_blob(fresh_blob)
    if hf["levels"] != ho["levels"] + 1 or hf["dim"] != ho["dim"]:
        raise ValueError("the grown model must add exactly one level")
    have = {(t["kind"], t["level"], t["step"]): t["w"] for t in to}
    out, mask = [], []
    for t in tf:
        k = (t["kind"], t["level"], t["step"])
        if k in have:
            if have[k].shape != t["w"].shape:
                raise ValueError(f"tensor {k} changes shape")
            out.append(dict(t, w=have[k]))
            mask.append(0)
        else:
            out.append(t)
            mask.append(1)
    return build_blob(hf, out), mask
