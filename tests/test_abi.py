"""The C-ABI library loads and exports every symbol include/mcmg.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mcmg_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2606_30495_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmcmg.so not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            names += _declared(h)
    assert "mcmg_setup" in names and "mcmg_apply" in names and "mcmg_solve" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding covers the same names
    for n in names:
        assert n in _lib.EXPORTS, n


def test_blob_layout_roundtrip():
    """The weight blob's table lists every tensor in canonical order at
    aligned offsets."""
    import struct
    import numpy as np
    import synth
    tens = synth.make_weights(2, (2, 8, 16), (2, 2, 2), (2, 2, 2), 0)
    blob = synth.pack_blob(2, (2, 8, 16), (2, 2, 2), (2, 2, 2), tens)
    assert blob[:8] == b"MCMGWB01"
    n = struct.unpack_from("<I", blob, 8 + 4 * 4 + 3 * 32)[0]
    assert n == len(tens) == 3 + (4 + 4 + 3) * 2 + (4 + 2)
    for k, t in enumerate(tens):
        kind, lvl, step, d0, d1, taps, off = struct.unpack_from("<6IQ", blob, 256 + 32 * k)
        assert off % 64 == 0 and (d0, d1, taps) == t["w"].shape
        got = np.frombuffer(blob, dtype=np.float32, count=d0 * d1 * taps, offset=off)
        assert np.array_equal(got.reshape(d0, d1, taps), t["w"])


def test_setup_errors_without_gpu_are_reported(monkeypatch):
    """Argument validation happens before any device work."""
    from paper_2606_30495_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmcmg.so not built")
    lib = _lib.lib()
    import numpy as np
    c = np.ones((4, 4))
    g = _lib.Grid(5, (ctypes.c_int * 3)(4, 4, 1))
    out = ctypes.c_void_p()
    st = lib.mcmg_setup(c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), g, 1.0, 0.1,
                        _lib.Pml(0, 0.0), _lib.Weights(None, 0), None, ctypes.byref(out))
    assert st == -1 and b"dim" in lib.mcmg_last_error()
