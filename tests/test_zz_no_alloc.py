"""mcmg_apply_noalloc (the entry point for callers that cannot allocate)
through the C ABI against mcmg_apply on the same handle and input: the
same kernels in the same order on the library's static scratch array give
the same bits.  Two calls in a row, the second on a smaller grid (the
array keeps the first call's contents), in 2D and 3D; a grid whose level
state exceeds the array is refused."""
import numpy as np
import pytest

import synth
from _gpu_common import handle, oracle_parts, problem, rel_l2, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _pair(H, seed):
    r = synth.random_rhs(H.ext_shape, seed)
    rd = to_dev(r)
    z_ref = to_dev(np.zeros_like(r))
    z_na = to_dev(np.full_like(r, np.nan))
    H.apply(rd, z_ref)
    H.apply_noalloc(rd, z_na)
    return r, to_host(z_ref), to_host(z_na)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_noalloc_equals_apply_two_calls_smaller_second(precision):
    say(f"[noalloc-2d] {precision}")
    big = problem(2, 64, 8, (2, 8, 16))          # 80^2, 3 levels
    small = problem(2, 24, 4, (2, 8, 16))        # 32^2, 3 levels
    Hb, Hs = handle(big, precision), handle(small, precision)
    _, zr, zn = _pair(Hb, 41)
    assert np.array_equal(zn, zr)
    r, zr2, zn2 = _pair(Hs, 42)
    assert np.array_equal(zn2, zr2)
    # and against the oracle on the smaller grid, to the precision's bar
    _, _, M = oracle_parts(small)
    err = rel_l2(zn2, M(r))
    say(f"  second call rel L2 vs oracle {err:.3e}")
    assert err <= (1e-5 if precision == "fp32" else 2e-2)
    # the handle's own path still works after the scratch calls
    _, zr3, zn3 = _pair(Hb, 43)
    assert np.array_equal(zn3, zr3)
    Hb.close()
    Hs.close()


def test_noalloc_3d_widths_then_smaller():
    say("[noalloc-3d]")
    a = problem(3, 40, 4, (2, 12, 24, 48, 96), ppw=8.0, medium="layered")   # 48^3
    b = problem(3, 14, 3, (2, 4, 8))                                        # 20^3
    Ha, Hb = handle(a), handle(b)
    _, zr, zn = _pair(Ha, 44)
    assert np.array_equal(zn, zr)
    _, zr2, zn2 = _pair(Hb, 45)
    assert np.array_equal(zn2, zr2)
    Ha.close()
    Hb.close()


def test_noalloc_refuses_a_grid_beyond_the_array():
    """2D 1024^2 + 16-cell PML (1056^2), 6 levels 2/8/16/32/64/64: the level
    state is about 106 MiB, more than the 64 MiB array; refused with
    MCMG_E_ARG before any device work."""
    from paper_2606_30495_amd import McmgError
    say("[noalloc-too-big]")
    p = problem(2, 1024, 16, (2, 8, 16, 32, 64, 64))
    H = handle(p)
    r = to_dev(np.zeros(H.ext_shape, dtype=np.complex128))
    z = to_dev(np.zeros(H.ext_shape, dtype=np.complex128))
    with pytest.raises(McmgError) as exc:
        H.apply_noalloc(r, z)
    H.close()
    assert exc.value.status == -1          # MCMG_E_ARG
