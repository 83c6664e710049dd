"""The 3D V-cycle at the channel widths of the 192^3 layered workload
(channels 2/12/24/48/96, 3^3 kernels, 5 levels) against the FP64 oracle
(Alg. 2), on a grid the oracle finishes in seconds: 40^3 interior + 4-cell
PML = 48^3 extended, levels 48, 24, 12, 6, 3.

Each tile shape that the 216^3 plan picks for some convolution is forced
through MCMG_FORCE_TILE (where it is a candidate), so the wide-channel
matrix-core paths of that plan run here: in BF16 the weights stream through
LDS in several chunks (at C = 48 and C = 96 the packed weights exceed the
96 KB chunk budget); in FP32 they are read from global memory by runs of
four K steps, and at C = 48 and C = 96 (channels in multiples of 16) the K
walker advances once per group; two and four column tiles per block, four
node rows per wave, and the prolongation from C = 96 to C = 48 as a
384-column depth-to-space GEMM.  Bars: one application within 1e-5
relative L2 (FP32) and 2e-2 (BF16); three FGMRES(20) iterations follow the
oracle's history."""
import numpy as np
import pytest

import synth
from _gpu_common import handle, oracle_parts, problem, rel_l2, say, to_dev, to_host
from oracle import helmholtz, krylov

pytestmark = pytest.mark.gpu

DIM, N, NPML, CH = 3, 40, 4, (2, 12, 24, 48, 96)
# every (mt, ntw, rpw) the packaged 216^3 plan holds, FP32 and BF16
PLAN_TILES = ["1,1,4", "1,2,2", "1,1,1", "1,2,1", "2,2,1", "1,4,1", "2,2,2", "1,1,2", "1,4,2"]
# the z-marching form of the C = 12 stride-1 convolutions (FP32), a tile of its own
ZMARCH_TILE = "1,1,8"

_cache = {}


def _setup():
    if "p" not in _cache:
        p = problem(DIM, N, NPML, CH, ppw=8.0, medium="layered")
        op, W, M = oracle_parts(p)
        shape = (N + 2 * NPML,) * DIM
        r = synth.random_rhs(shape, 21)
        _cache.update(p=p, op=op, M=M, r=r, z=M(r))
    return _cache


def test_level_shapes_and_channels():
    """The handle's level hierarchy is the one the oracle builds."""
    say("[widths3d-levels]")
    d = _setup()
    H = handle(d["p"])
    sides = [48, 24, 12, 6, 3]
    for l, (side, C) in enumerate(zip(sides, CH), start=1):
        shape, c = H.level_shape(l)
        assert tuple(shape) == (side,) * 3 and c == C
        assert d["M"].feats["a"][l].shape == (C,) + (side,) * 3
    H.close()


def _apply(H, r):
    """z = MG(r) through the C ABI, with the matrix-core kernels it launched."""
    H.prof_enable(True)
    z = to_dev(np.zeros_like(r))
    H.apply(to_dev(r), z)
    names = {rec["name"] for rec in H.prof_report()}
    H.prof_enable(False)
    return to_host(z), sorted(n for n in names if n.startswith(("mconv_kernel", "mconvz_kernel")))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_apply_default_plan(precision):
    say(f"[widths3d-apply] {precision}")
    d = _setup()
    H = handle(d["p"], precision)
    z, _ = _apply(H, d["r"])
    err = rel_l2(z, d["z"])
    say(f"  rel L2 {err:.3e}")
    H.close()
    _cache[("z", precision)] = z
    assert err <= (1e-5 if precision == "fp32" else 2e-2), err
    if precision == "bf16":
        assert err > 1e-6


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("tile", PLAN_TILES + [ZMARCH_TILE])
def test_apply_forced_plan_tiles(tile, precision, monkeypatch):
    """The forced tile really runs (it names launched kernels), the result is
    within the bar, and it equals the default plan's bitwise: every tile
    takes each output's K-sum in the same order."""
    monkeypatch.setenv("MCMG_FORCE_TILE", tile)
    say(f"[widths3d-tile] {tile} {precision}")
    d = _setup()
    H = handle(d["p"], precision)
    z, kernels = _apply(H, d["r"])
    H.close()
    err = rel_l2(z, d["z"])
    mt, ntw, rpw = tile.split(",")
    if tile == ZMARCH_TILE:
        forced = [k for k in kernels if k.startswith("mconvz_kernel<")]
        if precision == "bf16":          # FP32 only: nothing to force
            assert not forced, kernels
            return
    else:
        forced = [k for k in kernels if k.endswith(f", {mt}, {ntw}, {rpw}>")]
    say(f"  rel L2 {err:.3e}; {len(forced)} of {len(kernels)} convolution kernels on the tile")
    assert forced, kernels
    assert err <= (1e-5 if precision == "fp32" else 2e-2), err
    if ("z", precision) in _cache:
        assert np.array_equal(z, _cache[("z", precision)])


def test_features_match_oracle():
    """Alg. 1 at these widths: a_l, s_l within 1e-5."""
    import torch
    say("[widths3d-setup]")
    d = _setup()
    H = handle(d["p"])
    for l in range(1, len(CH) + 1):
        shape, C = H.level_shape(l)
        a = torch.zeros(tuple(shape) + (C,), dtype=torch.float32, device="cuda")
        s = torch.zeros_like(a)
        H.get_features(l, a, s)
        assert rel_l2(to_host(a), np.moveaxis(d["M"].feats["a"][l], 0, -1)) < 1e-5
        assert rel_l2(to_host(s), np.moveaxis(d["M"].feats["s"][l], 0, -1)) < 1e-5
    H.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_fgmres20_three_iterations_follow_oracle(precision):
    """FGMRES(20) (the 216^3 workload's restart length): the residual
    estimates of three iterations and the iterate against the oracle's
    FGMRES with the FP64 V-cycle (FP32: 1e-5 / 1e-4; BF16: 5e-2)."""
    say(f"[widths3d-fgmres] {precision}")
    d = _setup()
    p, op, M = d["p"], d["op"], d["M"]
    f = synth.point_source(N, NPML, (0.1, 0.5, 0.5), DIM)
    if "fg" not in _cache:
        _cache["fg"] = krylov.fgmres(lambda x: helmholtz.apply(op, x), M, f, m=20, tol=1e-6,
                                     maxit=3)
    uo, io = _cache["fg"]
    H = handle(p, precision, restart=20)
    u = to_dev(np.zeros_like(f))
    info = H.solve(to_dev(f), u, tol=1e-6, maxit=3)
    H.close()
    hg, ho = np.array(info["hist"]), np.array(io["hist"])
    say(f"  gpu {hg} oracle {ho}")
    assert info["iters"] == io["iters"] == 3
    tol_h, tol_u = (1e-5, 1e-4) if precision == "fp32" else (5e-2, 5e-2)
    assert np.max(np.abs(hg - ho) / ho) < tol_h
    assert rel_l2(to_host(u), uo) < tol_u
    true = np.linalg.norm(f - helmholtz.apply(op, to_host(u))) / np.linalg.norm(f)
    assert abs(info["relres_true"] - true) <= 1e-10 * true
