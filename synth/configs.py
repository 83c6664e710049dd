"""Workload configurations (problem sizes, levels, channels, solver settings)."""
from dataclasses import dataclass, field
from typing import Tuple


@dataclass(frozen=True)
class Config:
    name: str
    dim: int                     # spatial dimension D (2 or 3)
    n: int                       # interior nodes per axis
    npml: int                    # PML cells per side (extended grid = n + 2*npml)
    ppw: float                   # points per wavelength at the slowest speed
    channels: Tuple[int, ...]    # C_1..C_L (C_1 = 2 = Re/Im of the complex field)
    nu1: Tuple[int, ...]         # pre-smoothing steps per level
    nu2: Tuple[int, ...]         # post-smoothing steps per level
    restart: int                 # FGMRES restart length m
    tol: float = 1e-6
    maxit: int = 500
    weight_seed: int = 0
    medium: str = "bump"
    medium_seed: int = 0
    source: Tuple[float, ...] = ()
    extra: dict = field(default_factory=dict, compare=False, hash=False)

    @property
    def levels(self) -> int:
        return len(self.channels)

    @property
    def n_ext(self) -> int:
        return self.n + 2 * self.npml

    @property
    def h(self) -> float:
        return 1.0 / self.n


def ext_side(n: int, npml: int) -> int:
    return n + 2 * npml


def level_sides(n_ext: int, levels: int):
    """Side length per level as the configurations document it (ceil halving)."""
    out = [n_ext]
    for _ in range(levels - 1):
        out.append((out[-1] + 1) // 2)
    return out


CONFIGS = {
    # Plain method, small (parity workload).
    "bump64": Config(name="bump64", dim=2, n=64, npml=8, ppw=10.0,
                     channels=(2, 8, 16), nu1=(2, 2, 2), nu2=(2, 2, 2),
                     restart=30, maxit=500, weight_seed=0, medium="bump",
                     source=(0.5, 0.25)),
    # 2D 1024^2, GRF speed in [1.5, 4.5].
    "grf1024": Config(name="grf1024", dim=2, n=1024, npml=16, ppw=10.0,
                      channels=(2, 8, 16, 32, 64, 64), nu1=(2,) * 6, nu2=(2,) * 6,
                      restart=30, maxit=500, weight_seed=0, medium="grf", medium_seed=1,
                      source=(0.5, 0.25), extra={"corr": 0.05, "cmin": 1.5, "cmax": 4.5}),
    # Batched: 64 problems of uneven side (sides drawn per problem).
    "ellipses64": Config(name="ellipses64", dim=2, n=0, npml=16, ppw=8.0,
                         channels=(2, 8, 16, 32, 64), nu1=(2,) * 5, nu2=(2,) * 5,
                         restart=30, maxit=500, weight_seed=0, medium="ellipses",
                         medium_seed=2,
                         extra={"count": 64, "sides": (128, 256, 384, 512, 768)}),
    # 3D 192^3, layered medium + sphere.
    "layered192": Config(name="layered192", dim=3, n=192, npml=12, ppw=8.0,
                         channels=(2, 12, 24, 48, 96), nu1=(2,) * 5, nu2=(2,) * 5,
                         restart=20, maxit=500, weight_seed=0, medium="layered",
                         medium_seed=4, source=(0.1, 0.5, 0.5)),
}
