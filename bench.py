"""Benchmark: FGMRES + McMg V-cycle iterations per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config grf1024]
                    [--precision fp32|bf16] [--no-cpu]

A step is one FGMRES iteration of the whole hot path: one V-cycle (lift,
smoothing, restriction, coarsest level, prolongation, projection), one FP64
Helmholtz+PML matvec, the FP64 Gram-Schmidt pass(es) and the Givens update;
the timed region is one solve of K iterations from u = 0 (it also contains
the initial residual, the solution update u += Z y and the final FP64 true
residual).  Inputs are resident in HBM before timing starts.  Prints one
JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3     # vector and matrix FP32
PEAK_BF16_TFLOPS = 2500.0    # dense MFMA
PEAK_FP64_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="grf1024")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=3)
    return ap.parse_args()


def roofline_for(rec, precision):
    """Roofline entry for one kernel record {avg_ms, flops_per_launch,
    bytes_per_launch}: the bound is the one its algorithmic intensity sits
    under (ridge = peak flops / peak bytes)."""
    fl, by, ms = rec["flops_per_launch"], rec["bytes_per_launch"], rec["avg_ms"]
    name = rec["name"]
    if name.startswith("mconv_kernel") and "bf16" in name:
        peak_fl, unit_bound = PEAK_BF16_TFLOPS, "mfma"
    elif name.startswith("mconv_kernel"):
        peak_fl, unit_bound = PEAK_FP32_TFLOPS, "mfma"
    elif name.startswith(("multidot", "update", "zupdate", "helm")):
        peak_fl, unit_bound = PEAK_FP64_TFLOPS, "alu"
    else:
        peak_fl, unit_bound = PEAK_FP32_TFLOPS, "alu"
    ridge = peak_fl * 1e12 / (PEAK_HBM_GBS * 1e9)
    intensity = fl / max(by, 1.0)
    if intensity < ridge:
        ach = by / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(ach, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None}
    ach = fl / (ms * 1e-3) / 1e12
    return {"bound": unit_bound, "achieved": round(ach, 3), "peak": peak_fl, "unit": "TFLOP/s",
            "frac": round(ach / peak_fl, 4), "traffic": None}


def cpu_baseline(cfg, c, omega, h, f, tens, iters):
    """The FP64 oracle on the host cores: setup + `iters` FGMRES iterations of
    the same workload (a bounded sample of the solve)."""
    import numpy as np
    from oracle import helmholtz, krylov, mcmg
    try:
        import threadpoolctl
        blas = [p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()
                if p.get("user_api") == "blas"]
        threads = max(blas) if blas else 1
    except Exception:
        threads = 1
    t0 = time.perf_counter()
    op = helmholtz.setup_operator(c, omega, h, cfg.npml)
    W = mcmg.Weights(cfg.dim, cfg.channels, cfg.nu1, cfg.nu2, tens)
    M = mcmg.Preconditioner(W, np.sqrt(op["k2"]), h)
    t1 = time.perf_counter()
    _, info = krylov.fgmres(lambda x: helmholtz.apply(op, x), M, f, m=cfg.restart,
                            tol=cfg.tol, maxit=iters)
    t2 = time.perf_counter()
    return {"value": round(info["iters"] / (t2 - t1), 5), "unit": "iters/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{cfg.name}: oracle setup ({t1 - t0:.1f} s) then {info['iters']} FGMRES "
                      f"iterations ({t2 - t1:.1f} s) from u=0; BLAS threads {threads}, NumPy "
                      f"elementwise work single-threaded; host {os.cpu_count()} CPUs"}


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(independent solves shard across GPUs without communication; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import synth
    from paper_2606_30495_amd import Handle

    cfg = synth.CONFIGS[a.config]
    c, omega, h, f = synth.make_problem(cfg)
    tens = synth.make_weights(cfg.dim, cfg.channels, cfg.nu1, cfg.nu2, cfg.weight_seed)
    blob = synth.pack_blob(cfg.dim, cfg.channels, cfg.nu1, cfg.nu2, tens)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = Handle(c, omega, h, cfg.npml, blob, precision=a.precision, restart=cfg.restart)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3

    fd = torch.from_numpy(f).to("cuda")
    ud = torch.zeros_like(fd)
    if a.warmup > 0:
        H.solve(fd, ud, tol=cfg.tol, maxit=a.warmup, hist_cap=0)
    # timed region: one solve of K iterations from u = 0
    ud.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = H.solve(fd, ud, tol=cfg.tol, maxit=a.steps, hist_cap=0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    iters = info["iters"]
    value = iters / el
    # same solve again with per-launch HIP-event timing for the kernel breakdown
    ud.zero_()
    H.prof_enable(True)
    H.solve(fd, ud, tol=cfg.tol, maxit=a.steps, hist_cap=0)
    recs = H.prof_report()
    H.prof_enable(False)
    recs.sort(key=lambda r: -r["total_ms"])
    dom = recs[0]
    roof = roofline_for(dom, a.precision)
    roof["kernel"] = dom["name"]
    roof["launches_per_step"] = round(dom["launches"] / max(iters, 1), 2)
    roof["avg_launch_us"] = round(dom["avg_ms"] * 1e3, 3)
    line = {
        "metric": "FGMRES+V-cycle iters/s (solves/s to rel-res 1e-6; p50/p99 solve latency)",
        "value": round(value, 3), "unit": "iters/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(el / max(iters, 1) * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if a.precision == "fp32" else "bf16",
        "data": "synthetic (seeded medium, random-init weights N(0,1/fan_in) seed 0)",
        "config": {"workload": cfg.name, "dim": cfg.dim, "n_interior": cfg.n, "npml": cfg.npml,
                   "n_ext": cfg.n_ext, "levels": cfg.levels, "channels": list(cfg.channels),
                   "nu": [cfg.nu1[0], cfg.nu2[0]], "restart": cfg.restart,
                   "precision": a.precision, "outer": "f64"},
        "solve": {"iters": iters, "relres_true": info["relres_true"],
                  "converged": info["converged"], "setup_ms": round(setup_ms, 2)},
        "roofline": roof,
        "kernels": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
                    for r in recs[:16]],
    }
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg, c, omega, h, f, tens, a.cpu_iters)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
