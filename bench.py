"""Benchmark: FGMRES + McMg V-cycle iterations per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config layered192]
                    [--precision fp32|bf16] [--no-cpu]

The headline workload is the largest single-solve configuration: the 3D
192^3 layered medium (216^3 extended, 5 levels 2/12/24/48/96, FGMRES(20)),
with the V-cycle in FP32, the paper's preconditioner precision (Sec. 4.1).

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
PEAK_FP32_MFMA_TFLOPS = 157.3   # dense FP32 matrix cores
# FP32 vector rate without packed-FP32 instructions (the library is built
# with them disabled): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz;
# the 157.3 TFLOP/s vector figure needs packed FP32
PEAK_FP32_VALU_TFLOPS = 78.6
PEAK_BF16_TFLOPS = 2500.0       # dense MFMA
PEAK_FP64_TFLOPS = 78.6
# iteration cap of the serving leg: the classical stand-in coefficients need
# 150-750 iterations on most of these media and 1.6-1.9k on the ellipse
# medium with the widest contrast (speeds 1.5-9.9) at restart 30
SERVE_MAXIT = 2500


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="layered192")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--grf-steps", type=int, default=30,
                    help="iterations of the 2D 1024^2 leg in each precision (0: skip)")
    ap.add_argument("--single", action="store_true", help="skip the other-precision leg")
    ap.add_argument("--solves", type=int, default=50,
                    help="right-hand sides of the solve-to-tolerance leg (0: skip)")
    ap.add_argument("--batched-iters", type=int, default=30,
                    help="iterations of the batched leg (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=16,
                    help="requests of the serving leg (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=40.0)
    ap.add_argument("--serve-scale", default="small", choices=list(SERVE_SCALES),
                    help="size classes of the serving leg")
    ap.add_argument("--born-iters", type=int, default=20,
                    help="Born-series steps per method in the Born leg (0: skip)")
    ap.add_argument("--train-steps", type=int, default=15000,
                    help="Adam steps of the training leg, about four minutes (0: skip)")
    ap.add_argument("--train-seconds", type=float, default=None,
                    help="0 skips the training leg (same as --train-steps 0)")
    ap.add_argument("--trained-rhs", type=int, default=10,
                    help="right-hand sides solved with the trained weights")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=1,
                    help="FGMRES iterations of the oracle sample")
    ap.add_argument("--cpu-side", type=int, default=104,
                    help="interior side of the oracle's reduced-grid sample of a 3D "
                         "headline workload")
    a = ap.parse_args()
    if a.train_seconds == 0:
        a.train_steps = 0
    return a


# kernel-name prefixes of the matrix-core launches: implicit-GEMM
# convolutions (tiled and z-marching forms) and fused smoothing steps
MATRIX_CORE_KERNELS = ("mconv_kernel", "mconvz_kernel", "mstep_kernel")


def roofline_for(rec, precision):
    """Roofline entry for one kernel record {avg_ms, flops_per_launch,
    bytes_per_launch}: the bound is the one its algorithmic intensity sits
    under (ridge = peak flops / peak bytes)."""
    fl, by, ms = rec["flops_per_launch"], rec["bytes_per_launch"], rec["avg_ms"]
    name = rec["name"]
    if name.startswith(("mconv_kernel<", "mstep_kernel<")) and ", true," in name:
        peak_fl, unit_bound = PEAK_BF16_TFLOPS, "mfma"
    elif name.startswith(MATRIX_CORE_KERNELS):     # (the z-marching form is float32)
        peak_fl, unit_bound = PEAK_FP32_MFMA_TFLOPS, "mfma"
    elif name.startswith(("multidot", "update", "zupdate", "helm")):
        peak_fl, unit_bound = PEAK_FP64_TFLOPS, "alu"
    else:
        peak_fl, unit_bound = PEAK_FP32_VALU_TFLOPS, "alu"
    ridge = peak_fl * 1e12 / (PEAK_HBM_GBS * 1e9)
    intensity = fl / max(by, 1.0)
    if intensity < ridge:
        ach = by / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(ach, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None}
    ach = fl / (ms * 1e-3) / 1e12
    return {"bound": unit_bound, "achieved": round(ach, 3), "peak": peak_fl, "unit": "TFLOP/s",
            "frac": round(ach / peak_fl, 4), "traffic": None}


def mfma_for(recs, precision, ms_per_step, iters):
    """Matrix-core utilisation of the V-cycle convolutions: the algorithmic
    flops (2 per MAC) of every matrix-core launch of the profiled solve
    (implicit-GEMM convolutions and fused steps) over their summed
    event-timed durations, against the dense peak of the operand type."""
    mm = [r for r in recs if r["name"].startswith(MATRIX_CORE_KERNELS)]
    fl = sum(r["flops_per_launch"] * r["launches"] for r in mm)
    ms = sum(r["total_ms"] for r in mm)
    if not mm or ms <= 0:
        return None
    peak = PEAK_BF16_TFLOPS if precision == "bf16" else PEAK_FP32_MFMA_TFLOPS
    ach = fl / (ms * 1e-3) / 1e12
    return {"kernels": "matrix-core convolutions (mconv_kernel, mconvz_kernel, mstep_kernel)",
            "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 5),
            "ms_per_step": round(ms / max(iters, 1), 4),
            "share_of_step": round(ms / max(iters, 1) / ms_per_step, 3)}


def run_leg(cfg, c, omega, h, f, blob, precision, steps, warmup):
    """Setup, warm up, then time one solve of `steps` iterations from u = 0;
    repeat it with per-launch HIP-event timing for the kernel breakdown."""
    import torch
    from paper_2606_30495_amd import Handle
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = Handle(c, omega, h, cfg.npml, blob, precision=precision, restart=cfg.restart)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    fd = torch.from_numpy(f).to("cuda")
    ud = torch.zeros_like(fd)
    if warmup > 0:
        H.solve(fd, ud, tol=cfg.tol, maxit=warmup, hist_cap=0)
    ud.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = H.solve(fd, ud, tol=cfg.tol, maxit=steps, hist_cap=0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    iters = info["iters"]
    ud.zero_()
    H.prof_enable(True)
    H.solve(fd, ud, tol=cfg.tol, maxit=steps, hist_cap=0)
    recs = H.prof_report()
    recs.sort(key=lambda r: -r["total_ms"])
    # live average duration of the dominant kernel: its recorded launches
    # replayed back to back between one HIP event pair on the handle's stream
    replay_ms, replay_n = H.prof_replay(recs[0]["name"], reps=3)
    recs[0]["event_pair_avg_ms"] = recs[0]["avg_ms"]
    recs[0]["avg_ms"] = replay_ms
    recs[0]["replayed_launches"] = replay_n
    H.prof_enable(False)
    H.close()
    return {"value": iters / el, "ms_per_step": el / max(iters, 1) * 1e3, "iters": iters,
            "info": info, "recs": recs, "setup_ms": setup_ms}


def solves_leg(precision, nrhs, seed=5):
    """Solve-to-tolerance throughput on the small workload (64^2 interior,
    8-cell PML, Gaussian bump, 3 levels 2/8/16): random-init weights never
    reach 1e-6, so this leg runs the same V-cycle with hand-set classical
    coefficients (shifted-Laplacian multigrid in McMg's tensor structure,
    synth.classical).  nrhs point sources at seeded random interior nodes,
    each solved from u = 0 to true relative residual 1e-6, one after another;
    latency = call to return."""
    import numpy as np
    import torch
    import synth
    from paper_2606_30495_amd import Handle
    cfg = synth.CONFIGS["bump64"]
    c, omega, h, _ = synth.make_problem(cfg)
    tens, feats = synth.shifted_laplacian(c, omega, h, cfg.npml, cfg.channels, cfg.nu1, cfg.nu2)
    blob = synth.pack_blob(cfg.dim, cfg.channels, cfg.nu1, cfg.nu2, tens)
    H = Handle(c, omega, h, cfg.npml, blob, precision=precision, restart=cfg.restart)
    for l, (a, s) in enumerate(feats, start=1):
        H.set_features(l, torch.from_numpy(a).cuda(), torch.from_numpy(s).cuda())
    rng = np.random.Generator(np.random.PCG64(seed))
    fs = [torch.from_numpy(synth.point_source(cfg.n, cfg.npml, tuple(rng.uniform(0.1, 0.9, 2)), 2)).cuda()
          for _ in range(nrhs)]
    u = torch.zeros_like(fs[0])
    H.solve(fs[0], u, tol=cfg.tol, maxit=cfg.maxit, hist_cap=0)   # warm-up
    lat, its, ok, worst = [], [], 0, 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in fs:
        u.zero_()
        t1 = time.perf_counter()
        info = H.solve(f, u, tol=cfg.tol, maxit=cfg.maxit, hist_cap=0)
        lat.append(time.perf_counter() - t1)
        its.append(info["iters"])
        ok += int(info["converged"])
        worst = max(worst, info["relres_true"])
    el = time.perf_counter() - t0
    H.close()
    lat = np.array(lat) * 1e3
    return {"workload": "bump64 (64^2 + 8-cell PML, 3 levels 2/8/16), classical coefficients",
            "precision": precision, "nrhs": nrhs, "solves_per_s": round(ok / el, 3),
            "iters_per_s": round(sum(its) / el, 2), "mean_iters": round(float(np.mean(its)), 2),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "converged": ok, "max_relres_true": worst}


def batched_leg(precision, iters):
    """The batched workload (64 independent 2D problems, sides drawn from
    {128, 256, 384, 512, 768}, high-contrast ellipses, 5 levels 2/8/16/32/64,
    random-init weights): `iters` FGMRES iterations of every problem in one
    engine (one launch per operation for all 64, captured tick replayed),
    against the same iterations one problem at a time through mcmg_solve.
    Random-init weights do not converge, so every problem runs exactly
    `iters` iterations in both forms and the results are bitwise equal."""
    import numpy as np
    import torch
    import synth
    from paper_2606_30495_amd import Handle, solve_batch
    cfg = synth.CONFIGS["ellipses64"]
    probs = synth.make_batch(cfg)
    tens = synth.make_weights(2, cfg.channels, cfg.nu1, cfg.nu2, cfg.weight_seed)
    blob = synth.pack_blob(2, cfg.channels, cfg.nu1, cfg.nu2, tens)
    t0 = time.perf_counter()
    hs = [Handle(p["c"], p["omega"], p["h"], cfg.npml, blob, precision=precision,
                 restart=cfg.restart) for p in probs]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    fs = [torch.from_numpy(p["f"]).cuda() for p in probs]
    us = [torch.zeros_like(f) for f in fs]
    solve_batch(hs, fs, us, tol=cfg.tol, maxit=2)           # warm-up (workspaces, tables)
    for u in us:
        u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, infos = solve_batch(hs, fs, us, tol=cfg.tol, maxit=iters)
    torch.cuda.synchronize()
    el_b = time.perf_counter() - t0
    nit = sum(i["iters"] for i in infos)
    ub = [u.clone() for u in us]
    for u in us:
        u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_its = 0
    for H, f, u in zip(hs, fs, us):
        seq_its += H.solve(f, u, tol=cfg.tol, maxit=iters, hist_cap=0)["iters"]
    torch.cuda.synchronize()
    el_s = time.perf_counter() - t0
    same = all(torch.equal(a, b) for a, b in zip(ub, us))
    for H in hs:
        H.close()
    sides = sorted(p["n"] for p in probs)
    return {"workload": "ellipses64: 64 2D problems, sides " +
                        "/".join(str(s) for s in sorted(set(sides))) +
                        " (+2x16 PML), 5 levels 2/8/16/32/64, random-init weights",
            "precision": precision, "problems": len(probs), "iters_each": iters,
            "unknowns_total": int(sum((s + 2 * cfg.npml) ** 2 for s in sides)),
            "iters_per_s": round(nit / el_b, 2), "ms_per_batched_iter": round(el_b / iters * 1e3, 3),
            "sequential_iters_per_s": round(seq_its / el_s, 2),
            "speedup_vs_sequential": round((nit / el_b) / (seq_its / el_s), 3),
            "bitwise_equal_to_sequential": bool(same), "setup_s": round(setup_s, 2)}


SERVE_SCALES = {
    # scaled trace of the default run: small sides so that the one-at-a-time
    # comparator finishes in about a minute
    "small": {"sides2d": (64, 96, 128), "sides3d": (24, 32), "maxit": SERVE_MAXIT},
    # the serving configuration's size classes (2D 256-2048, 3D 64-160); the
    # classical stand-in needs thousands of iterations at the larger sides,
    # so every right-hand side is capped
    "full": {"sides2d": (256, 512, 768, 1024, 1536, 2048), "sides3d": (64, 96, 128, 160),
             "maxit": 300},
}


def served_leg(nreq, rate, seed=3, scale="small"):
    """The serving workload, scaled to a short run: Poisson arrivals (rate
    requests/s, seeded) over 16 cached media (12 2D: bump / GRF / ellipses,
    sides 64-128 + 16-cell PML, the 6-level 2/8/16/32/64/64 model; 4 3D
    layered media, sides 24-32 + 12-cell PML, the 5-level 2/12/24/48/96
    model), 1-8 point-source right-hand sides per request, each solved to
    true relative residual 1e-6 with classical coefficients (random-init
    weights never converge).  Served: BF16 V-cycle convolutions through the
    continuous-batching server (HBM budget 200 GB), iteration cap 1000 for
    both paths.  Comparator: the plain
    FP32 path, one right-hand side at a time in arrival order, on the same
    trace in real time.  Latency = arrival to the request's last solution."""
    import numpy as np
    import torch
    import synth
    from paper_2606_30495_amd import Handle, Server
    sc = SERVE_SCALES[scale]
    maxit = sc["maxit"]
    media = synth.serve_media(seed, sides2d=sc["sides2d"], sides3d=sc["sides3d"])
    trace = synth.serve_trace(media, nreq, rate, seed)
    models = {2: synth.CONFIGS["grf1024"], 3: synth.CONFIGS["layered192"]}
    built = []
    for m in media:
        mc = models[m["dim"]]
        tens, feats = synth.shifted_laplacian(m["c"], m["omega"], m["h"], m["npml"], mc.channels,
                                              mc.nu1, mc.nu2)
        built.append((mc, synth.pack_blob(m["dim"], mc.channels, mc.nu1, mc.nu2, tens), feats))

    def handle(i, prec):
        m, (mc, blob, feats) = media[i], built[i]
        H = Handle(m["c"], m["omega"], m["h"], m["npml"], blob, precision=prec, restart=mc.restart)
        for l, (a, s) in enumerate(feats, start=1):
            H.set_features(l, torch.from_numpy(a).cuda(), torch.from_numpy(s).cuda())
        return H

    fs = [[torch.from_numpy(f).cuda() for f in r["fs"]] for r in trace]
    nrhs = sum(len(r["fs"]) for r in trace)
    # served (BF16)
    srv = Server(hbm_budget=200 << 30)
    mids = [srv.add_handle(handle(i, "bf16")) for i in range(len(media))]
    warm = {}
    for i, m in enumerate(media):          # one warm-up solve per medium
        warm.setdefault(m["dim"], []).append(i)
    for dim, idx in warm.items():
        i = idx[0]
        f = torch.from_numpy(synth.point_source(media[i]["n"], media[i]["npml"],
                                                (0.5,) * dim, dim)).cuda()
        torch.cuda.synchronize()
        srv.submit(mids[i], [f], [torch.zeros_like(f)], maxit=min(maxit, 50))
    torch.cuda.synchronize()
    got = 0
    while got < len(warm):
        got += len(srv.poll(64, wait_ms=100))
    us = [[torch.zeros_like(f) for f in r] for r in fs]
    torch.cuda.synchronize()
    done, i = {}, 0
    rid_of = {}
    t0 = time.perf_counter()
    t_note = t0
    while len(done) < nreq:
        now = time.perf_counter() - t0
        while i < nreq and trace[i]["t"] <= now:
            rid_of[srv.submit(mids[trace[i]["medium"]], fs[i], us[i], tol=1e-6, maxit=maxit)] = i
            i += 1
        wait_ms = 20 if i >= nreq else max(0, min(20, int((trace[i]["t"] - now) * 1e3)))
        for c in srv.poll(64, wait_ms=wait_ms):
            done[rid_of[c["req_id"]]] = c
        if time.perf_counter() - t_note > 20.0:     # long traces: a line every 20 s
            t_note = time.perf_counter()
            progress(f"served: {len(done)} of {nreq} requests finished")
    t_end = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    lat_s = np.array([done[k]["latency_s"] for k in range(nreq)]) * 1e3
    ok_s = sum(done[k]["nrhs"] for k in range(nreq) if done[k]["status"] == 0)
    worst_s = max(done[k]["relres_max"] for k in range(nreq))
    its_s = sum(done[k]["iters_total"] for k in range(nreq))
    # plain FP32, one right-hand side at a time, same arrivals
    hs = [handle(i, "fp32") for i in range(len(media))]
    u = {k: torch.zeros_like(fs[k][0]) for k in range(nreq)}
    for dim, idx in warm.items():
        j = idx[0]
        f = torch.from_numpy(synth.point_source(media[j]["n"], media[j]["npml"], (0.5,) * dim, dim)).cuda()
        hs[j].solve(f, torch.zeros_like(f), tol=1e-6, maxit=min(maxit, 50), hist_cap=0)
    torch.cuda.synchronize()
    lat_p, ok_p, its_p, worst_p = [], 0, 0, 0.0
    t0 = time.perf_counter()
    t_note = t0
    for k, r in enumerate(trace):
        if time.perf_counter() - t_note > 20.0:
            t_note = time.perf_counter()
            progress(f"one at a time: request {k} of {nreq}")
        now = time.perf_counter() - t0
        if now < r["t"]:
            time.sleep(r["t"] - now)
        for f in fs[k]:
            u[k].zero_()
            info = hs[r["medium"]].solve(f, u[k], tol=1e-6, maxit=maxit, hist_cap=0)
            ok_p += int(info["converged"])
            its_p += info["iters"]
            worst_p = max(worst_p, info["relres_true"])
        lat_p.append(time.perf_counter() - t0 - r["t"])
    t_end_p = time.perf_counter() - t0
    for H in hs:
        H.close()
    lat_p = np.array(lat_p) * 1e3
    s2, s3 = sc["sides2d"], sc["sides3d"]
    return {"workload": f"serve: {nreq} Poisson requests at {rate}/s (seed {seed}) over 16 cached "
                        f"media (12 2D sides {s2[0]}-{s2[-1]}, 4 3D sides {s3[0]}-{s3[-1]}), "
                        f"1-8 rhs each, classical coefficients, tol 1e-6, cap {maxit} iterations",
            "rhs": nrhs, "sides": [media[i]["n"] for i in range(len(media))],
            "served_bf16": {"solves_per_s": round(ok_s / t_end, 2), "converged": ok_s,
                            "iters_per_s": round(its_s / t_end, 1),
                            "p50_ms": round(float(np.percentile(lat_s, 50)), 2),
                            "p99_ms": round(float(np.percentile(lat_s, 99)), 2),
                            "max_relres_true": worst_s, "inflight_peak": st["inflight_peak"],
                            "bytes_peak": st["bytes_peak"], "ticks": st["ticks"],
                            "rebuilds": st["rebuilds"]},
            "plain_fp32_one_at_a_time": {"solves_per_s": round(ok_p / t_end_p, 2), "converged": ok_p,
                                         "iters_per_s": round(its_p / t_end_p, 1),
                                         "p50_ms": round(float(np.percentile(lat_p, 50)), 2),
                                         "p99_ms": round(float(np.percentile(lat_p, 99)), 2),
                                         "max_relres_true": worst_p},
            "speedup_solves_per_s": round((ok_s / t_end) / max(ok_p / t_end_p, 1e-12), 3)}


def traffic_for(kernel):
    """Counter-measured HBM bytes per launch of `kernel` from the committed
    rocprofv3 summaries profiles/traffic*.md (FETCH_SIZE + WRITE_SIZE, scaled
    by the copy-kernel calibration); None when absent or when the kernel's
    source changed since."""
    import glob
    import hashlib
    import re
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic*.md"))):
        m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
        if not m:
            continue
        try:
            table = json.loads(m.group(1))
        except ValueError:
            continue
        ent = table.get("kernels", {}).get(kernel)
        if not ent:
            continue
        src = os.path.join(ROOT, ent["source"])
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != ent["sha256"]:
            return None
        return ent["bytes_per_launch"]
    return None


def _host_cpu():
    """CPU model name and logical CPU count of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(cfg, iters, side):
    """The FP64 oracle on the host cores, on a bounded sample of the workload.

    2D: setup + `iters` FGMRES iterations of the workload itself.  3D: one
    oracle V-cycle at 216^3 takes minutes, so the sample is the same model,
    medium recipe, ppw, PML and source at a reduced interior side `side`:
    setup + `iters` FGMRES iterations, scaled to the full grid by node count
    (every step of an iteration is linear in the node count) and labelled
    extrapolated."""
    import dataclasses
    import numpy as np
    import synth
    from oracle import helmholtz, krylov, mcmg
    try:
        import threadpoolctl
        blas = [p.get("num_threads", 1) for p in threadpoolctl.threadpool_info()
                if p.get("user_api") == "blas"]
        threads = max(blas) if blas else 1
    except Exception:
        threads = 1
    scfg = cfg if cfg.dim == 2 else dataclasses.replace(cfg, n=side)
    c, omega, h, f = synth.make_problem(scfg)
    tens = synth.make_weights(scfg.dim, scfg.channels, scfg.nu1, scfg.nu2, scfg.weight_seed)
    t0 = time.perf_counter()
    op = helmholtz.setup_operator(c, omega, h, scfg.npml)
    W = mcmg.Weights(scfg.dim, scfg.channels, scfg.nu1, scfg.nu2, tens)
    M = mcmg.Preconditioner(W, np.sqrt(op["k2"]), h)
    t1 = time.perf_counter()
    _, info = krylov.fgmres(lambda x: helmholtz.apply(op, x), M, f, m=scfg.restart,
                            tol=scfg.tol, maxit=iters)
    t2 = time.perf_counter()
    scale = (scfg.n_ext / cfg.n_ext) ** cfg.dim
    rate = info["iters"] / (t2 - t1) * scale
    model, ncpu = _host_cpu()
    if scfg is cfg:
        what = f"{cfg.name}: oracle setup ({t1 - t0:.1f} s) then {info['iters']} FGMRES iterations " \
               f"({t2 - t1:.1f} s) from u=0"
    else:
        what = (f"{cfg.name} model and medium recipe at {scfg.n}^3 interior + {scfg.npml}-cell PML "
                f"({scfg.n_ext}^3 nodes): oracle setup ({t1 - t0:.1f} s) then {info['iters']} "
                f"FGMRES iteration(s) ({t2 - t1:.1f} s) from u=0, extrapolated to {cfg.n_ext}^3 "
                f"by node count (x{1 / scale:.2f})")
    return {"value": round(rate, 6), "unit": "iters/s", "cores": threads, "kind": "oracle",
            "extrapolated": scfg is not cfg,
            "sample": f"{what}; BLAS threads {threads}, NumPy elementwise work single-threaded; "
                      f"host {model}, {ncpu} logical CPUs"}


def born_leg(iters, precision="bf16"):
    """Born-series form (Born+McMg, u <- u + MG(G(f - A_per u)), G by FFT) on
    the 2D 1024^2 GRF medium with a 16-cell sponge layer, run for `iters`
    steps from u = 0, plus the FFT passes' HIP-event timing.  The iteration
    count is fixed (random-init weights), so the leg measures the cost per
    Born step."""
    import torch
    import synth
    from paper_2606_30495_amd import Handle
    cfg = synth.CONFIGS["grf1024"]
    c, omega, h, f = synth.make_problem(cfg)
    tens = synth.make_weights(cfg.dim, cfg.channels, cfg.nu1, cfg.nu2, cfg.weight_seed)
    blob = synth.pack_blob(cfg.dim, cfg.channels, cfg.nu1, cfg.nu2, tens)
    H = Handle(c, omega, h, cfg.npml, blob, precision=precision, restart=2, absorber="sponge")
    H.born_setup()
    k0sq, eps = H.born_params()
    fd = torch.from_numpy(f).to("cuda")
    ud = torch.zeros_like(fd)
    out = {"workload": f"{cfg.name} with a {cfg.npml}-cell sponge layer, periodic Born operator",
           "precision": precision, "k0sq": k0sq, "eps": eps}
    H.born_solve(fd, ud, method="mcmg", tol=1e-300, maxit=2, hist_cap=0)   # warm-up
    ud.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = H.born_solve(fd, ud, method="mcmg", tol=1e-300, maxit=iters, hist_cap=0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["mcmg"] = {"iters_per_s": round(info["iters"] / el, 3),
                   "ms_per_step": round(el / max(info["iters"], 1) * 1e3, 4)}
    ud.zero_()
    H.prof_enable(True)
    H.born_solve(fd, ud, method="mcmg", tol=1e-300, maxit=iters, hist_cap=0)
    recs = H.prof_report()
    fft = []
    for r in sorted(recs, key=lambda r: r["name"]):
        if not r["name"].startswith("fft_kernel"):
            continue
        replay_ms, _ = H.prof_replay(r["name"], reps=3)
        gbs = r["bytes_per_launch"] / (replay_ms * 1e-3) / 1e9
        fft.append({"kernel": r["name"], "launches_per_step": round(r["launches"] / iters, 2),
                    "avg_launch_us": round(replay_ms * 1e3, 3), "achieved_gbs": round(gbs, 1),
                    "frac_hbm": round(gbs / PEAK_HBM_GBS, 4),
                    "bytes_per_launch": r["bytes_per_launch"]})
    H.prof_enable(False)
    out["fft"] = fft
    tot = sum(r["total_ms"] for r in recs)
    out["fft_share_of_step"] = round(sum(r["total_ms"] for r in recs
                                         if r["name"].startswith("fft_kernel")) / max(tot, 1e-9), 4)
    H.close()
    return out


def trained_leg(steps, nrhs, seed=7):
    """Training (Eq. loss_fun, the residual loss on N(0, I) residuals) and the
    trained preconditioner deployed on the small workload.

    The 64^2 bump model (3 levels 2/8/16, nu 2/2) starts from the seeded
    random initialisation and is trained with Adam on four bump media with
    seeded +-10 % speed perturbations (batch 2: the parameter-owning medium
    and one of the others in turn), learning rate 1e-2 / 3.3e-3 / 1e-3 /
    3.3e-4 over the first 20 % / next 30 % / next 30 % / last 20 % of `steps`
    (a fixed count, so the run is deterministic: the weight gradients are
    fixed-order reductions; starting at 3e-2 the loss settled near 0.5 and
    the trained V-cycle did not reach 1e-6 within 2500 iterations).  The absorbing layer is the sponge of Sec. 2.1 (the
    setting of the paper's main text).  The trained weights are then
    deployed on the bump64 medium itself (not one of the training media)
    and `nrhs` seeded point sources are solved to true relative residual
    1e-6 (FGMRES(30), cap 2500) in both precisions, next to the classical
    stand-in coefficients on the same problem."""
    import numpy as np
    import torch
    import synth
    from paper_2606_30495_amd import Handle, train_step
    cfg = synth.CONFIGS["bump64"]
    tens = synth.make_weights(cfg.dim, cfg.channels, cfg.nu1, cfg.nu2, 0)
    blob = synth.pack_blob(cfg.dim, cfg.channels, cfg.nu1, cfg.nu2, tens)
    h = 1.0 / cfg.n
    rng = np.random.Generator(np.random.PCG64(seed))
    hs = []
    for _ in range(4):
        c = synth.medium_bump(cfg.n, cfg.dim) * rng.uniform(0.9, 1.1, size=(cfg.n,) * cfg.dim)
        hs.append(Handle(c, synth.omega_for_ppw(c, cfg.ppw, h), h, cfg.npml, blob,
                         absorber="sponge"))
    shape = hs[0].ext_shape
    gen = torch.Generator(device="cuda").manual_seed(seed)

    def draw():
        return [torch.complex(torch.randn(shape, generator=gen, device="cuda", dtype=torch.float64),
                              torch.randn(shape, generator=gen, device="cuda", dtype=torch.float64))
                for _ in range(2)]

    def lr_at(k):
        f = k / max(steps, 1)
        return 1e-2 if f < 0.2 else 1e-2 / 3 if f < 0.5 else 1e-3 if f < 0.8 else 1e-3 / 3

    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        losses.append(train_step([hs[0], hs[1 + k % 3]], draw(), lr=lr_at(k)))
        if (k + 1) % 2500 == 0:
            progress(f"training: step {k + 1} of {steps}, loss {float(np.mean(losses[-100:])):.4f}")
    k = steps
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    trained = hs[0].export_blob()
    for H in hs:
        H.close()

    c, omega, hh, _ = synth.make_problem(cfg)
    srng = np.random.Generator(np.random.PCG64(5))
    fs = [torch.from_numpy(synth.point_source(cfg.n, cfg.npml, tuple(srng.uniform(0.1, 0.9, 2)), 2)).cuda()
          for _ in range(nrhs)]
    ctens, cfeats = synth.shifted_laplacian(c, omega, hh, cfg.npml, cfg.channels, cfg.nu1, cfg.nu2)
    cblob = synth.pack_blob(cfg.dim, cfg.channels, cfg.nu1, cfg.nu2, ctens)

    def solves(b, prec, feats=None, n=None):
        H = Handle(c, omega, hh, cfg.npml, b, precision=prec, restart=cfg.restart, absorber="sponge")
        if feats is not None:
            for l, (a, s_) in enumerate(feats, start=1):
                H.set_features(l, torch.from_numpy(a).cuda(), torch.from_numpy(s_).cuda())
        u = torch.zeros_like(fs[0])
        H.solve(fs[0], u, tol=cfg.tol, maxit=20, hist_cap=0)          # warm-up
        lat, its, ok = [], [], 0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for f in fs[:n]:
            u.zero_()
            t2 = time.perf_counter()
            info = H.solve(f, u, tol=cfg.tol, maxit=2500, hist_cap=0)
            lat.append(time.perf_counter() - t2)
            its.append(info["iters"])
            ok += int(info["converged"])
        tot = time.perf_counter() - t1
        H.close()
        lat = np.array(lat) * 1e3
        return {"precision": prec, "solves_per_s": round(ok / tot, 3), "converged": ok,
                "mean_iters": round(float(np.mean(its)), 1),
                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3)}

    return {"workload": "bump64 medium (64^2 + 8-cell sponge layer, 3 levels 2/8/16), "
                        f"{nrhs} point sources to 1e-6; trained on 4 perturbed bump media",
            "train": {"steps": k, "seconds": round(el, 2), "steps_per_s": round(k / el, 2),
                      "batch": 2, "loss_first": round(losses[0], 4),
                      "loss_last20": round(float(np.mean(losses[-20:])), 4)},
            "trained": [solves(trained, p) for p in ("fp32", "bf16")],
            "random_init": solves(blob, "fp32", n=2),
            "classical": [solves(cblob, p, cfeats) for p in ("fp32", "bf16")]}


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload_name(cfg):
    side = "x".join([str(cfg.n_ext)] * cfg.dim)
    return (f"{cfg.name}: {cfg.dim}D {cfg.n}^{cfg.dim} interior + {cfg.npml}-cell PML ({side}), "
            f"{cfg.levels} levels {'/'.join(str(c) for c in cfg.channels)}, FGMRES({cfg.restart})")


def leg_summary(leg):
    return {"value": round(leg["value"], 3), "ms_per_step": round(leg["ms_per_step"], 4),
            "relres_true": leg["info"]["relres_true"], "dominant_kernel": leg["recs"][0]["name"]}


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(independent solves shard across GPUs without communication, one process "
              "per GPU)", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth

    cfg = synth.CONFIGS[a.config]
    c, omega, h, f = synth.make_problem(cfg)
    tens = synth.make_weights(cfg.dim, cfg.channels, cfg.nu1, cfg.nu2, cfg.weight_seed)
    blob = synth.pack_blob(cfg.dim, cfg.channels, cfg.nu1, cfg.nu2, tens)

    head = run_leg(cfg, c, omega, h, f, blob, a.precision, a.steps, a.warmup)
    progress(f"{cfg.name} {a.precision} leg: {head['value']:.1f} iters/s")
    other = "fp32" if a.precision == "bf16" else "bf16"
    cmp_leg = None if a.single else run_leg(cfg, c, omega, h, f, blob, other, a.steps, a.warmup)
    if cmp_leg is not None:
        progress(f"{cfg.name} {other} leg: {cmp_leg['value']:.1f} iters/s")
    recs = head["recs"]
    dom = recs[0]
    roof = roofline_for(dom, a.precision)
    roof["traffic"] = traffic_for(dom["name"])
    roof["kernel"] = dom["name"]
    roof["launches_per_step"] = round(dom["launches"] / max(head["iters"], 1), 2)
    roof["avg_launch_us"] = round(dom["avg_ms"] * 1e3, 3)
    line = {
        "metric": "FGMRES+V-cycle iters/s (solves/s to rel-res 1e-6; p50/p99 solve latency)",
        "value": round(head["value"], 3), "unit": "iters/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if a.precision == "fp32" else "bf16",
        "data": "synthetic (seeded medium, random-init weights N(0,1/fan_in) seed 0)",
        "config": {"workload": workload_name(cfg), "dim": cfg.dim, "n_interior": cfg.n,
                   "npml": cfg.npml, "n_ext": cfg.n_ext, "levels": cfg.levels,
                   "channels": list(cfg.channels), "nu": [cfg.nu1[0], cfg.nu2[0]],
                   "restart": cfg.restart, "precision": a.precision, "outer": "f64"},
        "solve": {"iters": head["iters"], "relres_true": head["info"]["relres_true"],
                  "converged": head["info"]["converged"], "setup_ms": round(head["setup_ms"], 2)},
        "roofline": roof,
        "mfma": mfma_for(recs, a.precision, head["ms_per_step"], head["iters"]),
        "kernels": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
                    for r in recs[:16]],
    }
    if cmp_leg is not None:
        line["compare"] = dict(precision=other, **leg_summary(cmp_leg))
    if a.grf_steps > 0 and cfg.name != "grf1024":
        g = synth.CONFIGS["grf1024"]
        gc, gomega, gh, gf = synth.make_problem(g)
        gt = synth.make_weights(g.dim, g.channels, g.nu1, g.nu2, g.weight_seed)
        gb = synth.pack_blob(g.dim, g.channels, g.nu1, g.nu2, gt)
        line["grf1024"] = {"workload": workload_name(g)}
        for prec in ("fp32", "bf16"):
            leg = run_leg(g, gc, gomega, gh, gf, gb, prec, a.grf_steps, a.warmup)
            line["grf1024"][prec] = leg_summary(leg)
        progress("grf1024 legs done")
    if a.solves > 0:
        line["solves"] = [solves_leg(p, a.solves) for p in ("bf16", "fp32")]
        progress("solve-to-tolerance legs done")
    if a.batched_iters > 0:
        line["batched"] = batched_leg("bf16", a.batched_iters)
        progress("batched leg done")
    if a.serve_requests > 0:
        line["served"] = served_leg(a.serve_requests, a.serve_rate, scale=a.serve_scale)
        progress("served leg done")
    if a.born_iters > 0:
        line["born"] = born_leg(a.born_iters)
        progress("Born leg done")
    if a.train_steps > 0:
        line["trained"] = trained_leg(a.train_steps, a.trained_rhs)
        progress("training leg done")
    if not a.no_cpu:
        progress("CPU oracle baseline ...")
        line["cpu_baseline"] = cpu_baseline(cfg, a.cpu_iters, a.cpu_side)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
