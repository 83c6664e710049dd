"""Summaries of rocprofv3 CSV output (kernel stats and PMC counters).

    python3 -m paper_2606_30495_amd.profsum stats <kernel_stats.csv> [top]
    python3 -m paper_2606_30495_amd.profsum traffic --fetch <dir> --write <dir>
        --cal-fetch <dir> --cal-write <dir> --cal-bytes B
        [--kernel NAME=SOURCE ...] [--src NAME_PREFIX=SOURCE ...]

    python3 -m paper_2606_30495_amd.profsum periter <kernel_trace.csv> <marker kernel> [n]
    python3 -m paper_2606_30495_amd.profsum mfma <dir> [prefix ...]
    python3 -m paper_2606_30495_amd.profsum counters <dir> [prefix ...]

`mfma` summarises a run with `--pmc MfmaUtil MfmaFlopsBF16` (or
SQ_INSTS_VALU_MFMA_MOPS_F32, counted in units of 512 flops) per kernel name
(those starting with one of the prefixes, default mconv_kernel, mconvz_kernel and
mstep_kernel): dispatches, mean matrix-core flops per dispatch as counted
by the hardware, mean dispatch duration, flops over duration, and
MfmaUtil, the matrix-core busy cycles over the busy cycles of all SIMDs.

`periter` splits a kernel trace at the dispatches of a marker kernel
launched once per iteration (the last n + 1 of them, default n = 10) and
prints, per kernel name and grid size (blocks), the mean time per
iteration, the launches per iteration and the mean launch duration.

`counters` prints, per kernel name (those starting with one of the
prefixes, default all), the dispatch count and the mean per dispatch of
every counter the run collected.

`traffic` averages FETCH_SIZE and WRITE_SIZE (KiB per dispatch) per kernel
name, scales each by the calibration copy kernel's bytes-moved / counter
ratio and prints a Markdown summary with a JSON block
{"kernels": {name: {bytes_per_launch, fetch_bytes, write_bytes, source,
sha256}}} that bench.py reads (it ignores an entry whose source changed).
"""
import csv
import glob
import hashlib
import json
import os
import re
import sys


def short(name):
    for p in ("void ", "mcmg::(anonymous namespace)::"):
        name = name.replace(p, "")
    name = re.sub(r"\(.*$", "", name)
    return name.strip()


def stats(path, top=30):
    rows = list(csv.DictReader(open(path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    out.append(f"\ntotal kernel time {total / 1e6:.3f} ms over {sum(int(r['Calls']) for r in rows)} dispatches")
    return "\n".join(out)


def counter_means(d, counter):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    acc = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            if r.get("Counter_Name") != counter:
                continue
            k = short(r["Kernel_Name"])
            acc.setdefault(k, []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}


def traffic(args):
    kv = dict(a.split("=", 1) for a in args["kernel"])
    prefixes = [a.split("=", 1) for a in args["src"]]
    fetch, nf = counter_means(args["fetch"], "FETCH_SIZE")
    write, nw = counter_means(args["write"], "WRITE_SIZE")
    cf, _ = counter_means(args["cal_fetch"], "FETCH_SIZE")
    cw, _ = counter_means(args["cal_write"], "WRITE_SIZE")
    cal_bytes = float(args["cal_bytes"])
    ckf = max(cf.items(), key=lambda x: x[1])
    ckw = max(cw.items(), key=lambda x: x[1])
    sf = cal_bytes / (ckf[1] * 1024.0)
    sw = cal_bytes / (ckw[1] * 1024.0)
    lines = [f"copy calibration: `{ckf[0]}` moves {cal_bytes:.0f} B per launch; FETCH_SIZE reads "
             f"{ckf[1]:.0f} KiB (scale {sf:.4f}), WRITE_SIZE reads {ckw[1]:.0f} KiB (scale {sw:.4f})", ""]
    table = {"kernels": {}}
    lines.append("| kernel | dispatches | FETCH KiB | WRITE KiB | scaled bytes/launch |")
    lines.append("|---|---|---|---|---|")
    for k in sorted(fetch, key=lambda x: -fetch[x] * nf[x])[:40]:
        fb = fetch[k] * 1024.0 * sf
        wb = write.get(k, 0.0) * 1024.0 * sw
        lines.append(f"| `{k}` | {nf[k]} | {fetch[k]:.1f} | {write.get(k, 0.0):.1f} | {fb + wb:.4e} |")
        src = kv.get(k)
        if src is None:
            for pre, path in prefixes:
                if k.startswith(pre):
                    src = path
                    break
        if src is not None:
            sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
            table["kernels"][k] = {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                                   "source": os.path.relpath(src), "sha256": sha}
    lines.append("")
    lines.append("```json")
    lines.append(json.dumps(table, indent=1))
    lines.append("```")
    return "\n".join(lines)


def replay_run(trace, kernel):
    """Longest run of consecutive dispatches of `kernel` in a kernel trace
    (the back-to-back replay bench.py issues for its dominant kernel):
    dispatch count, mean kernel duration and mean start-to-start period."""
    rows = list(csv.DictReader(open(trace)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    best, cur = [], []
    for r in rows:
        if short(r["Kernel_Name"]) == kernel:
            cur.append(r)
        else:
            if len(cur) > len(best):
                best = cur
            cur = []
    if len(cur) > len(best):
        best = cur
    if not best:
        return f"no dispatch of `{kernel}`"
    dur = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in best]
    span = int(best[-1]["End_Timestamp"]) - int(best[0]["Start_Timestamp"])
    return (f"`{kernel}`: longest back-to-back run {len(best)} dispatches, mean kernel duration "
            f"{sum(dur) / len(dur) / 1e3:.3f} us, mean start-to-start {span / len(best) / 1e3:.3f} us")


def per_iteration(trace, marker, n=10):
    rows = list(csv.DictReader(open(trace)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    idx = [i for i, r in enumerate(rows) if short(r["Kernel_Name"]) == marker]
    if len(idx) < 2:
        return f"fewer than two dispatches of `{marker}`"
    seg = idx[-(n + 1):]
    n = len(seg) - 1
    tot, cnt = {}, {}
    for a, b in zip(seg[:-1], seg[1:]):
        for r in rows[a + 1:b + 1]:
            blocks = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]) // max(
                1, int(r["Workgroup_Size_X"]) * int(r["Workgroup_Size_Y"]) * int(r["Workgroup_Size_Z"]))
            k = (short(r["Kernel_Name"]), blocks)
            tot[k] = tot.get(k, 0) + int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            cnt[k] = cnt.get(k, 0) + 1
    wall = int(rows[seg[-1]]["End_Timestamp"]) - int(rows[seg[0]]["End_Timestamp"])
    out = [f"{n} iterations (from one `{marker}` to the next): kernel time "
           f"{sum(tot.values()) / n / 1e3:.1f} us per iteration, wall {wall / n / 1e3:.1f} us", "",
           "| kernel | blocks | us per iteration | launches per iteration | avg us |", "|---|---|---|---|---|"]
    for k in sorted(tot, key=lambda k: -tot[k]):
        out.append(f"| `{k[0]}` | {k[1]} | {tot[k] / n / 1e3:.1f} | {cnt[k] / n:.1f} | {tot[k] / cnt[k] / 1e3:.1f} |")
    return "\n".join(out)


def counters(d, prefixes):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    per = {}
    names = []
    for f in files:
        for r in csv.DictReader(open(f)):
            k = short(r["Kernel_Name"])
            if prefixes and not k.startswith(tuple(prefixes)):
                continue
            c = r["Counter_Name"]
            if c not in names:
                names.append(c)
            per.setdefault(k, {}).setdefault(c, {})
            disp = r.get("Dispatch_Id", r.get("Correlation_Id", ""))
            per[k][c][disp] = per[k][c].get(disp, 0.0) + float(r["Counter_Value"])
    out = ["| kernel | dispatches | " + " | ".join(names) + " |",
           "|---|---|" + "---|" * len(names)]
    rows = []
    for k, cs in per.items():
        n = max(len(v) for v in cs.values())
        means = [sum(cs[c].values()) / max(len(cs[c]), 1) if c in cs else float("nan") for c in names]
        rows.append((k, n, means))
    rows.sort(key=lambda t: -t[1])
    for k, n, means in rows:
        out.append(f"| `{k}` | {n} | " + " | ".join(f"{m:.4g}" for m in means) + " |")
    return "\n".join(out)


# matrix-core flops per dispatch: a derived metric, or the MOPS counter (in
# units of 512 flops)
FLOP_COUNTERS = {"MfmaFlopsBF16": 1.0, "MfmaFlopsF32": 1.0,
                 "SQ_INSTS_VALU_MFMA_MOPS_BF16": 512.0, "SQ_INSTS_VALU_MFMA_MOPS_F32": 512.0}


def hw_flops(v):
    return sum(v[c] * f for c, f in FLOP_COUNTERS.items() if c in v)


def mfma(d, prefixes):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    per = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            k = short(r["Kernel_Name"])
            if not k.startswith(tuple(prefixes)):
                continue
            e = per.setdefault(k, {})
            disp = e.setdefault(r["Dispatch_Id"], {"dur": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
            disp[r["Counter_Name"]] = float(r["Counter_Value"])
    out = ["| kernel | dispatches | hw MFMA flops / dispatch | mean duration us | TFLOP/s (hw flops / duration) | MfmaUtil % |",
           "|---|---|---|---|---|---|"]
    tot_fl = tot_ns = 0.0
    rows = []
    for k, e in per.items():
        ds = [v for v in e.values() if "MfmaUtil" in v and any(c in v for c in FLOP_COUNTERS)]
        if not ds:
            continue
        fl = sum(hw_flops(v) for v in ds)
        ns = sum(v["dur"] for v in ds)
        util = sum(v["MfmaUtil"] for v in ds) / len(ds)
        tot_fl += fl
        tot_ns += ns
        rows.append((ns, f"| `{k}` | {len(ds)} | {fl / len(ds):.4g} | {ns / len(ds) / 1e3:.2f} | "
                         f"{fl / max(ns, 1) / 1e3:.1f} | {util:.2f} |"))
    out += [r for _, r in sorted(rows, reverse=True)]
    out.append(f"\nall listed kernels: {tot_fl / max(tot_ns, 1) / 1e3:.1f} TFLOP/s of matrix-core work "
               f"over their summed durations")
    return "\n".join(out)


def main(argv):
    if argv[0] == "mfma":
        print(mfma(argv[1], argv[2:] or ["mconv_kernel", "mconvz_kernel", "mstep_kernel"]))
        return
    if argv[0] == "counters":
        print(counters(argv[1], argv[2:]))
        return
    if argv[0] == "periter":
        print(per_iteration(argv[1], argv[2], int(argv[3]) if len(argv) > 3 else 10))
        return
    if argv[0] == "replay":
        print(replay_run(argv[1], argv[2]))
        return
    if argv[0] == "stats":
        print(stats(argv[1], int(argv[2]) if len(argv) > 2 else 30))
        return
    if argv[0] == "traffic":
        args = {"kernel": [], "src": []}
        i = 1
        while i < len(argv):
            key = argv[i].lstrip("-").replace("-", "_")
            if key in ("kernel", "src"):
                args[key].append(argv[i + 1])
            else:
                args[key] = argv[i + 1]
            i += 2
        print(traffic(args))
        return
    raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
