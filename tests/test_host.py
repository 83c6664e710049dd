"""Host-side logic on the CPU: the rocprofv3 summary tools that the committed
profiles come from, the bench's stale-counter check, and the seeded input
generators (determinism, shapes, the level geometry of the workloads)."""
import csv
import hashlib
import json
import os

import numpy as np
import pytest

import synth
from paper_2606_30495_amd import profsum


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def _counters(d, counter, values):
    """A counter_collection.csv holding one row per (kernel, value)."""
    rows = [[k, counter, v] for k, vs in values.items() for v in vs]
    _write_csv(os.path.join(d, "run", "run_counter_collection.csv"),
               ["Kernel_Name", "Counter_Name", "Counter_Value"], rows)


def test_short_kernel_names():
    assert profsum.short("void mcmg::(anonymous namespace)::helm_kernel<2, float, 0>(mcmg::HArgs, int)") \
        == "helm_kernel<2, float, 0>"
    assert profsum.short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_per_iteration_breakdown(tmp_path):
    """profsum periter splits a kernel trace at a once-per-iteration marker
    kernel: the kernels after one marker up to and including the next form
    an iteration, keyed by name and grid size (blocks)."""
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Grid_Size_Y",
           "Grid_Size_Z", "Workgroup_Size_X", "Workgroup_Size_Y", "Workgroup_Size_Z"]
    rows, t = [], 0

    def k(name, dur_us, blocks):                  # timestamps in ns
        nonlocal t
        rows.append([name, t, t + dur_us * 1000, blocks * 256, 1, 1, 256, 1, 1])
        t += dur_us * 1000 + 5000

    k("void warm(int)", 999, 1)                   # before the first marker: not counted
    for it in range(3):
        k("void mcmg::(anonymous namespace)::mark<1>(int)", 10, 4)
        k("void a(int)", 100 + it, 8)
        k("void a(int)", 50, 16)                  # same name, other grid: its own row
        k("void b(int)", 20, 8)
    k("void mcmg::(anonymous namespace)::mark<1>(int)", 10, 4)
    path = tmp_path / "trace.csv"
    _write_csv(str(path), hdr, rows)
    out = profsum.per_iteration(str(path), "mark<1>", 3)
    lines = {ln.split("|")[1].strip().strip("`") + "/" + ln.split("|")[2].strip(): ln
             for ln in out.splitlines() if ln.startswith("| `")}
    # us per iteration: a with 8 blocks ran 100, 101 and 102 us in the three
    # iterations; with 16 blocks 50 us each; launches per iteration: 1
    assert float(lines["a/8"].split("|")[3]) == pytest.approx(101.0)
    assert float(lines["a/16"].split("|")[3]) == pytest.approx(50.0)
    assert float(lines["b/8"].split("|")[5]) == pytest.approx(20.0)
    assert float(lines["mark<1>/4"].split("|")[4]) == pytest.approx(1.0)
    assert "warm" not in out


def test_traffic_scales_by_the_copy_calibration(tmp_path):
    """Bytes per launch = FETCH_SIZE KiB x 1024 x (copy bytes / copy FETCH
    bytes) + the same for WRITE_SIZE; the JSON table records the source's
    sha256.  Counter values are averaged over a kernel's dispatches."""
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    _counters(tmp_path / "f", "FETCH_SIZE", {"void k_a<1>(int)": [100.0, 300.0], "k_b": [10.0]})
    _counters(tmp_path / "w", "WRITE_SIZE", {"void k_a<1>(int)": [50.0, 50.0], "k_b": [0.0]})
    # a 1 MiB copy whose counters read half (fetch) and all (write) of it
    _counters(tmp_path / "cf", "FETCH_SIZE", {"__amd_rocclr_copyBuffer": [512.0]})
    _counters(tmp_path / "cw", "WRITE_SIZE", {"__amd_rocclr_copyBuffer": [1024.0]})
    out = profsum.traffic({"kernel": [], "src": [f"k_a={src}"], "fetch": str(tmp_path / "f"),
                           "write": str(tmp_path / "w"), "cal_fetch": str(tmp_path / "cf"),
                           "cal_write": str(tmp_path / "cw"), "cal_bytes": str(1 << 20)})
    table = json.loads(out.split("```json\n")[1].split("\n```")[0])
    ent = table["kernels"]["k_a<1>"]
    assert ent["fetch_bytes"] == pytest.approx(200.0 * 1024 * 2.0)
    assert ent["write_bytes"] == pytest.approx(50.0 * 1024 * 1.0)
    assert ent["bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2.0 + 50.0 * 1024)
    assert ent["sha256"] == hashlib.sha256(src.read_bytes()).hexdigest()
    assert "k_b" not in table["kernels"]          # no source named for it


def test_bench_drops_counters_of_a_changed_source(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "k.hip"
    src.write_text("v1\n")
    table = {"kernels": {"k_a<1>": {"bytes_per_launch": 1234.0, "source": "k.hip",
                                    "sha256": hashlib.sha256(b"v1\n").hexdigest()}}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_x.md").write_text(
        "# t\n\n```json\n" + json.dumps(table) + "\n```\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_for("k_a<1>") == 1234.0
    assert bench.traffic_for("k_b") is None
    src.write_text("v2\n")
    assert bench.traffic_for("k_a<1>") is None


def test_replay_run_takes_the_longest_back_to_back_run(tmp_path):
    """Dispatches of K at 0/10/20 us (run of 3, 4 us each) and at 100 us
    (run of 1), with another kernel between: the longest run is the first."""
    rows = []
    for t0 in (0, 10_000, 20_000):
        rows.append(["void K(int)", t0, t0 + 4_000])
    rows.append(["other", 30_000, 31_000])
    rows.append(["void K(int)", 100_000, 109_000])
    path = tmp_path / "trace.csv"
    _write_csv(str(path), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    line = profsum.replay_run(str(path), "K")
    assert "run 3 dispatches" in line
    assert "mean kernel duration 4.000 us" in line
    assert "mean start-to-start 8.000 us" in line      # (24 us span) / 3
    assert profsum.replay_run(str(path), "missing").startswith("no dispatch")


def test_generators_are_seeded():
    cfg = synth.CONFIGS["bump64"]
    a = synth.make_problem(cfg)
    b = synth.make_problem(cfg)
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    w1 = synth.make_weights(2, cfg.channels, cfg.nu1, cfg.nu2, 0)
    w2 = synth.make_weights(2, cfg.channels, cfg.nu1, cfg.nu2, 0)
    w3 = synth.make_weights(2, cfg.channels, cfg.nu1, cfg.nu2, 1)
    assert len(w1) == len(w2) == len(w3)
    assert all(np.array_equal(a["w"], b["w"]) for a, b in zip(w1, w2))
    assert any(not np.array_equal(a["w"], c["w"]) for a, c in zip(w1, w3))
    # scale: the sample std of the largest tensor near sqrt(1 / (fan-in x taps))
    names = synth.weights.weight_names(2, cfg.channels, cfg.nu1, cfg.nu2)
    k = max(range(len(w1)), key=lambda i: w1[i]["w"].size)
    fan_in = names[k][5]
    assert 0.9 < w1[k]["w"].std() * np.sqrt(fan_in * 9) < 1.1
    r1, r2 = synth.random_rhs((5, 7), 3), synth.random_rhs((5, 7), 3)
    assert np.array_equal(r1, r2) and r1.dtype == np.complex128


def test_workload_geometry():
    """Extended sides and per-level sides of the single-problem workloads
    (ceil halving), and the point source on an interior node."""
    g = synth.CONFIGS["grf1024"]
    assert synth.level_sides(synth.ext_side(g.n, g.npml), len(g.channels)) == [1056, 528, 264, 132, 66, 33]
    l3 = synth.CONFIGS["layered192"]
    assert synth.level_sides(synth.ext_side(l3.n, l3.npml), len(l3.channels)) == [216, 108, 54, 27, 14]
    f = synth.point_source(64, 8, (0.5, 0.25), 2)
    assert f.shape == (80, 80) and f.sum() == 1.0 and f[8 + 32, 8 + 16] == 1.0


def test_batched_workload_sizes_and_sources():
    """The 64-problem batch: sides from the configured set, ellipse speeds
    within [1, 10], sources zero in the PML, frequencies at the configured
    points per wavelength."""
    cfg = synth.CONFIGS["ellipses64"]
    probs = synth.make_batch(cfg)
    assert len(probs) == cfg.extra["count"]
    for p in probs:
        s = p["n"]
        assert s in cfg.extra["sides"]
        assert p["c"].shape == (s, s)
        assert p["c"].min() >= 1.0 and p["c"].max() <= 10.0
        f = p["f"]
        assert f.shape == (s + 2 * cfg.npml,) * 2
        assert np.all(f[:cfg.npml] == 0) and np.all(f[-cfg.npml:] == 0)
        assert np.all(f[:, :cfg.npml] == 0) and np.all(f[:, -cfg.npml:] == 0)
        wavelength = 2 * np.pi * p["c"].min() / p["omega"]
        assert wavelength == pytest.approx(cfg.ppw * p["h"])
