"""bench.py's result line and counter parsing, on the CPU: the final JSON
line keeps the fields the harness reads and stays compact with every leg
present at its largest size, and the FETCH_SIZE / WRITE_SIZE reader picks the
kernel's and the calibration copy's dispatches from a rocprofv3 database."""
import json
import os
import sqlite3
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

X = 1.0 / 3.0  # long decimal expansions, the worst case for the line's length


def _mh_point(T):
    side = {"acceptance": X, "ess_per_s": X * 1e6, "bias_se": X, "bias_m_se": -X}
    sec = {"per_chain_per_s": X * 1e3}
    return {"T": T, "learned": dict(side), "gibbs": dict(side), "ess_ratio": X, "ess_min_ratio": X,
            "train_s": X, "train_step_ms": X, "train_frac_bf16": X,
            "sectors": {"learned": dict(sec), "gibbs": dict(sec)}}


def _all_legs():
    """Every leg that summarise() reads, with as many entries as the legs
    produce at their defaults (and the optional 96x96 conditional run)."""
    lm = {"channels": 64, "learned": {"acceptance": X}, "ess_min_ratio": X,
          "points_agreeing_within_3se": 64, "points": [{}] * 64}
    conf = {"points": [{"S_max_off_gamma": X} for _ in range(6)]}
    return {
        "c1": {"latency_ms": X * 1e2, "sweeps_device_ms": X * 10, "E_per_spin": -1.75 + X / 1e5, "m": X / 1e3},
        "batched_uneven": {"spin_updates_per_s": X * 1e12, "ms": X * 1e3, "load_balance_efficiency": X},
        "scale": {"sizes": [{"L": 48, "spin_updates_per_s": X * 1e12}, {"L": 96, "spin_updates_per_s": X * 1e12}]},
        "learned_mh": {"points": [_mh_point(T) for T in (0.4, 0.2, 0.1)]},
        "learned_mh_points": {"48": lm, "96": lm},
        "tts": {"points": [{"phase": ph, "L": Lt, "tts99_sweeps": X * 1e5}
                           for ph in ("fm", "dimer", "neel", "third") for Lt in (6, 12, 18)]},
        "phase_map": {"spin_updates_per_s": X * 1e12,
                      "shift_from_T0_boundaries": {k: {"mean_shift": -X} for k in
                                                   ("neel_third", "dimer_third", "third_fm")}},
        "confined": {"strip": conf, "periodic": conf},
        "raw_filters": {k: {"spin_updates_per_s": X * 1e12} for k in
                        ("periodic_18x18", "open_18x18", "strip_12x18", "square_kernel_18x18")},
        "precision": {"by_T": [{"T": T, "q16": {"transitions": {"third_to_fm": {"h_mid": 5 + X}}},
                                "fpga": {"transitions": {"third_to_fm": {"h_mid": 5 + X}}}}
                               for T in (0.1, 0.25, 0.5)]},
    }


def _full_result():
    prof = {"traffic_bytes_per_launch": 441837824.0, "valu_lane_insts_per_spin_sweep": 25.79,
            "lds_bytes_per_spin_sweep": 6.36}
    res = bench.headline_result([578.0 + X, 578.1, 578.2], [575.0 + X] * 3, 262144, bench.S, 64, 1, 1,
                                {"rows_per_lane": 1, "waves_per_block": 1, "tune_rate": X * 1e12}, 187.0 + X,
                                prof, 3, 1)
    rl = res["roofline"]
    rl["traffic"] = 441837824.0 + X
    rl["traffic_source"] = {"fetch_kib": 191457.125, "write_kib": 48568.0, "fetch_scale": 2.0, "write_scale": 1.0,
                            "how": "rocprofv3 --pmc, this run"}
    res["legs"] = bench.summarise(_all_legs())
    res["cpu_baseline"] = {"value": X * 1e9, "unit": "spin-updates/s", "cores": 16, "kind": "oracle",
                           "per_core": X * 1e8, "cpu_model": "x" * 64, "cpus_available": 16,
                           "sample": "64 chains of the 18x18 workload (4 per process, 16 single-threaded oracle "
                                     "processes on disjoint chains), full 10000-sweep schedule each, 20.0 s wall",
                           "parity_sampled_chains": True}
    res["detail_file"] = os.path.join("gpurun_out", "bench_detail.json")
    return res


def test_final_line_is_compact_and_complete():
    """With every leg present, the last line parses as one JSON object with
    the contract's fields and stays under 4 KB (the harness keeps only the
    last 8 KB of output)."""
    line = bench.final_line(_full_result())
    assert "\n" not in line
    assert len(line.encode()) < 4096, len(line)
    r = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in r, k
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r["roofline"], k
    assert abs(r["roofline"]["frac"] - r["roofline"]["achieved"] / r["roofline"]["peak"]) < 1e-12
    assert r["config"]["workload"] and r["n_gpus"] == 1
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in r["cpu_baseline"], k


def test_headline_value_is_median_step_throughput():
    """value = spin-sweeps of the step / median step time; the roofline's
    achieved = kernel rate (mean HIP-event time) x the lazy-exact work model."""
    res = bench.headline_result([500.0, 400.0, 600.0], [390.0, 410.0], 1000, 100, 1, 1, 1, None, 1.0, {}, 3, 0)
    work = 1000 * 100 * bench.L * bench.L
    assert res["value"] == pytest.approx(work / 0.5)
    assert res["ms_per_step"] == 500.0
    assert res["roofline"]["kernel_ms"] == pytest.approx(400.0)
    assert res["roofline"]["achieved"] == pytest.approx(work / 0.4 * bench.OPS_LAZY / 1e12)
    assert res["roofline"]["traffic"] is None


def _pmc_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, dispatch_id int, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()


def test_pmc_reader_picks_kernel_and_calibration_copy(tmp_path):
    """Per-dimension rows of one dispatch are summed; the largest kernel
    dispatch and the largest copy (the 1 GiB calibration, not the small
    state copies) are returned; other counters and kernels are ignored."""
    db = str(tmp_path / "pmc_results.db")
    k = "void crbmlib::gk::gibbs_kernel<18, 1, false>(crbmlib::GibbsArgs)"
    _pmc_db(db, [(k, "FETCH_SIZE", 7, 100000.0), (k, "FETCH_SIZE", 7, 91457.125),
                 (k, "WRITE_SIZE", 7, 48568.0),
                 ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 1, 524308.0), ("__amd_rocclr_copyBuffer", "FETCH_SIZE", 2, 523.5),
                 ("crbmlib::(anonymous namespace)::pack_kernel(unsigned int*)", "FETCH_SIZE", 3, 9e9),
                 ("void crbmlib::gk::gibbs_kernel<24, 1, false>(crbmlib::GibbsArgs)", "FETCH_SIZE", 4, 9e9)])
    kern, copy = bench.pmc_kib(db, "FETCH_SIZE", "gibbs_kernel<18, 1")
    assert kern == 191457.125 and copy == 524308.0
    with pytest.raises(RuntimeError):
        bench.pmc_kib(db, "WRITE_SIZE", "gibbs_kernel<18, 1")  # no copy dispatch for this counter


_FAKE_PROFILER = """#!{python}
import os, sqlite3, sys, time
a = sys.argv[1:]
ctr, d = a[a.index("--pmc") + 1], a[a.index("-d") + 1]
mode = os.environ.get("FAKE_PROFILER_MODE", "ok")
if mode == "hang":
    time.sleep(60)
if mode == "nodb":
    sys.exit(3)
os.makedirs(os.path.join(d, "host"), exist_ok=True)
con = sqlite3.connect(os.path.join(d, "host", "pmc_results.db"))
con.execute("create table counters_collection (kernel_name text, counter_name text, dispatch_id int, value real)")
kern = "void crbmlib::gk::gibbs_kernel<18, 1, false>(crbmlib::GibbsArgs)"
vals = {{"FETCH_SIZE": (191000.0, 524288.0), "WRITE_SIZE": (48000.0, 1048576.0)}}[ctr]
con.executemany("insert into counters_collection values (?, ?, ?, ?)",
                [(kern, ctr, 5, vals[0]), ("__amd_rocclr_copyBuffer", ctr, 6, vals[1]),
                 ("__amd_rocclr_copyBuffer", ctr, 7, 12.0)])
con.commit()
"""


def _fake_profiler(tmp_path, monkeypatch, mode):
    import shutil
    exe = tmp_path / "rocprofv3"
    exe.write_text(_FAKE_PROFILER.format(python=sys.executable))
    exe.chmod(0o755)
    monkeypatch.setattr(shutil, "which", lambda name: str(exe) if name == "rocprofv3" else None)
    monkeypatch.setenv("FAKE_PROFILER_MODE", mode)


def test_live_traffic_scales_both_counters_by_the_copy(tmp_path, monkeypatch):
    """The two child runs' databases are found, the kernel's and the 1 GiB
    copy's dispatches read, and each counter scaled by the copy's bytes over
    its reading: FETCH x 2, WRITE x 1 here."""
    _fake_profiler(tmp_path, monkeypatch, "ok")
    tb, info = bench.measure_traffic(1, 1, timeout=60, out_root=str(tmp_path / "out"))
    assert tb == pytest.approx((191000.0 * 2.0 + 48000.0) * 1024.0)
    assert info["fetch_scale"] == 2.0 and info["write_scale"] == 1.0
    assert info["fetch_kib"] == 191000.0 and info["write_kib"] == 48000.0


def test_live_traffic_failures_are_reported_and_bounded(tmp_path, monkeypatch):
    """A child that writes no database, or that does not finish in time, ends
    the measurement with an error (the bench then falls back or reports
    null); a hung child is killed at the limit."""
    import time
    _fake_profiler(tmp_path, monkeypatch, "nodb")
    with pytest.raises(RuntimeError, match="no database"):
        bench.measure_traffic(1, 1, timeout=60, out_root=str(tmp_path / "out"))
    _fake_profiler(tmp_path, monkeypatch, "hang")
    t0 = time.perf_counter()
    with pytest.raises(RuntimeError, match="no result within 2 s"):
        bench.measure_traffic(1, 1, timeout=2, out_root=str(tmp_path / "out"))
    assert time.perf_counter() - t0 < 20


def test_other_chain_counts_need_the_headline_only_flags():
    """--chains-per-point changes the workload, so bench.py accepts it only
    for a bare headline timing (no CPU baseline, no traffic, no legs) and
    exits with status 2 before touching a GPU otherwise."""
    import subprocess
    for extra in ([], ["--headline-only"], ["--headline-only", "--no-cpu-baseline"],
                  ["--headline-only", "--traffic", "off"]):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--chains-per-point", "4032"] + extra,
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 2 and "--chains-per-point" in r.stderr, (extra, r.returncode, r.stderr)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--chains-per-point", "0", "--headline-only",
                        "--no-cpu-baseline", "--traffic", "off"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "positive" in r.stderr
