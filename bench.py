#!/usr/bin/env python3
"""Benchmark: CRBM block-Gibbs sampling of the Shastry-Sutherland Ising lattice
on one MI355X.

One step = the whole annealing workload at 18x18 (the paper's largest lattice,
324 spins): J2/J1 in {0.5, 1.0, 1.5, 2.0} x 16 fields h/J1 = 3j/15 in [0, 3]
= 64 Hamiltonian points, 4096 chains each (262,144 chains), geometric anneal
T 5.0 -> 0.05 over 10^4 sweeps, 16.16 fixed-point couplings, then the exact
final-state energy and magnetisation of every point.  Inputs (tables, initial
spins) are resident in HBM before the timed region.

The other legs (uneven batch, 48x48 / 96x96 scale, time-to-solution,
hardware precision, learned MH at 18x18 and at the scale points) follow the
headline.  Progress lines start with '#'; the last line is one compact JSON
object (metric, value = visible spin-updates/s, roofline of the Gibbs kernel,
a few numbers per leg, CPU-oracle baseline); the full per-leg tables go to
the --detail-out file.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin-updates/s + energy ESS/s at 18x18, learned-MH vs plain Gibbs"
L = 18
S = 10000
CHAINS = 4096
SEED = 0x5EED000000000002
J2S = (0.5, 1.0, 1.5, 2.0)
HS = tuple(3.0 * j / 15 for j in range(16))

# Algorithmic integer work per visible spin and sweep, three models (the
# headline fraction uses the first; the others are reported beside it):
#
# lazy_exact: what an exact Gibbs decision needs.  3.5 stochastic units (1
#   spin + 2.5 hidden units); comparing a uniform U with a threshold t bit by
#   bit from the top ends at the first bit where they differ, after 2 bits on
#   average, so 7 random bits = 7/128 of a Philox4x32-10 block (10 rounds x
#   (2 multiplies + 2 three-input xors) = 40 ops); one compare per unit; the
#   hidden unit's 2-spin pattern (1 op) and the spin's 5-term pattern (4 ops)
#   plus its table lookup (1 op).
PHILOX_BLOCK_OPS = 40.0
OPS_LAZY = 7.0 / 128.0 * PHILOX_BLOCK_OPS + 3.5 + 2.5 * 1.0 + 1.0 * (4.0 + 1.0)
# slot16: a 16-bit uniform slot (1/8 block) and one compare per unit
OPS_SLOT16 = 3.5 * (PHILOX_BLOCK_OPS / 8.0 + 1.0)
# uniform32: a full 32-bit uniform (1/4 block) and one compare per unit; the
#   kernel draws fewer random bits than this, so its fraction exceeds 1
OPS_U32 = 3.5 * (PHILOX_BLOCK_OPS / 4.0 + 1.0)
# MI355X integer VALU peak: 256 CUs x 64 lanes x 2.4 GHz (one 32-bit op per lane per clock)
ALU_PEAK_OPS = 256 * 64 * 2.4e9
# MI355X dense bf16 matrix-core peak, FLOP/s
BF16_PEAK_FLOPS = 2.5e15
# masked-tap work of one 18x18 forward pass of the 12-layer 32-channel proposal:
# layer 1 4 taps x 1 -> 32, layers 2-11 5 taps x 32 -> 32, layer 12 5 taps x 32 -> 1
AR_FLOP_PER_SAMPLE = 2 * 324 * (4 * 1 * 32 + 10 * 5 * 32 * 32 + 5 * 32 * 1)
# MI355X LDS peak: 256 CUs x 128 bytes per clock x 2.4 GHz
LDS_PEAK_BPS = 256 * 128 * 2.4e9


def instances(crbm, chains=CHAINS):
    out = []
    k = 0
    for J2 in J2S:
        for h in HS:
            out.append(crbm.Instance(L=L, J1=1.0, J2=J2, h=h, n_chains=chains, sched="geometric", T0=5.0,
                                     T1=0.05, id=k))
            k += 1
    return out


PROFILE = os.path.join(ROOT, "profiles", "gibbs_kernel_18x18_anneal_64pts.md")
PROFILE_KEYS = ("traffic_bytes_per_launch", "valu_lane_insts_per_spin_sweep", "lds_bytes_per_spin_sweep",
                "kernel_sources_sha256_12")


def profile_fields():
    """Counter figures of the 18x18 Gibbs kernel from its committed rocprofv3
    summary ("key: value" lines), or {} once the kernel sources differ from
    the ones that were profiled (the summary records their hash)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("gibbs_kernel.h", "crbm_internal.h"):
        with open(os.path.join(ROOT, "paper_2511_20911_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    try:
        with open(PROFILE) as fh:
            fields = dict(line.split(": ", 1) for line in fh.read().splitlines()
                          if line.split(": ", 1)[0] in PROFILE_KEYS)
    except OSError:
        return {}
    if fields.get("kernel_sources_sha256_12", "").strip() != h.hexdigest()[:12]:
        return {}
    return {k: float(v) for k, v in fields.items() if k != "kernel_sources_sha256_12"}


COPY_MIB = 1024  # the plain device copy that calibrates FETCH_SIZE and WRITE_SIZE


def pmc_kib(db, counter, kernel_prefix):
    """KiB that `counter` reads for the largest dispatch of the kernel whose
    name contains kernel_prefix and for the largest __amd_rocclr_copyBuffer
    dispatch (the calibration copy), from a rocprofv3 --pmc results database."""
    import sqlite3
    con = sqlite3.connect(db)
    per = {}
    for name, ctr, disp, val in con.execute(
            "select kernel_name, counter_name, dispatch_id, value from counters_collection"):
        if ctr != counter:
            continue
        key = ("kernel" if kernel_prefix in name else "copy" if "__amd_rocclr_copyBuffer" in name else None)
        if key is not None:
            per[(key, disp)] = per.get((key, disp), 0.0) + float(val)
    con.close()
    kern = [v for (k, _), v in per.items() if k == "kernel"]
    copy = [v for (k, _), v in per.items() if k == "copy"]
    if not kern or not copy:
        raise RuntimeError(f"{counter}: no {kernel_prefix!r} or copy dispatch in {db}")
    return max(kern), max(copy)


def measure_traffic(rows, wpb, timeout=90, out_root=None):
    """HBM bytes of one launch of the 18x18 Gibbs kernel, measured now: two
    child runs of this script under rocprofv3 --pmc (FETCH_SIZE, then
    WRITE_SIZE), each holding one full launch of the same tiling and a plain
    1 GiB device copy; each counter is scaled by the bytes the copy moves
    over what it reads for the copy.  Returns (bytes, detail).  A child takes
    a few seconds; one that has not finished in `timeout` seconds is killed
    with its process group, and the first failure ends the measurement."""
    import glob
    import shutil
    import signal
    import subprocess
    exe = shutil.which("rocprofv3") or "/opt/rocm/bin/rocprofv3"
    out_root = out_root or os.path.join(ROOT, "gpurun_out", "bench_pmc")
    kname = f"gibbs_kernel<{L}, {rows}"
    res = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        d = os.path.join(out_root, ctr)
        shutil.rmtree(d, ignore_errors=True)
        cmd = [exe, "--pmc", ctr, "-d", d, "-o", "pmc", "--", sys.executable, os.path.join(ROOT, "bench.py"),
               "--headline-only", "--no-cpu-baseline", "--tiling", f"{rows},{wpb}", "--detail-out=",
               "--steps", "1", "--warmup", "0", "--copy-mib", str(COPY_MIB), "--traffic", "off"]
        proc = subprocess.Popen(cmd, cwd="/tmp", env=dict(os.environ, TMPDIR="/tmp"), start_new_session=True,
                                stdout=subprocess.DEVNULL, stderr=subprocess.PIPE)
        try:
            _, err = proc.communicate(timeout=timeout)
        except subprocess.TimeoutExpired:
            os.killpg(proc.pid, signal.SIGKILL)
            proc.wait()
            raise RuntimeError(f"rocprofv3 --pmc {ctr}: no result within {timeout} s")
        dbs = glob.glob(os.path.join(d, "**", "*results.db"), recursive=True)
        if not dbs:
            tail = err.decode(errors="replace").strip().splitlines()[-3:]
            raise RuntimeError(f"rocprofv3 --pmc {ctr} (exit {proc.returncode}) wrote no database: {tail}")
        res[ctr] = pmc_kib(dbs[0], ctr, kname)
    (fk, fc), (wk, wc) = res["FETCH_SIZE"], res["WRITE_SIZE"]
    copy_kib = COPY_MIB * 1024.0
    f_scale, w_scale = copy_kib / fc, copy_kib / wc
    traffic = (fk * f_scale + wk * w_scale) * 1024.0
    return traffic, {"fetch_kib": _r(fk, 7), "write_kib": _r(wk, 7), "fetch_scale": _r(f_scale, 4),
                     "write_scale": _r(w_scale, 4)}


def _oracle_worker(job):
    """One host process of the CPU baseline: full-schedule oracle chains of
    the 18x18 workload (a list of (point index, chain)).  Returns the final
    states and the process's own elapsed time."""
    import oracle
    t0 = time.perf_counter()
    finals = {}
    for k, ch in job:
        J2, h = J2S[k // 16], HS[k % 16]
        oi = oracle.Instance(L, 1.0, J2, h, "geometric", 5.0, 0.05, id=k)
        s, _, _ = oracle.run_chain(oi, S, SEED, ch, 0, S)
        finals[(k, ch)] = s
    return finals, time.perf_counter() - t0


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def cpu_baseline(chains_per_proc=4, max_procs=16):
    """The CPU oracle (plain single-threaded C) on a bounded sample of the
    same workload: one oracle process per host core (at most max_procs), each
    running chains_per_proc full-schedule chains of its own; chain p of point
    (4p + j) mod 64 for process p, so the processes' chains are disjoint and
    spread over the points.  Runs before the GPU is touched (forked workers)."""
    import multiprocessing as mp
    model, avail = host_cpu()
    procs = max(1, min(max_procs, avail))
    jobs = [[((4 * p + j) % 64, p) for j in range(chains_per_proc)] for p in range(procs)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    finals = {}
    for f, _ in res:
        finals.update(f)
    per_chain = S * L * L
    per_proc = [chains_per_proc * per_chain / dt for _, dt in res]
    rate = len(finals) * per_chain / wall
    return {"value": rate, "unit": "spin-updates/s", "cores": procs, "kind": "oracle",
            "per_core": float(sum(per_proc) / len(per_proc)),
            "cpu_model": model, "cpus_available": avail,
            "sample": f"{len(finals)} chains of the 18x18 workload ({chains_per_proc} per process, "
                      f"{procs} single-threaded oracle processes on disjoint chains), full {S}-sweep "
                      f"schedule each, {wall:.1f} s wall"}, finals


def c1_leg(crbm, torch):
    """The 6x6 job (36 spins): J1 = 1, J2/J1 = 0.5, h = 0, 256 chains, linear
    anneal T 3.0 -> 0.1 over 2000 sweeps, seed 0x5EED...01.  A tiny job, so
    its figure is latency: wall time of create (tables, seeded start) + the
    2000 sweeps + the exact observables of the last sweep, median of five
    runs after a warm-up, and the device time of the sweeps (HIP events).
    The final state is the Neel state of this point (E/N = -1.75, m = 0)."""
    import statistics
    r, w, _ = crbm.autotune(6, n_chains=256, n_sweeps=200)  # the tiling for this job's own chain count
    I = crbm.Instance(L=6, J1=1.0, J2=0.5, h=0.0, n_chains=256, sched="linear", T0=3.0, T1=0.1, id=0)
    wall, dev, obs = [], [], None
    for k in range(6):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        smp = crbm.Sampler([I], seed=0x5EED000000000001, n_sweeps=2000, measure_every=1, burn_in=1999)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream()
        e0.record(stream)
        smp.sample(2000)
        e1.record(stream)
        obs = smp.observables()[0]
        t1 = time.perf_counter()
        if k > 0:
            wall.append((t1 - t0) * 1e3)
            dev.append(e0.elapsed_time(e1))
        smp.close()
    work = 256 * 2000 * 36
    return {"workload": "SS Ising 6x6, J2/J1 = 0.5, h = 0, 256 chains, linear T 3.0 -> 0.1 over 2000 sweeps",
            "tiling": [r, w], "latency_ms": statistics.median(wall), "sweeps_device_ms": statistics.median(dev),
            "spin_updates_per_s": work / (statistics.median(dev) / 1e3),
            "E_per_spin": obs["E_per_spin"], "m": obs["m"], "abs_m": obs["abs_m"]}


def batched_uneven(crbm, torch):
    """Uneven batch (2048 instances, L in {6..48}, 256 chains, 5000 sweeps at
    fixed T) in one hipGraph launch of persistent kernels."""
    from paper_2511_20911_amd import workloads
    pts = workloads.batched_uneven()
    insts = [crbm.Instance(L=p.L, J1=p.J1, J2=p.J2, h=p.h, n_chains=p.n_chains, sched=p.sched, T0=p.T0,
                           T1=p.T1, id=p.id) for p in pts]
    sweeps = 5000
    for Lb in sorted({p.L for p in pts}):  # tuned on this size's share of the batch
        crbm.autotune(Lb, n_chains=sum(p.n_chains for p in pts if p.L == Lb), n_sweeps=20)
    smp = crbm.Sampler(insts, seed=workloads.SEED_BATCHED, n_sweeps=2 * sweeps, launch="graph")
    smp.sample(50)  # warm-up launch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    smp.sample(sweeps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    work = sum(p.n_chains * p.L * p.L for p in pts) * sweeps
    del smp
    # load balance: each lattice size of the batch alone (its own instances, same
    # tiling, direct launch), timed over the same sweeps; the sum of those times
    # is what a perfectly balanced batch would take
    alone = {}
    for Lb in sorted({p.L for p in pts}):
        sub = [I for I in insts if I.L == Lb]
        s1 = crbm.Sampler(sub, seed=workloads.SEED_BATCHED, n_sweeps=sweeps + 50)
        s1.sample(50)
        torch.cuda.synchronize()
        e0.record()
        s1.sample(sweeps)
        e1.record()
        torch.cuda.synchronize()
        alone[str(Lb)] = {"instances": len(sub), "ms": e0.elapsed_time(e1),
                          "spin_updates_per_s": sum(I.n_chains for I in sub) * Lb * Lb * sweeps /
                          (e0.elapsed_time(e1) / 1e3)}
        del s1
    sum_alone = sum(v["ms"] for v in alone.values())
    return {"workload": "2048 instances, L in {6,12,18,24,36,48} by seed, J2/J1~U[0.2,2.5], h/J1~U[0,3], "
                        "T~logU[0.05,5] fixed, 256 chains each, 5000 sweeps, one hipGraph launch",
            "spin_updates_per_s": work / (ms / 1e3), "ms": ms,
            "per_L_alone": alone, "sum_of_per_L_ms": sum_alone,
            "load_balance_efficiency": sum_alone / ms,
            "tiling": {str(Lb): crbm.get_tiling(Lb) for Lb in sorted({p.L for p in pts})}}


def scale_gibbs(crbm, torch, sizes=((48, 2000), (96, 500))):
    """Plain Gibbs at 48x48 and 96x96: 64 (J2/J1, h, T) points clustered on the
    T = 0 phase boundaries, 512 chains each, fixed T per point."""
    from paper_2511_20911_amd import workloads
    out = []
    for Ls, sweeps in sizes:
        pts = workloads.scale_points(Ls)
        insts = [crbm.Instance(L=p.L, J1=p.J1, J2=p.J2, h=p.h, n_chains=p.n_chains, sched=p.sched, T0=p.T0,
                               T1=p.T1, id=p.id) for p in pts]
        crbm.autotune(Ls, n_chains=sum(p.n_chains for p in pts), n_sweeps=20)
        smp = crbm.Sampler(insts, seed=workloads.SEED_SCALE, n_sweeps=sweeps + 20, measure_every=1,
                           burn_in=20 + sweeps // 2)
        smp.sample(20)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        smp.sample(sweeps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        obs = smp.observables()
        out.append({"L": Ls, "points": len(pts), "chains": smp.total_chains, "sweeps": sweeps,
                    "spin_updates_per_s": smp.total_chains * Ls * Ls * sweeps / (ms / 1e3), "ms": ms,
                    "tiling": crbm.get_tiling(Ls),
                    "E_per_spin_first4": [round(o["E_per_spin"], 5) for o in obs[:4]]})
        del smp
    return {"workload": "SS Ising 48x48 and 96x96, 64 points on the T=0 phase boundaries (offsets N(0,0.1)), "
                        "T~logU[0.1,1] fixed, 512 chains each; measured over the second half of the sweeps",
            "sizes": out}


def learned_mh(crbm, torch, temps=(0.4, 0.2, 0.1), steps=800, cycles=500):
    """Learned MH vs plain Gibbs at 18x18 on the 1/3 plateau (J2/J1 = 1, h/J1 = 3):
    per temperature, train the 12-layer 32-channel proposal on 2^20 Gibbs
    samples, then run 1 MH : 10 Gibbs sweeps on 8192 chains and plain Gibbs for
    the same wall time from the same seeded start; energy ESS/s of both and
    the bias of <E>/N against the exact transfer-matrix value."""
    from paper_2511_20911_amd import learned
    ref_path = os.path.join(ROOT, "tests", "golden", "plateau_reference.json")
    with open(ref_path) as f:
        vals = [v for v in json.load(f)["values"] if v["L"] == 12]
    ref = {v["T"]: v["E_per_spin"] for v in vals}
    ref_m = {v["T"]: v["m"] for v in vals}
    out = {"workload": "SS Ising 18x18, J1=1, J2/J1=1.0, h/J1=3.0 (1/3 plateau); proposal: 12 masked 3x3 conv "
                       "layers, 32 channels, bf16 weights, fp32 accumulation, trained on 2^20 Gibbs samples "
                       "(4096 chains annealed 5->T over 2e4 sweeps, 256 snapshots 20 sweeps apart, translation "
                       "and transpose augmentation); 8192 chains, 1 MH : 10 Gibbs vs plain Gibbs at equal wall "
                       "time, seeded +-1 start, first 20% discarded",
           "reference": "exact <E>/N and <m> by 12x12 row transfer matrix",
           "ess": "energy ESS (ess_per_s) and min over {energy, O_1/3 = max |S(q*)|^2/N^2} (ess_min_per_s)",
           "sectors": "moves between the six degenerate plateau ground states (orientation and phase of the "
                      "larger structure-factor amplitude), which E and O_1/3 do not see: 1024 chains from the "
                      "same equilibrated states, 100 steps each, untimed; per chain and second at the timed "
                      "comparison's cycle and sweep times (sector_moves_per_chain_s: [learned, gibbs])",
           "points": []}
    for T in temps:
        t0 = time.perf_counter()
        data = learned.training_set(L, 1.0, 1.0, 3.0, T)
        torch.cuda.synchronize()
        t_data = time.perf_counter() - t0
        net = crbm.ARNet(L, seed=5)
        net.init_params(seed=5, scale=0.5)
        t0 = time.perf_counter()
        loss = learned.train(net, data, steps=steps)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        del data
        r = learned.compare(net, L, 1.0, 1.0, 3.0, T, cycles=cycles)
        for k in ("learned", "gibbs"):
            d = r[k]["E_per_spin"] - ref[T]
            # se = 0: every kept sample has the same energy; then report the bias only if it is not rounding
            r[k]["bias_se"] = d / r[k]["se"] if r[k]["se"] > 0 else (0.0 if abs(d) < 1e-12 else None)
            dm = r[k]["m"] - ref_m[T]
            r[k]["bias_m_se"] = dm / r[k]["m_se"] if r[k]["m_se"] > 0 else (0.0 if abs(dm) < 1e-12 else None)
        # algorithmic training work: forward, data gradient and weight gradient over
        # the masked taps, 3 x 33.4 MFLOP per 18x18 sample, 1024 samples per step
        step_flop = 3 * AR_FLOP_PER_SAMPLE * 1024
        r.update({"T": T, "E_ref": ref[T], "data_s": t_data, "train_s": t_train, "train_steps": steps,
                  "train_step_ms": 1e3 * t_train / steps,
                  "train_tflops": step_flop / (t_train / steps) / 1e12,
                  "train_frac_bf16": step_flop / (t_train / steps) / BF16_PEAK_FLOPS,
                  "final_loss_per_site": loss,
                  "ess_ratio": r["learned"]["ess_per_s"] / r["gibbs"]["ess_per_s"],
                  "ess_min_ratio": r["learned"]["ess_min_per_s"] / r["gibbs"]["ess_min_per_s"]})
        # tunnelling between the six degenerate plateau ground states (untimed,
        # 1024 chains), as sector changes per chain and second of each sampler
        sec = learned.sector_moves(net, L, 1.0, 1.0, 3.0, T)
        sec["learned"]["per_chain_per_s"] = sec["learned"]["changes_per_chain_step"] / (
            r["learned"]["ms_per_cycle"] / 1e3)
        sec["gibbs"]["per_chain_per_s"] = sec["gibbs"]["changes_per_chain_step"] / (
            r["gibbs"]["us_per_sweep"] * r["learned"]["gibbs_per_mh"] / 1e6)
        r["sectors"] = sec
        out["points"].append(r)
        del net
        torch.cuda.empty_cache()
    return out


def learned_points(crbm, torch, L=48, steps=400, cycles=60, chains=512):
    """Conditional learned MH vs plain Gibbs over the 64 scale points at LxL
    (points near the T = 0 phase boundaries, 512 chains each, all in one
    handle): one 12-layer 32-channel network conditioned on (J2/J1, h/4, ln T)
    through per-layer bias offsets, trained on Gibbs samples of all points,
    then 1 MH : 10 Gibbs sweeps against plain Gibbs for the same wall time."""
    import numpy as np
    from paper_2511_20911_amd import learned, workloads
    pts = [(p.J2, p.h, p.T0) for p in workloads.scale_points(L)]
    t0 = time.perf_counter()
    data, pidx = learned.training_set_points(pts, L, chains, anneal_sweeps=2000, snapshots=16, spacing=50)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = crbm.ARNet(L, seed=5, cond_points=len(pts))
    net.set_points(np.array([learned.features(*p) for p in pts]))
    net.init_params(seed=5, scale=0.5)
    t0 = time.perf_counter()
    loss = learned.train_points(net, data, pidx, steps=steps, batch=256)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_train = int(data.shape[0])
    del data, pidx
    torch.cuda.empty_cache()
    r = learned.compare_points(net, pts, L, chains, cycles=cycles, gibbs_per_mh=10, trace_every=10)
    del net
    torch.cuda.empty_cache()
    r.update({"channels": 32, "workload": f"SS Ising {L}x{L}, the 64 scale points (4 phase-boundary lines, T ~ logU[0.1, 1]), "
                          f"{chains} chains each in one handle; conditional proposal: 12 masked 3x3 conv layers, "
                          "32 channels, bias offsets from a 3-32-384 tanh MLP of (J2/J1, h/4, ln T); trained on "
                          f"{n_train} Gibbs samples (anneal 5->T over 2000 sweeps, 16 snapshots 50 sweeps apart, "
                          "translation and transpose augmentation), "
                          f"{steps} Adam steps of batch 256; 1 MH : 10 Gibbs vs plain Gibbs at equal wall time, "
                          "seeded +-1 start, first 20% discarded",
              "ess": "sum over points of chains x kept samples / max(tau_E, tau_m)",
              "data_s": t_data, "train_s": t_train, "train_steps": steps, "final_loss_per_site": loss,
              "ess_min_ratio": r["learned"]["ess_min_per_s"] / r["gibbs"]["ess_min_per_s"]})
    return r


# Sec. III.C / Fig. 5 phase points and the paper's TTS_99 on its 30 MHz FPGA
# (one sample per 33.3 ns), context only
TTS_POINTS = (("fm", 1.0, 7.0, "33 ns"), ("dimer", 2.5, 0.0, "~5 us"), ("neel", 1.0, 0.0, "200 us"),
              ("one_third", 0.5, 4.0, "120 ms"))


def tts_leg(crbm, torch, sizes=(6, 12, 18), temps=(0.2, 0.3, 0.5, 0.7, 1.0), chains=8192, sweeps=20000,
            long_sweeps=100000, long_temps=(0.2, 0.3)):
    """Time-to-solution (Eq. (14)) at the four phase points: constant-T runs
    from the seeded random start, per-chain minimum energy and first hit on
    the device, p_gnd against the exact ordered ground state, best T of a
    small grid (the paper tunes beta per problem).  The 1/3 plateau at L >= 12
    is rarely solved within the grid's runs; it gets longer runs at the two
    lowest temperatures as well."""
    import numpy as np
    from paper_2511_20911_amd import tts as T

    fin = lambda x: None if x is None or not np.isfinite(x) else float(x)
    out = []
    for k, (phase, J2, h, paper) in enumerate(TTS_POINTS):
        for j, L in enumerate(sizes):
            base_id = 1000 + 100 * k + 10 * j
            r = T.phase_tts(L, J2, h, temps, chains, sweeps, seed=SEED + 5, id=base_id)
            assert r["phase"] == phase
            cands = [(x, sweeps) for x in r["by_T"]]
            if phase == "one_third" and L >= 12:
                r2 = T.phase_tts(L, J2, h, long_temps, chains, long_sweeps, seed=SEED + 6, id=base_id + 5)
                cands += [(x, long_sweeps) for x in r2["by_T"]]
            b, run_len = min(cands, key=lambda c: c[0]["tts_sweeps"])
            out.append({"phase": phase, "J2": J2, "h": h, "L": L, "best_T": b["T"], "run_sweeps": run_len,
                        "p_gnd": b["p_gnd"], "T_hit_sweeps": b["T_sweeps"], "tts99_sweeps": fin(b["tts_sweeps"]),
                        "tts99_latency_s": fin(b["tts_latency_s"]), "tts99_amortised_s": fin(b["tts_amortised_s"]),
                        "sweep_latency_us": b["sweep_latency_s"] * 1e6, "paper_fpga_tts99": paper,
                        "p_gnd_by_T": {f"{x['T']}@{n}": x["p_gnd"] for x, n in cands}})
    return {"protocol": f"{chains} independent constant-T runs per (phase, L, T), {sweeps} sweeps (1/3 plateau at "
                        f"L >= 12 also {long_sweeps} sweeps at T in {list(long_temps)}), from the seeded +-1 start; "
                        "p_gnd = share of runs whose lowest energy equals the exact ordered ground state; "
                        "T = mean first-hit sweep of those runs; TTS99 = T log(0.01)/log(1-p_gnd) (TTS100 = T); "
                        "best T of " + str(list(temps)),
            "times": "latency: one run sharing the GPU with the batch (device time per batch sweep); "
                     "amortised: device time per run-sweep",
            "context": "the paper's FPGA: one sample per 33.3 ns, so its TTS99 in sweeps is 1 (FM), ~150 (dimer), "
                       "~6e3 (Neel), ~3.6e6 (1/3) at its largest sizes",
            "points": out}


def _crossing(hs, m, level):
    """First h where m(h) rises through `level` (linear interpolation), or None."""
    for k in range(len(hs) - 1):
        if m[k] < level <= m[k + 1]:
            return hs[k] + (level - m[k]) * (hs[k + 1] - hs[k]) / (m[k + 1] - m[k])
    return None


def precision_leg(crbm, torch, temps=(0.1, 0.25, 0.5), n_h=65, h_max=8.0, chains=256, anneal=2000, measure=1000):
    """Magnetisation curve m(h) along J2/J1 = 1 at 18x18 (Fig. 3b) in the
    default 16.16 / 32-bit precision and in the hardware's Q5.4 / 16-bit one
    (App. A Dimension and Precision), at equal temperatures: geometric anneal
    5 -> T, then `measure` sweeps at T with exact accumulators.  For the two
    transitions (Neel -> 1/3 at h = 2, 1/3 -> FM at h = 5) it reports where m
    crosses the middle of its step and the 10-90 % width of the step."""
    import numpy as np

    hs = [h_max * k / (n_h - 1) for k in range(n_h)]
    steps = (("neel_to_third", 0.0, 1.0 / 3.0, 2.0), ("third_to_fm", 1.0 / 3.0, 1.0, 5.0))
    out = {"workload": f"SS Ising 18x18, J1 = J2 = 1, h in [0, {h_max}] ({n_h} points), {chains} chains each, "
                       f"geometric anneal 5 -> T over {anneal} sweeps then {measure} measured sweeps at T",
           "h": hs, "by_T": []}
    for T in temps:
        sched = np.concatenate([5.0 * (T / 5.0) ** (np.arange(anneal) / (anneal - 1)), np.full(measure, T)])
        row = {"T": T}
        for prec in ("q16", "fpga"):
            insts = [crbm.Instance(L=18, J1=1.0, J2=1.0, h=h, n_chains=chains, sched="explicit", T_explicit=sched,
                                   id=3000 + k) for k, h in enumerate(hs)]
            smp = crbm.Sampler(insts, seed=SEED + 7, n_sweeps=anneal + measure, measure_every=1, burn_in=anneal,
                               precision=prec)
            smp.sample(anneal + measure)
            obs = smp.observables()
            m = [float(o["m"]) for o in obs]
            smp.close()
            trans = {}
            for name, lo, hi, h_exact in steps:
                mid = _crossing(hs, m, lo + 0.5 * (hi - lo))
                a, b = _crossing(hs, m, lo + 0.1 * (hi - lo)), _crossing(hs, m, lo + 0.9 * (hi - lo))
                trans[name] = {"h_exact": h_exact, "h_mid": mid, "width_10_90": None if a is None or b is None else b - a}
            row[prec] = {"m": [round(x, 5) for x in m], "transitions": trans}
        out["by_T"].append(row)
    return out


def phase_map_leg(crbm, torch, L=18, chains=32, T=0.25, anneal=2000, measure=1000):
    """Magnetisation map m(J2/J1, h) of Fig. 3a at 18x18 (J2/J1 in [0, 3] by
    0.1, h/J1 in [-8, 8] by 0.25: 2015 points, 32 chains each, all in one
    handle; geometric anneal 3 -> T over `anneal` sweeps, then `measure`
    measured sweeps at T), and its transition lines: the fields where dm/dh
    peaks (Fig. 3b: the peaks of the first derivative sit at the critical
    points), each matched to the nearest T = 0 boundary of the four ordered
    phases (Neel | 1/3 at h = 4 - 2 J2, dimer | 1/3 at h = J2 - 2, 1/3 | FM at
    h = 4 + J2).  At T > 0 the lower line moves to smaller fields: the
    plateau's entropy favours it (Clausius-Clapeyron)."""
    import numpy as np
    from paper_2511_20911_amd import phase
    J2s = [round(0.1 * k, 2) for k in range(31)]
    hs = [-8.0 + 0.25 * k for k in range(65)]
    m, E, dt, work = phase.phase_map(J2s, hs, L=L, chains=chains, T=T, anneal=anneal, measure=measure)
    lines = []
    dev = {"neel_third": [], "dimer_third": [], "third_fm": []}
    for a, J2 in enumerate(J2s):
        found = [h for h in phase.transition_fields(hs, m[a]) if h > 0]
        exact = phase.boundaries_T0(J2)
        for x in exact:
            if not found:
                continue
            f = min(found, key=lambda v: abs(v - x))
            kind = "third_fm" if abs(x - (4 + J2)) < 1e-6 else ("neel_third" if J2 < 2 else "dimer_third")
            dev[kind].append(f - x)
        lines.append({"J2": J2, "h_transitions": [round(f, 3) for f in found],
                      "h_exact_T0": [round(x, 3) for x in exact]})
    summary = {k: {"mean_shift": float(np.mean(v)) if v else None, "max_abs_shift": float(np.max(np.abs(v))) if v else None,
                   "lines": len(v)} for k, v in dev.items()}
    return {"workload": f"SS Ising {L}x{L} periodic, J2/J1 in [0, 3] (31), h/J1 in [-8, 8] (65), {chains} chains per "
                        f"point in one handle, geometric anneal 3 -> {T} over {anneal} sweeps + {measure} measured "
                        "sweeps",
            "seconds": dt, "spin_updates_per_s": work / dt, "shift_from_T0_boundaries": summary, "lines": lines,
            "m": np.round(m, 4).tolist(), "J2": J2s, "h": hs}


def confined_leg(crbm, torch):
    """Laterally confined SS lattice of width 12 (12 columns open, 18 rows
    periodic; Sec. III.A-B, Fig. 3f, Fig. 4b,d) at J2/J1 = 1.5 across the
    confined transition at h = 3.5, against the periodic 18x18 lattice at the
    same points: <E>/N, <m> and the structure factor S(q)/N^2 (maximum,
    where, at (2pi/3, pi), (pi, 2pi/3) and Gamma, and two cuts)."""
    from paper_2511_20911_amd import phase
    hs = [2.5, 3.0, 3.5, 4.0, 4.5, 5.0]
    strip = phase.confined_scan(hs, width=12, length=18, J2=1.5, T=0.2)
    per = phase.confined_scan(hs, width=18, length=18, J2=1.5, T=0.2, open_cols=False, id0=6100)
    return {"workload": "SS Ising, J2/J1 = 1.5, h in {2.5 .. 5.0}; 12 x 18 strip (12 columns open, 18 rows periodic) "
                        "and 18 x 18 periodic; 512 chains per point, geometric anneal 5 -> 0.2 over 4000 sweeps, "
                        "2000 sweeps at 0.2, counts and displacement correlation every 4th sweep",
            "strip": strip, "periodic": per}


def raw_filter_leg(crbm, torch, sweeps=500, n_inst=64):
    """The general-lattice kernel (one coupling per filter, App. A
    Convoluter-Reverse; open axes) at 18x18: 64 instances x 4096 chains with
    ten random couplings each, periodic; the same with both axes open; the
    12 x 18 confined strip; and the square-lattice kernel on the SS couplings
    of the same size, all timed with HIP events over `sweeps` sweeps."""
    import numpy as np
    rng = np.random.default_rng(41)
    out = {}

    def timed(smp, work):
        smp.sample(20)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        smp.sample(sweeps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        return {"ms": ms, "spin_updates_per_s": work / (ms / 1e3)}

    for name, orr, oc, rows, cols in (("raw18_periodic", False, False, 18, 18), ("raw18_open", True, True, 18, 18),
                                      ("strip12x18", False, True, 18, 12)):
        lats = [crbm.Lattice(rows=rows, cols=cols, J=list(rng.uniform(-1.5, 1.5, 10)), h_even=float(rng.uniform(0, 3)),
                             h_odd=float(rng.uniform(0, 3)), open_rows=orr, open_cols=oc, n_chains=4096,
                             sched="const", T0=float(rng.uniform(0.3, 2.0)), id=7000 + k) for k in range(n_inst)]
        smp = crbm.LatticeSampler(lats, seed=SEED + 9, n_sweeps=sweeps + 20)
        out[name] = timed(smp, n_inst * 4096 * rows * cols * sweeps)
        del smp
    insts = [crbm.Instance(L=18, J1=1.0, J2=float(rng.uniform(0.5, 2)), h=float(rng.uniform(0, 3)), n_chains=4096,
                           sched="const", T0=float(rng.uniform(0.3, 2.0)), id=7100 + k) for k in range(n_inst)]
    smp = crbm.Sampler(insts, seed=SEED + 9, n_sweeps=sweeps + 20)
    out["square18_ss"] = timed(smp, n_inst * 4096 * 324 * sweeps)
    del smp
    out["workload"] = (f"{n_inst} instances x 4096 chains, constant T, {sweeps} sweeps: general-lattice kernel with ten "
                       "random filter couplings and random even/odd fields (18x18 periodic, 18x18 open, 12-wide strip), "
                       "and the square-lattice kernel on SS couplings (18x18)")
    return out


def _r(x, n=4):
    """Round to n significant digits for the compact result line."""
    if x is None:
        return None
    x = float(x)
    return float(f"{x:.{n}g}") if x == x and abs(x) != float("inf") else None


def headline_result(step_ms, kern_ms, chains, n_sweeps, n_points, rows, wpb, tuning, create_ms, prof, steps,
                    warmup):
    """The result line's headline fields from the measured step and kernel
    times (ms): value = median-step throughput, roofline of the Gibbs kernel
    from its mean HIP-event time, counter figures (prof) scaled to that
    speed."""
    import statistics
    ms = float(statistics.median(step_ms))
    spin_sweeps = chains * n_sweeps * L * L
    value = spin_sweeps / (ms / 1e3)
    kms = float(sum(kern_ms) / len(kern_ms))
    kernel_rate = spin_sweeps / (kms / 1e3)
    achieved = kernel_rate * OPS_LAZY
    roofline = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": ALU_PEAK_OPS / 1e12,
        "unit": "TOP/s",
        "frac": achieved / ALU_PEAK_OPS,
        "traffic": None,
        "kernel": f"gibbs_kernel<{L},{rows}>",
        "kernel_ms": kms,
        "work_model": "lazy_exact",
        "ops_per_spin_sweep": {"lazy_exact": OPS_LAZY, "slot16": OPS_SLOT16, "uniform32": OPS_U32},
        "frac_by_model": {"lazy_exact": _r(achieved / ALU_PEAK_OPS, 3),
                          "slot16": _r(kernel_rate * OPS_SLOT16 / ALU_PEAK_OPS, 3),
                          "uniform32": _r(kernel_rate * OPS_U32 / ALU_PEAK_OPS, 3)},
    }
    if prof:
        # issued VALU lane instructions per spin-sweep and the LDS (ds_bpermute)
        # bytes, from the SQ counters of the same kernel, at this run's speed
        if "valu_lane_insts_per_spin_sweep" in prof:
            v = prof["valu_lane_insts_per_spin_sweep"]
            roofline["valu_lane_insts_per_spin_sweep"] = v
            roofline["valu_issue_frac"] = _r(kernel_rate * v / ALU_PEAK_OPS, 3)
        if "lds_bytes_per_spin_sweep" in prof:
            lb = prof["lds_bytes_per_spin_sweep"]
            roofline["lds"] = {"achieved": _r(kernel_rate * lb / 1e12, 3), "peak": LDS_PEAK_BPS / 1e12,
                               "unit": "TB/s", "frac": _r(kernel_rate * lb / LDS_PEAK_BPS, 3)}
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "SS Ising 18x18 periodic, J1=1, J2/J1 in {0.5,1.0,1.5,2.0} x 16 h/J1 in [0,3], "
                        f"{chains // max(n_points, 1)} chains per point ({chains} chains), geometric anneal "
                        "T 5.0->0.05 over 10^4 sweeps, 16.16 fixed point, seeded +-1 start",
            "L": L, "points": n_points, "chains": chains, "sweeps": n_sweeps,
            "node_updates_per_s": value * 3.5,
            "step_ms_min_max": [min(step_ms), max(step_ms)],
            "create_and_tables_ms": create_ms,
            "tiling": {"rows_per_lane": rows, "lanes_per_chain": (L // 2) // rows, "waves_per_block": wpb,
                       "autotuned": tuning is not None},
        },
        "roofline": roofline,
    }
    return result


def final_line(result):
    """The one compact JSON line that ends the run."""
    return json.dumps(result, separators=(",", ":"))


def summarise(legs):
    """A few numbers per leg for the final result line (the full tables go to
    the detail file)."""
    out = {}
    c1 = legs.get("c1")
    if c1:
        out["c1"] = {"latency_ms": _r(c1["latency_ms"], 3), "sweeps_device_ms": _r(c1["sweeps_device_ms"], 3),
                     "E_per_spin": _r(c1["E_per_spin"], 5), "m": _r(c1["m"], 3)}
    b = legs.get("batched_uneven")
    if b:
        out["batched_uneven"] = {"spin_updates_per_s": _r(b["spin_updates_per_s"]), "ms": _r(b["ms"]),
                                 "load_balance_efficiency": _r(b["load_balance_efficiency"], 3),
                                 "frac": _r(b["spin_updates_per_s"] * OPS_LAZY / ALU_PEAK_OPS, 3)}
    s = legs.get("scale")
    if s:
        out["scale"] = {str(x["L"]): _r(x["spin_updates_per_s"]) for x in s["sizes"]}
        out["scale"]["frac"] = {str(x["L"]): _r(x["spin_updates_per_s"] * OPS_LAZY / ALU_PEAK_OPS, 3) for x in s["sizes"]}
    m = legs.get("learned_mh")
    if m:
        out["learned_mh"] = [{"T": p["T"], "acceptance": _r(p["learned"]["acceptance"], 3),
                              "ess_per_s_learned": _r(p["learned"]["ess_per_s"], 3),
                              "ess_per_s_gibbs": _r(p["gibbs"]["ess_per_s"], 3),
                              "ess_ratio": _r(p["ess_ratio"], 3), "ess_min_ratio": _r(p["ess_min_ratio"], 3),
                              "bias_se": [_r(p[k]["bias_se"], 2) for k in ("learned", "gibbs")],
                              "bias_m_se": [_r(p[k].get("bias_m_se"), 2) for k in ("learned", "gibbs")],
                              "train_step_ms": _r(p["train_step_ms"], 3), "train_frac_bf16": _r(p["train_frac_bf16"], 3),
                              "sector_moves_per_chain_s": [_r(p["sectors"][k]["per_chain_per_s"], 3)
                                                           for k in ("learned", "gibbs")] if "sectors" in p else None}
                             for p in m["points"]]
    c = legs.get("learned_mh_points")
    if c:
        out["learned_mh_points"] = {k: {"channels": v.get("channels"), "acceptance": _r(v["learned"]["acceptance"], 3),
                                        "ess_min_ratio": _r(v["ess_min_ratio"], 3),
                                        "agree_3se": v["points_agreeing_within_3se"], "points": len(v["points"])}
                                    for k, v in c.items()}
    t = legs.get("tts")
    if t:
        out["tts_sweeps"] = {f'{p["phase"]}@{p["L"]}': _r(p["tts99_sweeps"], 3) for p in t["points"]}
    pm = legs.get("phase_map")
    if pm:
        out["phase_map"] = {"spin_updates_per_s": _r(pm["spin_updates_per_s"], 3),
                            "mean_shift_from_T0": {k: _r(v["mean_shift"], 3)
                                                   for k, v in pm["shift_from_T0_boundaries"].items()}}
    cf = legs.get("confined")
    if cf:
        out["confined_S_peak_off_gamma"] = {k: [_r(p["S_max_off_gamma"], 3) for p in cf[k]["points"]]
                                            for k in ("strip", "periodic")}
    rf = legs.get("raw_filters")
    if rf:
        out["lattice_kernel"] = {k: _r(v["spin_updates_per_s"], 3) for k, v in rf.items() if isinstance(v, dict)}
    p = legs.get("precision")
    if p:
        out["precision_third_to_fm_h_mid"] = {
            str(r["T"]): [_r(r[q]["transitions"]["third_to_fm"]["h_mid"], 3) for q in ("q16", "fpga")]
            for r in p["by_T"]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed steps (the value is their median)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-chains", type=int, default=4, help="oracle chains per host process in the CPU baseline")
    ap.add_argument("--sweeps", type=int, default=S, help="sweeps per step (default: the full schedule)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (calibrates HBM byte counters)")
    ap.add_argument("--no-tune", action="store_true", help="skip the tiling autotuner")
    ap.add_argument("--tiling", type=str, default="",
                    help="R,W: use R cell rows per lane and W wavefronts per workgroup at 18x18 instead of tuning")
    ap.add_argument("--no-batched", action="store_true", help="skip the uneven-batch graph measurement")
    ap.add_argument("--no-mh", action="store_true", help="skip the learned-MH vs Gibbs ESS comparison")
    ap.add_argument("--no-scale", action="store_true", help="skip the 48x48 / 96x96 Gibbs measurement")
    ap.add_argument("--no-c5-mh", action="store_true", help="skip the conditional learned-MH comparison at 48x48")
    ap.add_argument("--no-c5-mh-96", action="store_true", help="skip the conditional learned-MH comparison at 96x96")
    ap.add_argument("--no-tts", action="store_true", help="skip the time-to-solution runs at the four phase points")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the m(h) comparison of the default and the hardware precision")
    ap.add_argument("--no-lattice", action="store_true",
                    help="skip the phase map, the confined-lattice S(q) scan and the general-lattice kernel timing")
    ap.add_argument("--headline-only", action="store_true", help="skip every leg but the headline")
    ap.add_argument("--legs", type=str, default="",
                    help="comma-separated legs to run after the headline (c1, batched_uneven, scale, tts, precision, "
                         "phase_map, confined, raw_filters, learned_mh, learned_mh_points); default: all")
    ap.add_argument("--traffic", choices=("live", "profile", "off"), default="live",
                    help="HBM traffic of the headline kernel: measured now by two rocprofv3 --pmc child runs "
                         "(live), taken from the committed profile while its kernel sources match (profile), "
                         "or not reported")
    ap.add_argument("--detail-out", type=str, default=os.path.join("gpurun_out", "bench_detail.json"),
                    help="file for the full per-leg tables ('' = none)")
    ap.add_argument("--chains-per-point", type=int, default=CHAINS,
                    help="chains per point of the headline launch, for measuring how the launch's last round of "
                         "wavefronts depends on the count (other counts need --headline-only --no-cpu-baseline "
                         "--traffic off; the line then names that workload)")
    args = ap.parse_args()
    if args.chains_per_point != CHAINS and not (args.headline_only and args.no_cpu_baseline and args.traffic == "off"):
        print("--chains-per-point other than the workload's needs --headline-only --no-cpu-baseline --traffic off",
              file=sys.stderr)
        sys.exit(2)
    if args.chains_per_point < 1:
        print("--chains-per-point must be positive", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1): chains are independent, and sharding them over "
              "several GPUs is a design, not an implemented path.", file=sys.stderr)
        sys.exit(2)
    if args.headline_only:
        args.no_batched = args.no_mh = args.no_scale = args.no_c5_mh = args.no_tts = args.no_precision = True
        args.no_lattice = True
    n_sweeps = min(args.sweeps, S)

    # the CPU baseline runs first, in forked host processes, before the GPU is touched
    base, finals = (None, {})
    if not args.no_cpu_baseline and n_sweeps == S:
        base, finals = cpu_baseline(chains_per_proc=args.cpu_chains)
        print(f"# cpu baseline: {base['sample']}", flush=True)

    import numpy as np
    import torch
    import paper_2511_20911_amd as crbm

    torch.cuda.set_device(0)
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tuning = None
    if args.tiling:
        r_, w_ = (int(x) for x in args.tiling.split(","))
        crbm.set_tiling(L, r_, w_)
    elif not args.no_tune:
        r, w, rate = crbm.autotune(L, n_chains=8192, n_sweeps=40)
        tuning = {"rows_per_lane": r, "waves_per_block": w, "tune_rate": rate}
    rows, wpb = crbm.get_tiling(L)
    insts = instances(crbm, chains=args.chains_per_point)
    t0 = time.perf_counter()
    smp = crbm.Sampler(insts, seed=SEED, n_sweeps=S, measure_every=1, burn_in=S - 1)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    init_spins, _ = smp.get_state()
    stream = torch.cuda.current_stream()

    step_ms, kern_ms = [], []
    obs = None
    for it in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        smp.set_state(init_spins, 0)
        smp.reset_observables()
        k0 = torch.cuda.Event(enable_timing=True)
        k1 = torch.cuda.Event(enable_timing=True)
        k0.record(stream)
        smp.sample(n_sweeps)
        k1.record(stream)
        obs = smp.observables() if n_sweeps == S else None
        torch.cuda.synchronize()
        t_end = time.perf_counter()
        if it >= args.warmup:
            step_ms.append((t_end - t_start) * 1e3)
            kern_ms.append(k0.elapsed_time(k1))
        print(f"# step {it}: {(t_end - t_start) * 1e3:.1f} ms", flush=True)

    prof = profile_fields() if n_sweeps == S else {}
    result = headline_result(step_ms, kern_ms, smp.total_chains, n_sweeps, len(insts), rows, wpb, tuning, create_ms,
                             prof, args.steps, args.warmup)
    roofline = result["roofline"]
    detail = {"headline": dict(result)}
    if obs is not None:
        E = np.array([o["E_per_spin"] for o in obs]).reshape(4, 16)
        m = np.array([o["m"] for o in obs]).reshape(4, 16)
        detail["final_state"] = {"J2": list(J2S), "E_per_spin_mean": E.round(5).tolist(),
                                 "m_mean": m.round(5).tolist()}
    parity = None
    if finals:
        spins, _ = smp.get_state()
        parts = smp.split_spins(spins.cpu())
        parity = all(np.array_equal(parts[i][ch].numpy(), s) for (i, ch), s in finals.items())
    del smp
    torch.cuda.empty_cache()

    # HBM traffic of the same launch: counters of two child runs while this
    # process is idle (skipped when this run is itself under a profiler)
    under_profiler = any(k.startswith("ROCPROF_") for k in os.environ)
    if n_sweeps == S and args.traffic == "live" and not under_profiler:
        t = time.perf_counter()
        try:
            tb, tinfo = measure_traffic(rows, wpb)
            roofline["traffic"] = tb
            roofline["traffic_source"] = dict(tinfo, how="rocprofv3 --pmc, this run")
        except Exception as exc:  # reported, and the committed figure (if current) stands in
            print(f"# traffic: live measurement failed: {exc}", flush=True)
            roofline["traffic_error"] = str(exc)[:200]
        print(f"# traffic: {time.perf_counter() - t:.1f} s", flush=True)
    if roofline["traffic"] is None and args.traffic != "off" and "traffic_bytes_per_launch" in prof:
        roofline["traffic"] = prof["traffic_bytes_per_launch"]
        roofline["traffic_source"] = {"how": "committed rocprofv3 profile of the same kernel sources"}

    legs = {}
    def leg(name, fn):
        t = time.perf_counter()
        legs[name] = fn()
        print(f"# leg {name}: {time.perf_counter() - t:.1f} s", flush=True)
    only = set(x for x in args.legs.split(",") if x)
    want = lambda name, off: (name in only) if only else not off  # noqa: E731
    if want("c1", args.no_batched):
        leg("c1", lambda: c1_leg(crbm, torch))
    if want("batched_uneven", args.no_batched):
        leg("batched_uneven", lambda: batched_uneven(crbm, torch))
    if want("scale", args.no_scale):
        leg("scale", lambda: scale_gibbs(crbm, torch))
    if want("tts", args.no_tts):
        leg("tts", lambda: tts_leg(crbm, torch))
    if want("precision", args.no_precision):
        leg("precision", lambda: precision_leg(crbm, torch))
    if want("phase_map", args.no_lattice):
        leg("phase_map", lambda: phase_map_leg(crbm, torch))
    if want("confined", args.no_lattice):
        leg("confined", lambda: confined_leg(crbm, torch))
    if want("raw_filters", args.no_lattice):
        leg("raw_filters", lambda: raw_filter_leg(crbm, torch))
    if want("learned_mh", args.no_mh):
        leg("learned_mh", lambda: learned_mh(crbm, torch))
    if want("learned_mh_points", args.no_c5_mh):
        def c5():
            r = {"48": learned_points(crbm, torch, 48)}
            if not args.no_c5_mh_96:
                r["96"] = learned_points(crbm, torch, 96, steps=200, cycles=20)
            return r
        leg("learned_mh_points", c5)
    detail.update(legs)
    result["legs"] = summarise(legs)
    if base is not None:
        base["parity_sampled_chains"] = parity
        result["cpu_baseline"] = base
        detail["cpu_baseline"] = base
    if args.detail_out:
        d = os.path.dirname(args.detail_out)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(args.detail_out, "w") as f:
            json.dump(detail, f, indent=1)
        result["detail_file"] = args.detail_out
    print(final_line(result), flush=True)


if __name__ == "__main__":
    main()
