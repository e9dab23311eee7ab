#!/usr/bin/env python3
"""Benchmark: CRBM block-Gibbs sampling of the Shastry-Sutherland Ising lattice
on one MI355X.

One step = the whole annealing workload at 18x18 (the paper's largest lattice,
324 spins): J2/J1 in {0.5, 1.0, 1.5, 2.0} x 16 fields h/J1 = 3j/15 in [0, 3]
= 64 Hamiltonian points, 4096 chains each (262,144 chains), geometric anneal
T 5.0 -> 0.05 over 10^4 sweeps, 16.16 fixed-point couplings, then the exact
final-state energy and magnetisation of every point.  Inputs (tables, initial
spins) are resident in HBM before the timed region.

Prints one JSON line (metric, value = visible spin-updates/s, roofline of the
Gibbs kernel, CPU-oracle baseline).
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

# Algorithmic integer work per visible spin and sweep:
# 3.5 stochastic units (1 spin + 2.5 hidden), each needing a 16-bit Philox
# slot (1/8 of a Philox4x32-10 block = 10 rounds x (2 mul-hi/lo + 2 xor3) = 40
# ops) and one integer compare.
OPS_PER_SPIN_SWEEP = 3.5 * (40.0 / 8.0 + 1.0)
# MI355X integer VALU peak: 256 CUs x 64 lanes x 2.4 GHz (one 32-bit op per lane per clock)
ALU_PEAK_OPS = 256 * 64 * 2.4e9


def instances(crbm, chains=CHAINS):
    out = []
    k = 0
    for J2 in J2S:
        for h in HS:
            out.append(crbm.Instance(L=L, J1=1.0, J2=J2, h=h, n_chains=chains, sched="geometric", T0=5.0,
                                     T1=0.05, id=k))
            k += 1
    return out


def measured_traffic():
    """HBM bytes per launch of the 18x18 Gibbs kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None once the kernel sources
    differ from the ones that were profiled."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "gibbs_kernel_18x18_anneal_64pts.md")
    h = hashlib.sha256()
    for f in ("gibbs_kernel.h", "crbm_internal.h"):
        with open(os.path.join(ROOT, "paper_2511_20911_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    try:
        fields = dict(line.split(": ", 1) for line in open(prof).read().splitlines()
                      if line.startswith(("traffic_bytes_per_launch: ", "kernel_sources_sha256_12: ")))
    except OSError:
        return None
    if fields.get("kernel_sources_sha256_12", "").strip() != h.hexdigest()[:12]:
        return None
    return int(fields["traffic_bytes_per_launch"])


def cpu_baseline(sample_points=3, chains_per_point=3):
    """The CPU oracle (single-threaded C) on a bounded sample of the same
    workload: the first chains of a few points, full schedule."""
    import numpy as np
    import oracle
    pts = [(J2S[0], HS[0]), (J2S[1], HS[15]), (J2S[2], HS[7]), (J2S[3], HS[3])][:sample_points]
    ids = {(J2, h): 16 * J2S.index(J2) + HS.index(h) for J2, h in pts}
    finals = {}
    t0 = time.perf_counter()
    for (J2, h) in pts:
        oi = oracle.Instance(L, 1.0, J2, h, "geometric", 5.0, 0.05, id=ids[(J2, h)])
        for ch in range(chains_per_point):
            s, _, _ = oracle.run_chain(oi, S, SEED, ch, 0, S)
            finals[(ids[(J2, h)], ch)] = s
    dt = time.perf_counter() - t0
    n = len(pts) * chains_per_point
    rate = n * S * L * L / dt
    return {"value": rate, "unit": "spin-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} chains ({sample_points} points x {chains_per_point}) x {S} sweeps at 18x18, "
                      f"{dt:.1f} s single-threaded"}, finals


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
        ref = {v["T"]: v["E_per_spin"] for v in json.load(f)["values"] if v["L"] == 12}
    out = {"workload": "SS Ising 18x18, J1=1, J2/J1=1.0, h/J1=3.0 (1/3 plateau); proposal: 12 masked 3x3 conv "
                       "layers, 32 channels, bf16 weights, fp32 accumulation, trained on 2^20 Gibbs samples "
                       "(4096 chains annealed 5->T over 2e4 sweeps, 256 snapshots 20 sweeps apart, translation "
                       "and transpose augmentation); 8192 chains, 1 MH : 10 Gibbs vs plain Gibbs at equal wall "
                       "time, seeded +-1 start, first 20% discarded",
           "reference": "exact <E>/N by 12x12 row transfer matrix",
           "ess": "energy ESS (ess_per_s) and min over {energy, O_1/3 = max |S(q*)|^2/N^2} (ess_min_per_s)",
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
        r.update({"T": T, "E_ref": ref[T], "data_s": t_data, "train_s": t_train, "train_steps": steps,
                  "final_loss_per_site": loss,
                  "ess_ratio": r["learned"]["ess_per_s"] / r["gibbs"]["ess_per_s"],
                  "ess_min_ratio": r["learned"]["ess_min_per_s"] / r["gibbs"]["ess_min_per_s"]})
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
    r.update({"workload": f"SS Ising {L}x{L}, the 64 scale points (4 phase-boundary lines, T ~ logU[0.1, 1]), "
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    ap.add_argument("--c5-mh-96", action="store_true", help="also run the conditional learned-MH comparison at 96x96")
    ap.add_argument("--no-tts", action="store_true", help="skip the time-to-solution runs at the four phase points")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the m(h) comparison of the default and the hardware precision")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1): chains are independent, and sharding them over "
              "several GPUs is a design, not an implemented path.", file=sys.stderr)
        sys.exit(2)

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
    insts = instances(crbm)
    t0 = time.perf_counter()
    smp = crbm.Sampler(insts, seed=SEED, n_sweeps=S, measure_every=1, burn_in=S - 1)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    init_spins, _ = smp.get_state()
    n_sweeps = min(args.sweeps, S)
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

    chains = smp.total_chains
    ms = float(np.mean(step_ms))
    value = chains * n_sweeps * L * L / (ms / 1e3)
    kms = float(np.mean(kern_ms))
    achieved = chains * n_sweeps * L * L * OPS_PER_SPIN_SWEEP / (kms / 1e3)
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "SS Ising 18x18 periodic, J1=1, J2/J1 in {0.5,1.0,1.5,2.0} x 16 h/J1 in [0,3], "
                        "4096 chains per point (262144 chains), geometric anneal T 5.0->0.05 over 10^4 sweeps, "
                        "16.16 fixed point, seeded +-1 start",
            "L": L, "points": len(insts), "chains": chains, "sweeps": n_sweeps,
            "node_updates_per_s": value * 3.5,
            "create_and_tables_ms": create_ms,
            "tiling": {"rows_per_lane": rows, "lanes_per_chain": (L // 2) // rows, "waves_per_block": wpb,
                       "autotuned": tuning is not None},
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": ALU_PEAK_OPS / 1e12,
            "unit": "TOP/s",
            "frac": achieved / ALU_PEAK_OPS,
            "traffic": measured_traffic() if n_sweeps == S else None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)",
            "kernel": f"gibbs_kernel<{L},{rows}>",
            "kernel_ms": kms,
            "ops_per_spin_sweep": OPS_PER_SPIN_SWEEP,
        },
    }
    if obs is not None:
        E = np.array([o["E_per_spin"] for o in obs]).reshape(4, 16)
        m = np.array([o["m"] for o in obs]).reshape(4, 16)
        result["final_state"] = {"J2": list(J2S), "E_per_spin_mean": E.round(5).tolist(),
                                 "m_mean": m.round(5).tolist()}
    if not args.no_batched:
        result["batched_uneven"] = batched_uneven(crbm, torch)
    if not args.no_scale:
        result["scale"] = scale_gibbs(crbm, torch)
    if not args.no_tts:
        result["tts"] = tts_leg(crbm, torch)
    if not args.no_precision:
        result["precision"] = precision_leg(crbm, torch)
    if not args.no_mh:
        result["learned_mh"] = learned_mh(crbm, torch)
    if not args.no_c5_mh:
        result["learned_mh_points"] = {"48": learned_points(crbm, torch, 48)}
        if args.c5_mh_96:
            result["learned_mh_points"]["96"] = learned_points(crbm, torch, 96, steps=200, cycles=20)
    if not args.no_cpu_baseline and n_sweeps == S:
        base, finals = cpu_baseline()
        result["cpu_baseline"] = base
        # the sampled oracle chains double as a parity check of this very run
        spins, _ = smp.get_state()
        parts = smp.split_spins(spins.cpu())
        result["cpu_baseline"]["parity_sampled_chains"] = all(
            np.array_equal(parts[i][ch].numpy(), s) for (i, ch), s in finals.items())
    print(json.dumps(result))


if __name__ == "__main__":
    main()
