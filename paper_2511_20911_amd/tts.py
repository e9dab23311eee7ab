"""Time-to-solution (Sec. III.C Eq. (14)) of the GPU Gibbs sampler.

A run is one chain started from its seeded +-1 state and sampled at a
constant temperature, or along a geometric anneal down to it.  For each run the device keeps the lowest energy seen
after any sweep and the sweep at which it was first reached (crbm_min_energy
over the counts trace, folded chunk by chunk so that long runs need no long
trace).  With the exact ground-state energy E_gs:

- p_gnd is the fraction of runs whose minimum equals E_gs;
- T is the mean first-hit time of those runs;
- TTS_l = T log(1 - l/100) / log(1 - p_gnd), or T itself when every run
  succeeds (TTS_100).

E_gs is the lowest of the four ordered states of the phase diagram
(Sec. III.A): ferromagnet, Neel, antiparallel dimers, and the UUD 1/3 plateau.
Each is computed exactly in 2^-16 units from its integer bond counts on the
periodic lattice (L a multiple of 6).  A run found below E_gs raises, since it
would contradict the candidate set.

Times are reported in sweeps, and from the device time of the whole batch of
runs: per sweep for one run sharing the GPU with the batch (latency), and per
run-sweep (amortised over the batch).
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import Instance, Sampler, min_energy

# (M, B1, B2) of each ordered state as fractions of N: spins, J1 bonds (2N),
# dimers (N/2)
_ORDERED = {
    "fm": ((1, 1), (2, 1), (1, 2)),
    "neel": ((0, 1), (-2, 1), (1, 2)),
    "dimer": ((0, 1), (0, 1), (-1, 2)),
    "one_third": ((1, 3), (-2, 3), (-1, 6)),
}


def quantise(x: float) -> int:
    """16.16 fixed point, rounded to nearest (ties away from zero)."""
    y = x * 65536.0
    return int(math.floor(abs(y) + 0.5)) * (1 if y >= 0 else -1)


def ordered_ground_state(L: int, J1: float, J2: float, h: float):
    """(phase, E_q) of the lowest ordered state, E_q = H in 2^-16 units from the
    quantised couplings (L a multiple of 6 so that every state fits)."""
    if L % 6:
        raise ValueError("the ordered states need L to be a multiple of 6")
    N = L * L
    J1q, J2q, hq = quantise(J1), quantise(J2), quantise(h)
    best = None
    for phase, ((mn, md), (b1n, b1d), (b2n, b2d)) in _ORDERED.items():
        M, B1, B2 = N * mn // md, N * b1n // b1d, N * b2n // b2d
        Eq = J1q * B1 + J2q * B2 - hq * M
        if best is None or Eq < best[1]:
            best = (phase, Eq)
    return best


def tts_from_runs(emin, first, e_gs_q: int, level: float = 99.0):
    """p_gnd, mean first-hit sweep T over the successful runs, and TTS_l in
    sweeps (inf when no run succeeds)."""
    emin = np.asarray(emin, np.int64)
    first = np.asarray(first, np.int64)
    if (emin < e_gs_q).any():
        raise RuntimeError("a run went below the ground-state energy of the ordered phases")
    hit = emin == e_gs_q
    p = float(hit.mean()) if emin.size else 0.0
    if not hit.any():
        return {"p_gnd": 0.0, "T_sweeps": None, "tts_sweeps": math.inf, "runs": int(emin.size)}
    T = float(first[hit].mean())
    t = T if p >= 1.0 else T * math.log(1.0 - level / 100.0) / math.log(1.0 - p)
    return {"p_gnd": p, "T_sweeps": T, "tts_sweeps": t, "runs": int(emin.size),
            "first_hit_median": float(np.median(first[hit])), "first_hit_max": int(first[hit].max())}


def runs(L: int, J1: float, J2: float, h: float, T: float, n_chains: int, n_sweeps: int, seed: int,
         id: int = 0, chunk: int = 2000, stream=None, anneal_from: Optional[float] = None):
    """n_chains independent runs of n_sweeps sweeps, at constant temperature T
    or (anneal_from given) on the geometric anneal anneal_from -> T.  Returns
    (emin, first) as host int64 arrays and the device seconds of the runs
    (sampling, trace and the minimum fold)."""
    import torch

    if anneal_from is None:
        inst = Instance(L=L, J1=J1, J2=J2, h=h, n_chains=n_chains, sched="const", T0=T, T1=T, id=id)
    else:
        inst = Instance(L=L, J1=J1, J2=J2, h=h, n_chains=n_chains, sched="geometric", T0=anneal_from, T1=T, id=id)
    smp = Sampler([inst], seed=seed, n_sweeps=n_sweeps, stream=stream)
    w = (-quantise(h), quantise(J1), quantise(J2))
    chunk = max(1, min(chunk, n_sweeps))
    trace = torch.empty((chunk, n_chains, 3), dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream() if stream is None else stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    emin = first = None
    ev0.record(st)
    for s0 in range(0, n_sweeps, chunk):
        n = min(chunk, n_sweeps - s0)
        smp.sample(n, trace=trace[:n])
        emin, first = min_energy(trace[:n], w, sweep0=s0, emin=emin, first=first, stream=st)
    ev1.record(st)
    ev1.synchronize()
    seconds = ev0.elapsed_time(ev1) / 1e3
    out = emin.cpu().numpy(), first.cpu().numpy(), seconds
    smp.close()
    return out


def phase_tts(L: int, J2: float, h: float, temps, n_chains: int, n_sweeps: int, seed: int, id: int = 0,
              level: float = 99.0, anneal_from: Optional[float] = None):
    """TTS_l at one phase point (J1 = 1) for each (final) temperature of
    `temps`, constant or annealed from anneal_from; returns the
    per-temperature results and the best (lowest TTS) one."""
    phase, e_gs = ordered_ground_state(L, 1.0, J2, h)
    res = []
    for k, T in enumerate(temps):
        emin, first, sec = runs(L, 1.0, J2, h, T, n_chains, n_sweeps, seed, id=id + k, anneal_from=anneal_from)
        r = tts_from_runs(emin, first, e_gs, level)
        lat = sec / n_sweeps                 # one sweep of the whole batch
        amort = sec / (n_sweeps * n_chains)  # per run-sweep
        r.update({"T": T, "anneal_from": anneal_from, "device_s": sec, "sweep_latency_s": lat, "run_sweep_s": amort,
                  "tts_latency_s": r["tts_sweeps"] * lat if math.isfinite(r["tts_sweeps"]) else math.inf,
                  "tts_amortised_s": r["tts_sweeps"] * amort if math.isfinite(r["tts_sweeps"]) else math.inf})
        res.append(r)
    best = min(res, key=lambda r: r["tts_sweeps"])
    return {"phase": phase, "L": L, "J2": J2, "h": h, "E_gs_per_spin": e_gs / 65536.0 / (L * L),
            "chains": n_chains, "sweeps": n_sweeps, "best": best, "by_T": res}
