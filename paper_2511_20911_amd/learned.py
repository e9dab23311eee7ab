"""Learned independent-Metropolis-Hastings proposal: training set, training
loop and the comparison with plain Gibbs sampling.

The proposal network, its training kernels and the MH step live in the HIP
library (crbm_ar_* and crbm_sample_mh); this module only orchestrates them
and moves data between device tensors:

* training_set: configurations drawn by the library's own Gibbs sampler
  (geometric anneal to the target temperature, then spaced snapshots at it);
* train: a training run in the library (crbm_ar_train): Adam steps of its
  fused forward / backward kernels on minibatches it draws on the device,
  each moved by a symmetry of the periodic Shastry-Sutherland lattice with
  the dimer layout of Fig. 1a (translations by two sites in either direction,
  the transpose (r, c) -> (c, r));
* compare: learned MH (1 MH step per `gibbs_per_mh` Gibbs sweeps) against
  plain Gibbs given the same wall-clock time, both from the same seeded start,
  with tau_int / ESS of the energy and of the plateau order parameter
  O_1/3 = max |S(q*)|^2 / N^2 (q* = (pi, 2pi/3), (2pi/3, pi); Sec. III.B) from
  the library's estimator;
* sector_moves: how often each sampler moves a chain between the plateau's
  six degenerate ground states (plateau_sectors, from the phases of the two
  structure-factor amplitudes), which E and O_1/3 cannot see.

Many points at once (the phase-boundary workloads): one conditional network
(bias offsets from an MLP of each point's features) serves every point of a
multi-instance handle: training_set_points, train_points and compare_points
mirror the single-point functions, with per-point energies, tau_int of E and
m, ESS and the 3-SE agreement of the two samplers.

The paper samples its CRBM by Gibbs only (Sec. II.B); the learned proposal is
an addition that leaves the stationary law unchanged (exact MH acceptance on
integer bond counts).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

from . import ARNet, Instance, Sampler, sample_mh, tau_int


def energy_weights(J1: float, J2: float, h: float):
    """(w_M, w_B1, w_B2) such that w . (M, B1, B2) = H in 2^-16 units (16.16 couplings)."""
    q = lambda x: int(round(x * 65536.0))
    return (-q(h), q(J1), q(J2))


def training_set(L, J1, J2, h, T, n_chains=4096, anneal_sweeps=20000, snapshots=256, spacing=20,
                 seed=77, T_start=5.0, id=1):
    """Gibbs samples at temperature T: a geometric anneal T_start -> T over
    anneal_sweeps sweeps, then `snapshots` states of every chain spaced by
    `spacing` sweeps at T.  Returns an int8 CUDA tensor [snapshots * n_chains, L, L]."""
    import torch
    N = L * L
    ann = Sampler([Instance(L=L, J1=J1, J2=J2, h=h, n_chains=n_chains, sched="geometric", T0=T_start, T1=T,
                            id=id)], seed=seed, n_sweeps=anneal_sweeps)
    ann.sample(anneal_sweeps)
    st, _ = ann.get_state()
    fixed = Sampler([Instance(L=L, J1=J1, J2=J2, h=h, n_chains=n_chains, sched="const", T0=T, id=id)],
                    seed=seed + 1, n_sweeps=snapshots * spacing)
    fixed.set_state(st, 0)
    out = torch.empty((snapshots, n_chains * N), dtype=torch.int8, device="cuda")
    for k in range(snapshots):
        fixed.sample(spacing, spins_out=out[k])
    return out.view(-1, L, L)


def train(net: ARNet, data, steps=800, batch=1024, lr=1e-3, lr_late=3e-4, late_from=0.625, seed=1):
    """Maximum-likelihood training in the library (crbm_ar_train): minibatches
    drawn on the device with random lattice symmetries (even translations,
    transpose).  Returns the per-site loss of the last step."""
    N = data.shape[1] * data.shape[2]
    return net.train(data.contiguous(), steps, batch=batch, lr=lr, lr_late=lr_late, late_from=late_from,
                     seed=seed) / N


@dataclass
class ChainStats:
    E_per_spin: float      # mean over chains and kept samples
    se: float              # standard error of <E>/N from the spread of the chain means
    tau: float             # integrated autocorrelation time of the energy (in samples)
    ess: float             # energy effective sample size (chains x kept samples / tau)
    O: float               # mean plateau order parameter O_1/3 = max |S(q*)|^2 / N^2
    O_se: float
    tau_O: float           # integrated autocorrelation time of O_1/3
    ess_min: float         # chains x kept samples / max(tau, tau_O)
    seconds: float         # wall time of the sampling phase
    m: float = 0.0         # mean magnetisation per spin
    m_se: float = 0.0      # its standard error from the spread of the chain means


def _stats(trace, order, weights, N, discard, seconds, max_lag):
    t = trace[discard:].double()
    E = (weights[0] * t[..., 0] + weights[1] * t[..., 1] + weights[2] * t[..., 2]) / 65536.0 / N
    cm = E.mean(0)
    tau, ess, _, _ = tau_int(trace, weights, discard=discard, max_lag=max_lag)
    o = order[discard:, :, 0].double() / float(N * N)
    om = o.mean(0)
    tau_o, _, _, _ = tau_int(order, (1, 0, 0), discard=discard, max_lag=max_lag)
    mm = (t[..., 0] / N).mean(0)
    n_kept = t.shape[0] * t.shape[1]
    return ChainStats(float(cm.mean()), float(cm.std() / math.sqrt(cm.numel())), tau, ess, float(om.mean()),
                      float(om.std() / math.sqrt(om.numel())), tau_o, n_kept / max(tau, tau_o), seconds,
                      float(mm.mean()), float(mm.std() / math.sqrt(mm.numel())))


def compare(net: ARNet, L, J1, J2, h, T, n_chains=8192, cycles=500, gibbs_per_mh=10, trace_every=50,
            seed=123, id=0):
    """Learned MH (cycles of gibbs_per_mh Gibbs sweeps + one MH step) against
    plain Gibbs run for the same wall time, both from the same seeded start;
    the first fifth of each run is discarded as burn-in.  Returns a dict with
    both samplers' energy statistics and ESS per second."""
    import torch
    N = L * L
    w = energy_weights(J1, J2, h)
    inst = Instance(L=L, J1=J1, J2=J2, h=h, n_chains=n_chains, sched="const", T0=T, id=id)
    mh = Sampler([inst], seed=seed, n_sweeps=max(1, cycles * gibbs_per_mh))
    tr = torch.empty((cycles, n_chains, 3), dtype=torch.int32, device="cuda")
    od = torch.empty_like(tr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc = sample_mh(mh, net, cycles, gibbs_per_mh, trace=tr, order=od)
    torch.cuda.synchronize()
    t_mh = time.perf_counter() - t0
    learned = _stats(tr, od, w, N, cycles // 5, t_mh, cycles // 2)
    del tr, od, mh
    # Gibbs sweep time at this size, then a run of the same wall time
    probe = Sampler([inst], seed=seed, n_sweeps=1100)
    probe.sample(100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    probe.sample(1000)
    torch.cuda.synchronize()
    per_sweep = (time.perf_counter() - t0) / 1000
    del probe
    n_s = max(10, int(t_mh / per_sweep) // trace_every)
    sweeps = n_s * trace_every
    gb = Sampler([inst], seed=seed, n_sweeps=sweeps)
    trg = torch.empty((n_s, n_chains, 3), dtype=torch.int32, device="cuda")
    odg = torch.empty_like(trg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gb.sample(sweeps, trace=trg, trace_every=trace_every, order=odg)
    torch.cuda.synchronize()
    t_g = time.perf_counter() - t0
    gibbs = _stats(trg, odg, w, N, n_s // 5, t_g, n_s // 2)
    return {
        "learned": {"cycles": cycles, "gibbs_per_mh": gibbs_per_mh, "acceptance": acc / (cycles * n_chains),
                    "ms_per_cycle": 1e3 * t_mh / cycles, **learned.__dict__,
                    "ess_per_s": learned.ess / t_mh, "ess_min_per_s": learned.ess_min / t_mh,
                    "tau_unit": "MH cycles"},
        "gibbs": {"sweeps": sweeps, "trace_every": trace_every, "us_per_sweep": 1e6 * per_sweep,
                  **gibbs.__dict__, "ess_per_s": gibbs.ess / t_g, "ess_min_per_s": gibbs.ess_min / t_g,
                  "tau_unit": f"{trace_every} sweeps"},
    }


def plateau_sectors(spins, threshold=0.05):
    """Ordering sector of each configuration [n, L, L] (+-1; L a multiple of
    6) on the 1/3 plateau, from the two structure-factor amplitudes of Sec.
    III.B Eq. (13): S_A = sum s(r, c) e^{i(pi r + 2 pi c / 3)} and S_B = sum
    s(r, c) e^{i(2 pi r / 3 + pi c)}.  Returns (orientation, phase, ordered):
    0 where |S_A| >= |S_B| else 1, the argument of the larger amplitude, and
    whether max |S|^2 / N^2 reaches `threshold` (an ordered state has about
    1/3, a disordered one about 1/N).  The six plateau ground states (three
    translations by two columns or rows, and the transpose) differ in
    orientation or by 2 pi / 3 in phase."""
    import numpy as np
    s = np.asarray(spins, dtype=np.float64)
    n, L = s.shape[0], s.shape[1]
    r = np.arange(L)[:, None]
    c = np.arange(L)[None, :]
    pa = np.exp(1j * (np.pi * r + 2.0 * np.pi * c / 3.0))
    pb = np.exp(1j * (2.0 * np.pi * r / 3.0 + np.pi * c))
    flat = s.reshape(n, L * L)
    sa = flat @ pa.reshape(-1)
    sb = flat @ pb.reshape(-1)
    orient = (np.abs(sb) > np.abs(sa)).astype(np.int8)
    amp = np.where(orient == 0, sa, sb)
    order = np.abs(amp) ** 2 / float(L * L) ** 2
    return orient, np.angle(amp), order >= threshold


def sector_changes(prev, cur):
    """Per chain, whether the ordering sector changed between two
    plateau_sectors results: both states ordered, and a different
    orientation or a phase step of more than pi / 3 (sectors are 2 pi / 3
    apart; thermal fluctuations of an ordered state move the phase far less)."""
    import numpy as np
    o0, p0, k0 = prev
    o1, p1, k1 = cur
    dp = np.angle(np.exp(1j * (p1 - p0)))
    return k0 & k1 & ((o0 != o1) | (np.abs(dp) > np.pi / 3.0))


def sector_moves(net: ARNet, L, J1, J2, h, T, n_chains=1024, warm_cycles=40, steps=100, gibbs_per_mh=10,
                 seed=777, id=0):
    """Tunnelling between the plateau's degenerate ground states, which the
    energy and O_1/3 do not see (both are the same in all six).  Learned MH
    runs warm_cycles cycles from a seeded start; plain Gibbs then starts from
    the same states (its own seed), and both run `steps` steps: one cycle
    (gibbs_per_mh sweeps + one MH step) or gibbs_per_mh sweeps.  After every
    step each chain's sector is taken from its state on the host.  Returns,
    per sampler, sector changes per chain and step, the fraction of chains
    that changed sector at least once, and the mean fraction of ordered
    states.  Untimed: the per-second rates follow from the timed comparison's
    cycle and sweep times."""
    import numpy as np
    import torch
    inst = Instance(L=L, J1=J1, J2=J2, h=h, n_chains=n_chains, sched="const", T0=T, id=id)
    total = (warm_cycles + steps) * gibbs_per_mh
    mh = Sampler([inst], seed=seed, n_sweeps=total)
    sample_mh(mh, net, warm_cycles, gibbs_per_mh)
    start, idx = mh.get_state()
    gb = Sampler([inst], seed=seed + 1, n_sweeps=total)
    gb.set_state(start, idx)

    def host(sp):
        return sp.view(n_chains, L, L).cpu().numpy()

    out = {}
    for name in ("learned", "gibbs"):
        prev = plateau_sectors(host(start))
        moved = np.zeros(n_chains, dtype=np.int64)
        ordered = float(prev[2].mean())
        for _ in range(steps):
            if name == "learned":
                sample_mh(mh, net, 1, gibbs_per_mh)
                sp, _ = mh.get_state()
            else:
                gb.sample(gibbs_per_mh)
                sp, _ = gb.get_state()
            cur = plateau_sectors(host(sp))
            moved += sector_changes(prev, cur)
            ordered += float(cur[2].mean())
            prev = cur
        out[name] = {"changes_per_chain_step": float(moved.mean()) / steps,
                     "chains_changed": float((moved > 0).mean()),
                     "ordered_fraction": ordered / (steps + 1)}
    torch.cuda.synchronize()
    out.update({"steps": steps, "chains": n_chains, "warm_cycles": warm_cycles,
                "step": f"learned: {gibbs_per_mh} Gibbs sweeps + 1 MH step; gibbs: {gibbs_per_mh} sweeps"})
    return out


# ---------------------------------------------------------------- many points, one conditional network

def features(J2, h, T):
    """Conditioning features of a point (J1 = 1): (J2/J1, h/(4 J1), ln T)."""
    return (float(J2), float(h) / 4.0, math.log(float(T)))


def training_set_points(points, L, chains, anneal_sweeps=4000, snapshots=32, spacing=50, seed=91, T_start=5.0,
                        id0=200):
    """Gibbs samples at every point (J2, h, T): one handle anneals all points
    geometrically from T_start to their own T, then `snapshots` states of
    every chain spaced by `spacing` sweeps at that T.  Returns (spins int8
    CUDA [snapshots * len(points) * chains, L, L], point index int32 CUDA
    [same])."""
    import torch
    N = L * L
    ann = Sampler([Instance(L=L, J1=1.0, J2=J2, h=h, n_chains=chains, sched="geometric", T0=T_start, T1=T,
                            id=id0 + k) for k, (J2, h, T) in enumerate(points)], seed=seed, n_sweeps=anneal_sweeps)
    ann.sample(anneal_sweeps)
    st, _ = ann.get_state()
    fixed = Sampler([Instance(L=L, J1=1.0, J2=J2, h=h, n_chains=chains, sched="const", T0=T, id=id0 + k)
                     for k, (J2, h, T) in enumerate(points)], seed=seed + 1, n_sweeps=snapshots * spacing)
    fixed.set_state(st, 0)
    total = len(points) * chains
    out = torch.empty((snapshots, total * N), dtype=torch.int8, device="cuda")
    for k in range(snapshots):
        fixed.sample(spacing, spins_out=out[k])
    pts = torch.arange(len(points), dtype=torch.int32, device="cuda").repeat_interleave(chains).repeat(snapshots)
    return out.view(-1, L, L), pts


def train_points(net: ARNet, data, pts, steps=600, batch=512, lr=1e-3, lr_late=3e-4, late_from=0.625, seed=1):
    """Maximum-likelihood training of a conditional network in the library on
    minibatches that mix the points.  Returns the last per-site loss."""
    N = data.shape[1] * data.shape[2]
    return net.train(data.contiguous(), steps, batch=batch, lr=lr, lr_late=lr_late, late_from=late_from, seed=seed,
                     points=pts.contiguous()) / N


def _point_stats(trace, c0, c1, weights, N, discard, max_lag):
    """<E>/N, its SE over chains, tau_int of E and of m, for chains [c0, c1)."""
    t = trace[discard:, c0:c1].double()
    E = (weights[0] * t[..., 0] + weights[1] * t[..., 1] + weights[2] * t[..., 2]) / 65536.0 / N
    cm = E.mean(0)
    tau_e = tau_int(trace, weights, c0=c0, c1=c1, discard=discard, max_lag=max_lag)[0]
    tau_m = tau_int(trace, (1, 0, 0), c0=c0, c1=c1, discard=discard, max_lag=max_lag)[0]
    return float(cm.mean()), float(cm.std() / math.sqrt(cm.numel())), tau_e, tau_m


def compare_points(net: ARNet, points, L, chains, cycles=100, gibbs_per_mh=10, trace_every=10, seed=321, id0=400):
    """Learned MH (cycles of gibbs_per_mh Gibbs sweeps + one MH step, each
    point's chains proposing at that point) against plain Gibbs run for the
    same wall time, both from the same seeded start over all points in one
    handle; the first fifth of each run is discarded.  Per point: <E>/N with
    SE, tau_int of E and m, ESS = chains x kept / max(tau_E, tau_m); totals
    over points; and whether the two samplers agree within 3 combined SE."""
    import torch
    N = L * L
    insts = [Instance(L=L, J1=1.0, J2=J2, h=h, n_chains=chains, sched="const", T0=T, id=id0 + k)
             for k, (J2, h, T) in enumerate(points)]
    n = chains * len(points)
    mh = Sampler(insts, seed=seed, n_sweeps=max(1, cycles * gibbs_per_mh))
    tr = torch.empty((cycles, n, 3), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc = sample_mh(mh, net, cycles, gibbs_per_mh, trace=tr)
    torch.cuda.synchronize()
    t_mh = time.perf_counter() - t0
    del mh
    probe = Sampler(insts, seed=seed, n_sweeps=60)
    probe.sample(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    probe.sample(50)
    torch.cuda.synchronize()
    per_sweep = (time.perf_counter() - t0) / 50
    del probe
    n_s = max(10, int(t_mh / per_sweep) // trace_every)
    sweeps = n_s * trace_every
    gb = Sampler(insts, seed=seed, n_sweeps=sweeps)
    trg = torch.empty((n_s, n, 3), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gb.sample(sweeps, trace=trg, trace_every=trace_every)
    torch.cuda.synchronize()
    t_g = time.perf_counter() - t0
    rows, ess_l, ess_g, agree = [], 0.0, 0.0, 0
    for k, (J2, h, T) in enumerate(points):
        w = energy_weights(1.0, J2, h)
        c0, c1 = k * chains, (k + 1) * chains
        El, sel, tel, tml = _point_stats(tr, c0, c1, w, N, cycles // 5, cycles // 2)
        Eg, seg, teg, tmg = _point_stats(trg, c0, c1, w, N, n_s // 5, n_s // 2)
        el = chains * (cycles - cycles // 5) / max(tel, tml)
        eg = chains * (n_s - n_s // 5) / max(teg, tmg)
        ess_l += el
        ess_g += eg
        ok = abs(El - Eg) <= 3.0 * math.sqrt(sel * sel + seg * seg) + 1e-12
        agree += ok
        rows.append({"J2": J2, "h": h, "T": T, "E_learned": El, "se_learned": sel, "tau_E_learned": tel,
                     "tau_m_learned": tml, "E_gibbs": Eg, "se_gibbs": seg, "tau_E_gibbs": teg, "tau_m_gibbs": tmg,
                     "agree_3se": bool(ok)})
    return {
        "learned": {"cycles": cycles, "gibbs_per_mh": gibbs_per_mh, "acceptance": acc / (cycles * n),
                    "ms_per_cycle": 1e3 * t_mh / cycles, "seconds": t_mh, "ess_min_per_s": ess_l / t_mh,
                    "tau_unit": "MH cycles"},
        "gibbs": {"sweeps": sweeps, "trace_every": trace_every, "us_per_sweep": 1e6 * per_sweep, "seconds": t_g,
                  "ess_min_per_s": ess_g / t_g, "tau_unit": f"{trace_every} sweeps"},
        "points_agreeing_within_3se": agree,
        "points": rows,
    }
