"""Phase-diagram and structure-factor experiments (Sec. III.A-B) on top of the
library's samplers: the magnetisation map m(J2/J1, h) of Fig. 3a with its
transition lines, laterally confined lattices (Fig. 3f) and the static
structure factor S(q) of Eq. (13).

Everything here is orchestration and host post-processing of the exact
integer sums the library returns (crbm_observables, crbm_lattice_observables);
no sampling arithmetic lives in this module.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

from . import Instance, Lattice, LatticeSampler, Sampler, ss_filters


def structure_factor(cn, n_samples: int, rows: int, cols: int, qr, qc) -> np.ndarray:
    """S(q)/N^2 on the grid qr x qc (radians per lattice spacing, rows and
    columns) from the displacement correlation sums Cn[dr, dc + cols - 1]
    (0 <= dr < rows, -cols < dc < cols, pairs inside the lattice) over
    n_samples states: S(q) = sum_{i,j} <s_i s_j> e^{i q.(R_i - R_j)}
    (Eq. (13)) = sum over displacements d of <Cn(d)> e^{i q.d} with
    Cn(-d) = Cn(d); divided by N^2 it is 1 for a perfectly ordered state at
    its own wave vector."""
    C = np.asarray(cn, np.float64).reshape(rows, 2 * cols - 1) / float(n_samples)
    dr = np.arange(rows)[:, None]
    dc = np.arange(-(cols - 1), cols)[None, :]
    # half-space d > 0 (dr > 0, or dr = 0 and dc > 0) counted twice, d = 0 once
    w = np.where((dr > 0) | ((dr == 0) & (dc > 0)), 2.0, 0.0) + np.where((dr == 0) & (dc == 0), 1.0, 0.0)
    Cw = C * w
    qr = np.asarray(qr, np.float64)
    qc = np.asarray(qc, np.float64)
    Er = np.cos(qr[:, None, None] * dr[None, :, :])          # [nqr, rows, 1]
    Sr = np.sin(qr[:, None, None] * dr[None, :, :])
    Ec = np.cos(qc[:, None, None] * dc[None, :, :])          # [nqc, 1, 2 cols - 1]
    Scs = np.sin(qc[:, None, None] * dc[None, :, :])
    # cos(a + b) = cos a cos b - sin a sin b, summed over displacements
    S = np.einsum("ird,jrd->ij", Er * Cw[None], np.broadcast_to(Ec, (len(qc), rows, 2 * cols - 1))) - \
        np.einsum("ird,jrd->ij", Sr * Cw[None], np.broadcast_to(Scs, (len(qc), rows, 2 * cols - 1)))
    N = rows * cols
    return S / (N * N)


def boundaries_T0(J2: float, h_max: float = 8.0):
    """Fields of the T = 0 transitions of the SS Ising model at J2/J1 (J1 = 1)
    for h in (0, h_max], from the energies per spin of the four ordered
    phases of Sec. III.A: FM 2 + J2/2 - h, Neel -2 + J2/2, antiparallel
    dimers -J2/2, UUD 1/3 plateau -2/3 - J2/6 - h/3.  Returns the sorted
    fields where the lowest of them changes."""
    hs = np.linspace(1e-6, h_max, 80001)
    E = np.stack([2 + J2 / 2 - hs, np.full_like(hs, -2 + J2 / 2), np.full_like(hs, -J2 / 2),
                  -2 / 3 - J2 / 6 - hs / 3])
    g = np.argmin(E, axis=0)
    out = []
    for k in np.nonzero(np.diff(g))[0]:
        a, b = g[k], g[k + 1]
        # exact crossing of the two lines
        sl = [-1.0, 0.0, 0.0, -1.0 / 3.0]
        c0 = [2 + J2 / 2, -2 + J2 / 2, -J2 / 2, -2 / 3 - J2 / 6]
        out.append((c0[b] - c0[a]) / (sl[a] - sl[b]))
    return sorted(out)


def phase_map(J2s: Sequence[float], hs: Sequence[float], L: int = 18, chains: int = 32, T: float = 0.1,
              T_start: float = 3.0, anneal: int = 1000, measure: int = 500, seed: int = 0x5EED00000000F100,
              id0: int = 5000):
    """<m> at every (J2/J1, h) point (J1 = 1) of an L x L periodic lattice, all
    points in one handle: geometric anneal T_start -> T, then `measure`
    measured sweeps at T (the protocol of Sec. III.A with a fixed final T).
    Returns m [len(J2s), len(hs)] and the handle's device time."""
    import time
    import torch
    sched = np.concatenate([T_start * (T / T_start) ** (np.arange(anneal) / (anneal - 1)), np.full(measure, T)])
    insts = [Instance(L=L, J1=1.0, J2=J2, h=h, n_chains=chains, sched="explicit", T_explicit=sched,
                      id=id0 + a * len(hs) + b) for a, J2 in enumerate(J2s) for b, h in enumerate(hs)]
    smp = Sampler(insts, seed=seed, n_sweeps=anneal + measure, measure_every=1, burn_in=anneal)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    smp.sample(anneal + measure)
    obs = smp.observables()
    dt = time.perf_counter() - t0
    m = np.array([o["m"] for o in obs]).reshape(len(J2s), len(hs))
    E = np.array([o["E_per_spin"] for o in obs]).reshape(len(J2s), len(hs))
    smp.close()
    return m, E, dt, sum(I.n_chains for I in insts) * L * L * (anneal + measure)


def transition_fields(hs, m, min_step: float = 0.1):
    """Fields of the steps of a magnetisation curve: local maxima of dm/dh
    (central differences) whose step in m over the neighbouring half-way
    points is at least min_step, refined by a parabola through the peak."""
    hs = np.asarray(hs, np.float64)
    m = np.asarray(m, np.float64)
    d = np.gradient(m, hs)
    out = []
    for k in range(1, len(hs) - 1):
        if d[k] >= d[k - 1] and d[k] > d[k + 1] and d[k] * (hs[k + 1] - hs[k - 1]) / 2 >= min_step / 2:
            lo, hi = max(0, k - 2), min(len(hs) - 1, k + 2)
            if m[hi] - m[lo] < min_step:
                continue
            a, b, c = d[k - 1], d[k], d[k + 1]
            den = a - 2 * b + c
            off = 0.5 * (a - c) / den if den != 0 else 0.0
            out.append(float(hs[k] + off * (hs[k + 1] - hs[k])))
    return out


def confined_scan(hs: Sequence[float], width: int = 12, length: int = 18, J2: float = 1.5, T: float = 0.2,
                  chains: int = 512, anneal: int = 4000, measure: int = 2000, every: int = 4, T_start: float = 5.0,
                  seed: int = 0x5EED00000000F200, id0: int = 6000, nq: int = 48, open_cols: bool = True):
    """Laterally confined SS lattices (Sec. III.A-B, Fig. 3f, Fig. 4b,d):
    `width` columns open, `length` rows periodic, J2/J1 = J2, one field per
    point; geometric anneal T_start -> T, then `measure` sweeps at T with the
    counts and the displacement correlation accumulated every `every`
    sweeps.  Per field: <E>/N, <m>, and S(q)/N^2 on an nq x nq grid of
    q in [0, 2 pi)^2 (rows, columns), its maximum and where it lies, and its
    values at the UUD wave vectors (pi, 2 pi/3), (2 pi/3, pi) and at Gamma.
    open_cols=False gives the periodic lattice of the same size, for comparison."""
    import time
    import torch
    sched = np.concatenate([T_start * (T / T_start) ** (np.arange(anneal) / (anneal - 1)), np.full(measure, T)])
    lats = [Lattice(rows=length, cols=width, J=ss_filters(1.0, J2), h_even=h, open_cols=open_cols, n_chains=chains,
                    sched="explicit", T_explicit=sched, id=id0 + k) for k, h in enumerate(hs)]
    smp = LatticeSampler(lats, seed=seed, n_sweeps=anneal + measure, measure_every=every, burn_in=anneal, corr=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    smp.sample(anneal + measure)
    acc, cn = smp.observables()
    dt = time.perf_counter() - t0
    qs = 2 * math.pi * np.arange(nq) / nq
    N = width * length
    Jq = np.array([round(x * 65536.0) for x in ss_filters(1.0, J2)], np.float64)
    rows = []
    for k, h in enumerate(hs):
        n = int(acc[k, 0])
        E = (acc[k, 3:13].astype(np.float64) @ Jq - round(h * 65536.0) * float(acc[k, 1] + acc[k, 2])) / 65536.0 / n / N
        S = structure_factor(cn[k], n, length, width, qs, qs)
        i, j = np.unravel_index(np.argmax(S), S.shape)
        Sx = S.copy()
        Sx[0, 0] = -1.0  # strongest peak away from Gamma (Gamma carries <M^2>/N^2)
        ix, jx = np.unravel_index(np.argmax(Sx), Sx.shape)
        pts = structure_factor(cn[k], n, length, width, [math.pi, 2 * math.pi / 3, 0.0],
                               [2 * math.pi / 3, math.pi, 0.0])
        rows.append({"h": float(h), "E_per_spin": float(E), "m": float(acc[k, 1] + acc[k, 2]) / n / N,
                     "S_max": float(S.max()), "q_max": [float(qs[i]), float(qs[j])],
                     "S_max_off_gamma": float(Sx.max()), "q_max_off_gamma": [float(qs[ix]), float(qs[jx])],
                     "S_pi_2pi3": float(pts[0, 0]), "S_2pi3_pi": float(pts[1, 1]), "S_gamma": float(pts[2, 2]),
                     "S_mean": float(S.mean()),
                     "S_cut_qr_pi": [round(float(x), 5) for x in structure_factor(cn[k], n, length, width,
                                                                                  [math.pi], qs)[0]],
                     "S_cut_qc_pi": [round(float(x), 5) for x in structure_factor(cn[k], n, length, width,
                                                                                  qs, [math.pi])[:, 0]]})
    smp.close()
    return {"points": rows, "q_grid": [float(x) for x in qs], "seconds": dt,
            "spin_updates": sum(I.n_chains for I in lats) * N * (anneal + measure)}
