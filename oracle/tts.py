"""Oracle for the ground-state search and the time-to-solution of Sec. III.C
(test infrastructure only: called by tests/ and the benchmark, never by the
library).

- Per-chain minimum energy: the plain definition over a run's counts trace
  (M, B1, B2) per sweep: E = w . (M, B1, B2) exactly in integers, the lowest
  value and the first sample that reaches it (numpy's argmin returns the first
  index of the minimum), counted in completed sweeps.
- Ground-state energy per spin: the lowest of the four ordered states of the
  phase diagram of Sec. III.A (ferromagnet, Neel, antiparallel dimers, the 1/3
  plateau of UUD rows), each written out from its bond counts on the periodic
  lattice (N spins, 2N J1 bonds, N/2 dimers, L a multiple of 6):
    FM      M = N,    B1 = 2N,     B2 = N/2
    Neel    M = 0,    B1 = -2N,    B2 = N/2   (dimers join same-sublattice sites)
    dimer   M = 0,    B1 = 0,      B2 = -N/2
    1/3     M = N/3,  B1 = -2N/3,  B2 = -N/6
  Pinned in the tests by the exact min-plus row transfer matrix at 6x6 over the
  phase points of Fig. 5 and points of every region of the phase diagram.
- TTS_l of Eq. (14): T log(1 - l/100) / log(1 - p_gnd), with p_gnd the
  fraction of independent runs that reach the ground state and T the mean
  time at which the successful runs first reach it; TTS_100 = T when every
  run succeeds.
"""
from __future__ import annotations

import math

import numpy as np

# (M, B1, B2) per spin of the four candidate ground states
PHASE_COUNTS = {
    "fm": (1.0, 2.0, 0.5),
    "neel": (0.0, -2.0, 0.5),
    "dimer": (0.0, 0.0, -0.5),
    "one_third": (1.0 / 3.0, -2.0 / 3.0, -1.0 / 6.0),
}


def phase_energy(phase, J1, J2, h):
    """E/N of an ordered phase, H = J1 B1 + J2 B2 - h M."""
    M, B1, B2 = PHASE_COUNTS[phase]
    return J1 * B1 + J2 * B2 - h * M


def ground_state(J1, J2, h):
    """(phase, E/N) of the lowest of the four ordered states."""
    best = min(PHASE_COUNTS, key=lambda p: phase_energy(p, J1, J2, h))
    return best, phase_energy(best, J1, J2, h)


def ground_energy_q(L, J1q, J2q, hq, phase):
    """Ground-state energy in 2^-16 units from the quantised couplings and the
    phase's integer bond counts on the periodic L x L lattice (L % 6 == 0)."""
    assert L % 6 == 0
    N = L * L
    M, B1, B2 = (round(x * N) for x in PHASE_COUNTS[phase])
    return J1q * B1 + J2q * B2 - hq * M


def min_energy(trace, w, sweep0=0, every=1):
    """trace: [n_samples, chains, 3] integer counts (M, B1, B2) of one run.
    Returns (emin, first) per chain: the lowest E = w . counts and the number of
    completed sweeps at its first sample, sweep0 + (t + 1) every."""
    t = np.asarray(trace, np.int64)
    E = w[0] * t[..., 0] + w[1] * t[..., 1] + w[2] * t[..., 2]
    emin = E.min(axis=0)
    first = sweep0 + (E.argmin(axis=0) + 1) * every
    return emin, first


def tts(p_gnd, T, level=99.0):
    """Eq. (14).  p_gnd = 0 -> inf; p_gnd = 1 -> T (TTS_100)."""
    if p_gnd <= 0.0:
        return math.inf
    if p_gnd >= 1.0:
        return T
    return T * math.log(1.0 - level / 100.0) / math.log(1.0 - p_gnd)
