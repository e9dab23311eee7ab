"""Exact averages of the Shastry-Sutherland Ising law on small periodic
lattices (test infrastructure only: called by tests/, by the script that
writes stored reference values, never by the library).

The law is exp(-H / T) with H = J1 sum_sq s s + J2 sum_dimer s s - h sum s
(Sec. I Eq. (1), field read as favouring up spins), on the L x L lattice of
Fig. 1a with the '\\' dimer on the plaquette with top-left site (2i, 2j) and
the '/' dimer on the plaquette with top-left site (2i+1, 2j+1).  Every bond
joins two sites of one row or of two consecutive rows, so a row transfer
matrix gives <E>/N and <m> exactly for L up to about 12 (2^L row states).
Pinned in the tests by brute-force enumeration of all 4x4 states and by the
closed-form ground-state energies of the Neel and 1/3 phases.
"""
from __future__ import annotations

import numpy as np


def _row_states(L):
    idx = np.arange(1 << L, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(L)[None, :]) & 1
    return (2 * bits - 1).astype(np.int64)


def transfer_parts(L, J1, J2, h):
    """Row transfer energies.  Every bond joins two sites of one row or of two
    consecutive rows, so the periodic lattice is a ring of rows.

    e_row[a]      : horizontal J1 bonds and field of a row in state a;
    e_even[a, b]  : bonds between an even row 2i (state a) and row 2i+1 (b):
                    vertical J1 and the '\\' dimers (2i, 2j)-(2i+1, 2j+1);
    e_odd[a, b]   : bonds between an odd row 2i+1 (a) and row 2i+2 (b):
                    vertical J1 and the '/' dimers (2i+1, 2j+2)-(2i+2, 2j+1)."""
    st = _row_states(L)
    e_row = J1 * (st * np.roll(st, -1, 1)).sum(1) - h * st.sum(1)
    vert = st @ st.T
    e_even = J1 * vert + J2 * (st[:, 0::2] @ st[:, 1::2].T)
    e_odd = J1 * vert + J2 * (np.roll(st, -2, 1)[:, 0::2] @ st[:, 1::2].T)
    return st, e_row.astype(np.float64), e_even.astype(np.float64), e_odd.astype(np.float64)


def tm_averages(L, J1, J2, h, T):
    """Exact <E>/N and <m> of the periodic L x L lattice (row transfer matrix;
    L <= 12).  Z = Tr (Te To)^(L/2); <E> and <m> are ratios of traces in which
    any common scale of the matrices cancels, so the Boltzmann factors are
    taken relative to the cheapest two-row path and the matrix power is
    renormalised at every step (no underflow at low T)."""
    st, e_row, e_even, e_odd = transfer_parts(L, J1, J2, h)
    Ee = e_row[:, None] + e_even          # row 2i's own energy + link to row 2i+1
    Eo = e_row[:, None] + e_odd
    half = 0.5 * float(np.min(Ee.min(axis=0) + Eo.min(axis=1)))  # half the cheapest path a -> b -> c
    Te = np.exp(-(Ee - half) / T)
    To = np.exp(-(Eo - half) / T)
    Mr = st.sum(1).astype(np.float64)
    pair = Te @ To
    sc = pair.max()
    pair = pair / sc
    dE = ((Te * Ee) @ To + Te @ (To * Eo)) / sc
    dM = ((Te * Mr[:, None]) @ To + Te @ (To * Mr[:, None])) / sc
    nb = L // 2
    P = np.eye(pair.shape[0])
    for _ in range(nb - 1):
        P = P @ pair
        P /= P.max()
    Z = np.trace(P @ pair)
    N = L * L
    return {"E": float(nb * np.trace(P @ dE) / Z / N), "m": float(nb * np.trace(P @ dM) / Z / N)}


def tm_ground_energy(L, J1, J2, h):
    """Exact ground-state energy per spin by a min-plus row transfer (L <= 8)."""
    st, e_row, e_even, e_odd = transfer_parts(L, J1, J2, h)
    Ee = e_row[:, None] + e_even
    Eo = e_row[:, None] + e_odd
    pair = _minplus(Ee, Eo)
    D = pair
    for _ in range(L // 2 - 1):
        D = _minplus(D, pair)
    return float(np.min(np.diag(D)) / (L * L))


def _minplus(A, B):
    return (A[:, :, None] + B[None, :, :]).min(axis=1)
