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


# ------------------------------------------------------------- general lattices

def lattice_transfer_parts(Lc, J, h_even, h_odd, open_c=False):
    """Row transfer energies of an Lc-column lattice with one coupling per
    filter (App. A Convoluter-Reverse) and a field per column parity (App. A
    Accumulator); columns open (no bond across the edge) or periodic.

    e_row[p][a]     : horizontal bonds and field of a row of parity p in state a
                      (filters 0/1 on even rows, 2/3 on odd rows, by the parity
                      of the left column);
    e_link[p][a, b] : bonds between a row of parity p (state a) and the row
                      below (b): vertical bonds (filters 4/6 below even rows,
                      5/7 below odd rows, by column parity), and the '\\' dimers
                      (2i, 2j)-(2i+1, 2j+1) below even rows (filter 8), the '/'
                      dimers (2i+1, 2j+2)-(2i+2, 2j+1) below odd rows (filter 9)."""
    st = _row_states(Lc).astype(np.float64)
    J = np.asarray(J, np.float64)
    ncol = Lc - 1 if open_c else Lc
    right = np.roll(st, -1, 1)
    e_row, e_link = [], []
    for p in (0, 1):
        jh = np.array([J[2 * p + (c % 2)] for c in range(Lc)])
        e = (st[:, :ncol] * right[:, :ncol]) @ jh[:ncol]
        e = e - h_even * st[:, 0::2].sum(1) - h_odd * st[:, 1::2].sum(1)
        e_row.append(e)
        jv = np.array([J[4 + 2 * (c % 2) + p] for c in range(Lc)])
        link = (st * jv[None, :]) @ st.T
        if p == 0:
            link = link + J[8] * (st[:, 0::2] @ st[:, 1::2].T)
        else:
            nd = Lc // 2 - 1 if open_c else Lc // 2
            link = link + J[9] * (np.roll(st, -2, 1)[:, 0::2][:, :nd] @ st[:, 1::2][:, :nd].T)
        e_link.append(link)
    return st, e_row, e_link


def lattice_tm_averages(Lr, Lc, J, h_even, h_odd, T, open_r=False, open_c=False):
    """Exact <E>/N and <m> of an Lr x Lc Shastry-Sutherland lattice with one
    coupling per filter, a field per column parity and each axis open or
    periodic (row transfer matrix over 2^Lc row states, Lc <= 12).

    Periodic rows: Z = Tr (A0 A1)^(Lr/2) with A_p[a, b] the weight of a row of
    parity p in state a and its bonds to the next row in state b.  Open rows:
    the bonds from the last row to the first are absent, so Z is a product of
    vectors and matrices, and <E>, <m> are sums over row positions of local
    insertions between a forward and a backward vector."""
    st, e_row, e_link = lattice_transfer_parts(Lc, J, h_even, h_odd, open_c)
    Mr = st.sum(1)
    N = Lr * Lc
    E = [e_row[p][:, None] + e_link[p] for p in (0, 1)]
    if not open_r:
        half = 0.5 * float(np.min(E[0].min(axis=0) + E[1].min(axis=1)))
        A = [np.exp(-(E[p] - half) / T) for p in (0, 1)]
        pair = A[0] @ A[1]
        sc = pair.max()
        pair = pair / sc
        dE = ((A[0] * E[0]) @ A[1] + A[0] @ (A[1] * E[1])) / sc
        dM = ((A[0] * Mr[:, None]) @ A[1] + A[0] @ (A[1] * Mr[:, None])) / sc
        nb = Lr // 2
        P = np.eye(pair.shape[0])
        for _ in range(nb - 1):
            P = P @ pair
            P /= P.max()
        Z = np.trace(P @ pair)
        return {"E": float(nb * np.trace(P @ dE) / Z / N), "m": float(nb * np.trace(P @ dM) / Z / N)}
    # open rows: rows 0..Lr-1, links r -> r+1 for r < Lr - 1; the last row (odd) has only its own energy
    e_last = e_row[1]
    shift = [float(E[p].min()) for p in (0, 1)]
    A = [np.exp(-(E[p] - shift[p]) / T) for p in (0, 1)]
    wl = np.exp(-(e_last - e_last.min()) / T)
    fw = [np.ones(st.shape[0])]
    for r in range(Lr - 1):
        v = fw[-1] @ A[r % 2]
        fw.append(v / v.max())
    bw = [None] * Lr
    bw[Lr - 1] = wl
    for r in range(Lr - 2, -1, -1):
        v = A[r % 2] @ bw[r + 1]
        bw[r] = v / v.max()
    Etot, Mtot = 0.0, 0.0
    for r in range(Lr - 1):
        p = r % 2
        z = fw[r] @ A[p] @ bw[r + 1]
        Etot += fw[r] @ (A[p] * E[p]) @ bw[r + 1] / z
        Mtot += fw[r] @ (A[p] * Mr[:, None]) @ bw[r + 1] / z
    z = fw[Lr - 1] @ wl
    Etot += fw[Lr - 1] @ (wl * e_last) / z
    Mtot += fw[Lr - 1] @ (wl * Mr) / z
    return {"E": float(Etot / N), "m": float(Mtot / N)}
