"""Independent numpy statement of the Shastry-Sutherland Ising model, used to pin
the oracle.  Nothing here is imported by the oracle or by the HIP library.

Geometry (Sec. I Eq. (1), lattice of Fig. 1a): L x L square lattice, periodic.
  J1 bonds: every nearest-neighbour edge of the square lattice (2N of them).
  J2 bonds: one diagonal on every other plaquette in a checkerboard pattern,
            orthogonal on neighbouring dimer plaquettes: the plaquette with
            top-left site (2i, 2j) carries the '\\' diagonal, the plaquette
            with top-left site (2i+1, 2j+1) carries the '/' diagonal (N/2 dimers,
            every site on exactly one).
Energy with the field favouring up spins: H = J1 sum s s + J2 sum s s - h sum s.
"""
from __future__ import annotations

import numpy as np


def nn_bonds(L):
    out = []
    for r in range(L):
        for c in range(L):
            out.append(((r, c), (r, (c + 1) % L)))
            out.append(((r, c), ((r + 1) % L, c)))
    return out


def dimer_bonds(L):
    out = []
    for i in range(L // 2):
        for j in range(L // 2):
            out.append(((2 * i, 2 * j), (2 * i + 1, 2 * j + 1)))
            out.append(((2 * i + 1, (2 * j + 2) % L), ((2 * i + 2) % L, 2 * j + 1)))
    return out


def bond_counts(spins):
    """spins: [..., L, L] of +-1.  Returns (M, B1, B2) as int64 arrays."""
    s = np.asarray(spins, np.int64)
    M = s.sum(axis=(-1, -2))
    B1 = (s * np.roll(s, -1, axis=-1)).sum(axis=(-1, -2)) + (s * np.roll(s, -1, axis=-2)).sum(axis=(-1, -2))
    L = s.shape[-1]
    B2 = np.zeros(s.shape[:-2], np.int64)
    for (a, b) in dimer_bonds(L):
        B2 = B2 + s[..., a[0], a[1]] * s[..., b[0], b[1]]
    return M, B1, B2


def energy(spins, J1, J2, h):
    M, B1, B2 = bond_counts(spins)
    return J1 * B1 + J2 * B2 - h * M


def all_states(L):
    """All 2^(L*L) configurations (only sensible for L = 4)."""
    n = L * L
    idx = np.arange(1 << n, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(n)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8).reshape(-1, L, L)


def exact_averages(L, J1, J2, h, T, states=None):
    """Exact <E>/N, <m>, <|m|> by enumeration."""
    st = all_states(L) if states is None else states
    M, B1, B2 = bond_counts(st)
    E = J1 * B1 + J2 * B2 - h * M
    N = L * L
    lw = -(E - E.min()) / T
    w = np.exp(lw)
    Z = w.sum()
    return {
        "E": float((w * E).sum() / Z / N),
        "m": float((w * M).sum() / Z / N),
        "abs_m": float((w * np.abs(M)).sum() / Z / N),
        "E_min": float(E.min() / N),
    }


# ------------------------------------------------------- structure factor

def structure_factor(corr_sum, n_samples, L):
    """S(q)/N from summed C(dr, dc) = sum_i s_i s_{i+d}: S(q) = sum_d C(d) e^{i q d} / N,
    returned as S(q)/N on the L x L grid q = 2 pi (a, b)/L."""
    C = np.asarray(corr_sum, np.float64) / n_samples
    F = np.fft.fft2(C).real  # sum_d C(d) e^{-i q d}; C is inversion symmetric
    N = L * L
    return F / N / N


# ------------------------------------------------------- general lattices

def lattice_bonds(Lr, Lc, open_r=False, open_c=False):
    """Bonds of an Lr x Lc Shastry-Sutherland lattice as (filter, site a, site b),
    written from the square-lattice edges and the dimer plaquettes of Fig. 1a,
    labelled by the parity of their first site: horizontal edge (r,c)-(r,c+1) is
    filter 0/1 on even rows (even/odd c) and 2/3 on odd rows; vertical edge
    (r,c)-(r+1,c) is 4/5 in even columns (even/odd r) and 6/7 in odd columns;
    the '\\' dimer (2i,2j)-(2i+1,2j+1) is 8 and the '/' dimer
    (2i+1,2j+2)-(2i+2,2j+1) is 9.  On an open axis the edges and dimers that
    would wrap around are left out."""
    out = []
    for r in range(Lr):
        for c in range(Lc):
            if c + 1 < Lc or not open_c:
                out.append((2 * (r % 2) + (c % 2), (r, c), (r, (c + 1) % Lc)))
            if r + 1 < Lr or not open_r:
                out.append((4 + 2 * (c % 2) + (r % 2), (r, c), ((r + 1) % Lr, c)))
    for i in range(Lr // 2):
        for j in range(Lc // 2):
            out.append((8, (2 * i, 2 * j), (2 * i + 1, 2 * j + 1)))
            if (2 * j + 2 < Lc or not open_c) and (2 * i + 2 < Lr or not open_r):
                out.append((9, (2 * i + 1, (2 * j + 2) % Lc), ((2 * i + 2) % Lr, 2 * j + 1)))
    return out


def lattice_counts(spins, Lr, Lc, open_r=False, open_c=False):
    """spins [..., Lr, Lc] -> int64 [..., 12] = (M_even, M_odd, B_0..B_9)."""
    s = np.asarray(spins, np.int64)
    out = np.zeros(s.shape[:-2] + (12,), np.int64)
    out[..., 0] = s[..., :, 0::2].sum(axis=(-1, -2))
    out[..., 1] = s[..., :, 1::2].sum(axis=(-1, -2))
    for k, a, b in lattice_bonds(Lr, Lc, open_r, open_c):
        out[..., 2 + k] += s[..., a[0], a[1]] * s[..., b[0], b[1]]
    return out


def lattice_energy(counts, J, h_even, h_odd):
    """H = sum_k J_k B_k - h_even M_even - h_odd M_odd from lattice_counts."""
    c = np.asarray(counts, np.float64)
    return c[..., 2:] @ np.asarray(J, np.float64) - h_even * c[..., 0] - h_odd * c[..., 1]


def lattice_exact(Lr, Lc, J, h_even, h_odd, T, open_r=False, open_c=False):
    """Exact <E>/N and <m> by enumeration of all 2^(Lr Lc) states (Lr Lc <= 16)."""
    n = Lr * Lc
    idx = np.arange(1 << n, dtype=np.int64)
    st = (2 * ((idx[:, None] >> np.arange(n)[None, :]) & 1) - 1).reshape(-1, Lr, Lc)
    cnt = lattice_counts(st, Lr, Lc, open_r, open_c)
    E = lattice_energy(cnt, J, h_even, h_odd)
    M = cnt[:, 0] + cnt[:, 1]
    w = np.exp(-(E - E.min()) / T)
    Z = w.sum()
    return {"E": float((w * E).sum() / Z / n), "m": float((w * M).sum() / Z / n), "E_min": float(E.min() / n)}
