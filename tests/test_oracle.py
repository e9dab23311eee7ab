"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints, exhaustive enumeration, an independent transfer matrix, closed
forms, or invariants.  A plausible mistake in the oracle (a wrong bond, sign,
weight formula, field sign, threshold rounding, counter map) fails one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import physics as P
from oracle import exact as EX

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


# ------------------------------------------------------------- geometry

def _bonds(L):
    out = []
    for i in range(L // 2):
        for j in range(L // 2):
            for k in range(10):
                a, b, t = oracle.bond_sites(L, k, i, j)
                out.append((a, b, t))
    return out


@pytest.mark.parametrize("L", [4, 6, 18])
def test_bond_table_is_the_ss_lattice(L):
    """The 10 filters cover every square-lattice edge once (J1) and every SS
    dimer once (J2); each site sits on 4 J1 bonds and 1 dimer."""
    bonds = _bonds(L)
    j1 = sorted(tuple(sorted((a, b))) for a, b, t in bonds if t == 1)
    j2 = sorted(tuple(sorted((a, b))) for a, b, t in bonds if t == 2)
    nn = sorted(tuple(sorted(e)) for e in P.nn_bonds(L))
    dm = sorted(tuple(sorted(e)) for e in P.dimer_bonds(L))
    assert j1 == nn
    assert j2 == dm
    deg1 = np.zeros((L, L), int)
    deg2 = np.zeros((L, L), int)
    for a, b, t in bonds:
        d = deg1 if t == 1 else deg2
        d[a] += 1
        d[b] += 1
    assert (deg1 == 4).all() and (deg2 == 1).all()


def test_node_counts_match_paper():
    """Sec. II.C / Sec. III: 324 visible + 810 hidden = 1134 nodes at 18x18;
    App. A: floor((L+1)/s)^2 hidden units per filter, 10 filters, stride 2."""
    g = GOLD["nodes_at_18"]
    L = g["L"]
    n_hidden = len(_bonds(L))
    assert L * L == g["visible"]
    assert n_hidden == g["hidden"]
    assert L * L + n_hidden == g["total"]
    s = GOLD["filters"]["stride"]
    assert n_hidden == GOLD["filters"]["count"] * ((L + 1) // s) ** 2
    # the wrapper output (L+M-1)^2 with M = 3: the filters of cell (0,0) span a
    # 3x3 window (offsets 0..M-1 in both directions)
    offs = [oracle.bond_sites(64, k, 0, 0) for k in range(10)]
    span_r = max(max(a[0], b[0]) for a, b, _ in offs)
    span_c = max(max(a[1], b[1]) for a, b, _ in offs)
    assert span_r + 1 == span_c + 1 == GOLD["wrapper_output"]["M"]


# -------------------------------------------------------------- weights

@pytest.mark.parametrize("J,T", [(1.0, 3.0), (1.0, 0.5), (-0.7, 1.3), (2.5, 0.05), (0.5, 10.0)])
def test_bond_weight_solves_eq_6_8(J, T):
    """Eqs. (5)-(8): for K = -J/T, cosh(2w) = exp(2|K|), sign on the second spin
    = sgn(K); summing the hidden unit out reproduces exp(K s_a s_b) with
    C = exp(-|K|)/2."""
    Jq = oracle.quantise(J)
    wq, sg = oracle.bond_weight(Jq, T)
    K = -(Jq / 65536.0) / T
    w = wq / 65536.0
    assert sg == (1 if K >= 0 else -1)
    if abs(K) < 20:
        # independent route: numpy arccosh of exp(2|K|)
        assert abs(w - 0.5 * np.arccosh(np.exp(2 * abs(K)))) <= 0.6 / 65536
        for sa in (-1, 1):
            for sb in (-1, 1):
                lhs = math.exp(K * sa * sb)
                rhs = 0.5 * math.exp(-abs(K)) * sum(math.exp(w * sa * h + sg * w * sb * h) for h in (-1, 1))
                # the 16.16 rounding of w (at most 2^-17) moves 2cosh(2w) by a relative 2 tanh(2w) 2^-17
                assert abs(lhs / rhs - 1) < 2.0 ** -15
    else:
        assert abs(w - (abs(K) + 0.5 * math.log(2))) < 1e-6


def test_weight_zero_coupling():
    wq, sg = oracle.bond_weight(0, 1.0)
    assert wq == 0 and sg == 1


@pytest.mark.parametrize("L,J2,h,T", [(4, 0.5, 0.0, 3.0), (4, 1.0, 3.0, 1.0), (4, 2.5, -1.5, 0.7), (6, 1.0, 2.0, 0.9)])
def test_crbm_marginal_is_boltzmann(L, J2, h, T):
    """Eq. (4): summing out every hidden unit gives exp(-H/T) up to a constant,
    for every spin state (exhaustive at 4x4, random states at 6x6).  The only
    slack is the 16.16 rounding of the weights and bias."""
    inst = oracle.Instance(L, 1.0, J2, h, "const", T)
    if L == 4:
        states = P.all_states(4)
    else:
        rng = np.random.default_rng(3)
        states = (2 * rng.integers(0, 2, (400, L, L)) - 1).astype(np.int8)
    J1q, J2q, hq = (oracle.quantise(x) for x in (1.0, J2, h))
    Eq = P.energy(states, J1q / 65536, J2q / 65536, hq / 65536)
    lm = np.array([oracle.log_marginal(inst, 1, 0, s) for s in states])
    d = lm + Eq / T
    n_bonds = 10 * (L // 2) ** 2
    # each bond's log 2cosh is off by at most ~2 * 2^-16 * tanh (weight rounding), bias by N * 2^-17
    assert d.max() - d.min() < 2 * n_bonds * 2.0 ** -16 + L * L * 2.0 ** -16


# ------------------------------------------------------------ threshold

def test_threshold_properties():
    """Sigmoid by the closest 32-bit value (App. A sigmoid module):
    t(0) = 2^31, monotone, within 1/2 ulp of 2^32 sigmoid(2y), saturating."""
    assert oracle.threshold(0) == 1 << 31
    ys = np.unique(np.concatenate([np.arange(0, 4000, 7), np.geomspace(1, 3e6, 400).astype(np.int64)]))
    ts = np.array([oracle.threshold(int(y)) for y in ys], dtype=np.float64)
    assert (np.diff(ts) >= 0).all()
    from scipy.special import expit
    ref = expit(2.0 * ys / 65536.0) * 2.0 ** 32
    ok = ts < 2 ** 32 - 1
    assert np.all(np.abs(ts[ok] - ref[ok]) <= 0.5 + 1e-6 * ref[ok] * 2 ** -20)
    assert oracle.threshold(10 ** 9) == 2 ** 32 - 1


def test_schedules():
    S = 2000
    lin = oracle.Instance(6, sched="linear", T0=3.0, T1=0.1)
    geo = oracle.Instance(6, sched="geometric", T0=5.0, T1=0.05)
    assert oracle.schedule_T(lin, S, 0) == 3.0 and abs(oracle.schedule_T(lin, S, S - 1) - 0.1) < 1e-15
    assert abs(oracle.schedule_T(geo, S, S - 1) - 0.05) < 1e-15
    Tl = np.array([oracle.schedule_T(lin, S, s) for s in range(S)])
    Tg = np.array([oracle.schedule_T(geo, S, s) for s in range(S)])
    assert np.allclose(np.diff(Tl), (0.1 - 3.0) / (S - 1))
    assert np.allclose(Tg[1:] / Tg[:-1], (0.05 / 5.0) ** (1 / (S - 1)))
    te = np.linspace(2, 1, 10)
    ex = oracle.Instance(6, sched="explicit", T_explicit=te)
    assert [oracle.schedule_T(ex, 10, s) for s in range(10)] == list(te)


# --------------------------------------------------------------- Philox

def test_philox_output_statistics():
    """Weak sanity pins of the Philox4x32-10 implementation (the strong pin,
    against rocRAND's Philox4x32-10, runs on the GPU): bit balance, byte
    histogram, lag-1 correlation, avalanche on a one-bit counter change."""
    outs = np.array([oracle.philox([c, 7, 3, 11], [0x1234, 0x5678]) for c in range(4000)], dtype=np.uint32)
    bits = ((outs[:, :, None] >> np.arange(32)) & 1).reshape(-1, 32)
    p = bits.mean(0)
    assert np.all(np.abs(p - 0.5) < 5 * math.sqrt(0.25 / bits.shape[0]))
    by = outs.view(np.uint8).ravel()
    hist = np.bincount(by, minlength=256)
    e = by.size / 256
    chi2 = ((hist - e) ** 2 / e).sum()
    assert chi2 < 255 + 6 * math.sqrt(2 * 255)
    u = outs.ravel().astype(np.float64) / 2 ** 32
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 5 / math.sqrt(u.size)
    flips = []
    for c in range(200):
        a = oracle.philox([c, 1, 2, 3], [9, 9])
        b = oracle.philox([c ^ 1 << (c % 32), 1, 2, 3], [9, 9])
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b)))
    assert abs(np.mean(flips) - 64) < 3


def test_uniforms_distinct_units_distinct_draws():
    """The counter map gives every unit of a sweep its own draw: at 6x6 and
    36x36 (two column words) the 32-bit uniforms of all hidden and visible
    units of one sweep are pairwise distinct (collisions would be a
    2^-32-rare accident) and uniform."""
    for L in (6, 36):
        C = L // 2
        uh = [oracle.uniform_hidden(99, 5, 3, 17, L, k, i, j) for k in range(10) for i in range(C) for j in range(C)]
        uv = [oracle.uniform_visible(99, 5, 3, 17, L, r, c) for r in range(L) for c in range(L)]
        assert len(set(uh)) == len(uh)
        assert len(set(uv)) == len(uv)
        u = np.array(uh + uv, np.float64) / 2 ** 32
        assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)


# ----------------------------------------------------- counts and S(q)

def test_counts_match_independent_geometry():
    rng = np.random.default_rng(0)
    for L in (4, 6, 12, 36):
        s = (2 * rng.integers(0, 2, (L, L)) - 1).astype(np.int8)
        M, B1, B2 = P.bond_counts(s)
        assert oracle.counts(L, s) == (int(M), int(B1), int(B2))


def test_structure_factor_of_perfect_states():
    """Sec. III.B: the Neel state peaks at (pi,pi); the 1/3 plateau (UUD rows,
    Sec. III.A) peaks at (2pi/3, pi)."""
    L = 6
    r, c = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    neel = np.where((r + c) % 2 == 0, 1, -1).astype(np.int8)
    S = P.structure_factor(oracle.corr(L, neel), 1, L)
    a, b = np.unravel_index(np.argmax(S), S.shape)
    assert (a, b) == (L // 2, L // 2) and abs(S[a, b] - 1.0) < 1e-12
    # a plateau ground state from the annealed oracle
    inst = oracle.Instance(6, 1.0, 1.0, 3.0, "geometric", 3.0, 0.05, id=2)
    s, _, _ = oracle.run_chain(inst, 2000, 11, 0, 0, 2000)
    assert s.sum() == 12  # m = 1/3
    S = P.structure_factor(oracle.corr(L, s), 1, L)
    S[0, 0] = 0.0
    peak = np.argwhere(S > S.max() - 1e-9)
    q = {(round(2 * math.pi * a / L, 9), round(2 * math.pi * b / L, 9)) for a, b in peak}
    tgt = GOLD["structure_factor_peaks"]["one_third"]
    want = {(round(tgt[0], 9), round(tgt[1], 9)), (round(tgt[1], 9), round(tgt[0], 9)),
            (round(2 * math.pi - tgt[0], 9), round(tgt[1], 9)), (round(tgt[1], 9), round(2 * math.pi - tgt[0], 9))}
    assert q & want


# --------------------------------------------------------- dynamics pins

def _uud(L, transpose=False, shift=0):
    """The 1/3-plateau UUD pattern: ferromagnetic rows (all up) every third row,
    between them two antiferromagnetic rows (Sec. III.A)."""
    s = np.zeros((L, L), np.int8)
    for r in range(L):
        k = (r + shift) % 3
        s[r] = 1 if k == 0 else (2 * ((np.arange(L) + k) % 2) - 1)
    return s.T.copy() if transpose else s


@pytest.mark.parametrize("L", [6, 12, 18])
def test_order_parameter_closed_forms(L):
    """Plateau structure factor |S(q*)|^2 at q* = (pi, 2pi/3) and (2pi/3, pi):
    the ferromagnet and the Neel state have none; each UUD state puts N^2/3 on
    its own orientation's wave vector (S(q*)/N = N/3, Sec. III.B), for every
    translation, and the transpose swaps the two components."""
    N = L * L
    assert oracle.order(L, np.ones((L, L), np.int8)) == (0, 0, 0)
    neel = (2 * ((np.arange(L)[:, None] + np.arange(L)[None, :]) % 2) - 1).astype(np.int8)
    assert oracle.order(L, neel) == (0, 0, 0)
    for shift in range(3):
        s = _uud(L, shift=shift)  # period 3 along rows, antiferromagnetic along columns
        assert oracle.order(L, s) == (N * N // 3, 0, N * N // 3)
        assert oracle.order(L, s.T.copy()) == (N * N // 3, N * N // 3, 0)


@pytest.mark.parametrize("seed", [1, 2])
def test_order_parameter_matches_fft(seed):
    """On random states the two components equal |DFT|^2 of the spins at the
    two wave vectors (numpy FFT on 6x6 and 12x12, where 2pi/3 is a lattice
    momentum)."""
    rng = np.random.default_rng(seed)
    for L in (6, 12):
        s = (2 * rng.integers(0, 2, (L, L)) - 1).astype(np.int8)
        F = np.fft.fft2(s.astype(np.float64))
        a = abs(F[L // 2, (2 * L // 3) % L]) ** 2  # q = (pi, -2pi/3): same modulus as (pi, 2pi/3)
        b = abs(F[(2 * L // 3) % L, L // 2]) ** 2
        m, oa, ob = oracle.order(L, s)
        assert oa == round(a) and ob == round(b) and m == max(oa, ob)


def test_trajectory_is_resumable_and_deterministic():
    inst = oracle.Instance(6, 1.0, 0.5, 0.0, "linear", 3.0, 0.1, id=4)
    s1, t1, _ = oracle.run_chain(inst, 400, 123, 2, 0, 400, trace=True)
    a, ta, _ = oracle.run_chain(inst, 400, 123, 2, 0, 150, trace=True)
    b, tb, _ = oracle.run_chain(inst, 400, 123, 2, 150, 400, spins=a, trace=True)
    assert (s1 == b).all()
    assert (t1 == np.concatenate([ta, tb])).all()
    _, t2, _ = oracle.run_chain(inst, 400, 124, 2, 0, 400, trace=True)
    assert not (t1 == t2).all()  # another seed gives another trajectory


def test_infinite_temperature_is_fair_coin():
    """At T -> infinity every weight and bias is 0 and every unit is a fair coin."""
    inst = oracle.Instance(6, 1.0, 0.5, 0.3, "const", 1e12, id=0)
    ms = []
    for ch in range(40):
        _, tr, _ = oracle.run_chain(inst, 1, 5, ch, 0, 50, trace=True)
        ms.append(tr[:, 0])
    m = np.concatenate(ms).astype(np.float64)
    assert abs(m.mean()) < 5 * math.sqrt(36 / m.size)
    assert abs(m.var() - 36) < 5 * 36 * math.sqrt(2 / m.size)


@pytest.mark.parametrize("J2,h,T", [(0.5, 0.0, 3.0), (1.0, 3.0, 1.0), (2.5, 0.0, 1.5), (1.0, 2.0, 0.8)])
def test_gibbs_matches_exact_4x4(J2, h, T):
    """Block Gibbs (Eqs. (11)-(12)) samples exp(-H/T): chain averages of E/N and
    m at 4x4 agree with exhaustive enumeration within 3 standard errors."""
    L, n_chains, S, burn = 4, 48, 1500, 300
    inst = oracle.Instance(L, 1.0, J2, h, "const", T, id=7)
    E_means, m_means = [], []
    J1q, J2q, hq = (oracle.quantise(x) for x in (1.0, J2, h))
    for ch in range(n_chains):
        _, tr, _ = oracle.run_chain(inst, S, 2024, ch, 0, S, trace=True)
        tr = tr[burn:].astype(np.float64)
        E = (J1q * tr[:, 1] + J2q * tr[:, 2] - hq * tr[:, 0]) / 65536 / 16
        E_means.append(E.mean())
        m_means.append(tr[:, 0].mean() / 16)
    ex = P.exact_averages(4, J1q / 65536, J2q / 65536, hq / 65536, T)
    for vals, ref in ((E_means, ex["E"]), (m_means, ex["m"])):
        v = np.array(vals)
        se = v.std(ddof=1) / math.sqrt(len(v))
        assert abs(v.mean() - ref) < 3 * se + 1e-12, (v.mean(), ref, se)


@pytest.mark.parametrize("J2,h,T", [(1.0, 3.0, 1.0), (0.5, 0.0, 0.7), (2.5, 1.0, 2.0), (1.5, -2.0, 0.4)])
def test_transfer_matrix_equals_enumeration_4x4(J2, h, T):
    """The row transfer matrix of oracle.exact reproduces brute-force
    enumeration of all 2^16 states of the 4x4 lattice."""
    tm = EX.tm_averages(4, 1.0, J2, h, T)
    en = P.exact_averages(4, 1.0, J2, h, T)
    assert abs(tm["E"] - en["E"]) < 1e-12 and abs(tm["m"] - en["m"]) < 1e-12


def test_transfer_matrix_low_temperature_plateau():
    """6x6 at (J2, h) = (1, 3): as T -> 0 the transfer matrix reaches the 1/3
    plateau's closed form E/N = -2 J1/3 - J2/6 - h/3 = -11/6, m = 1/3."""
    tm = EX.tm_averages(6, 1.0, 1.0, 3.0, 0.15)
    assert abs(tm["E"] + 11.0 / 6.0) < 1e-9 and abs(tm["m"] - 1.0 / 3.0) < 1e-9


def test_gibbs_matches_transfer_matrix_6x6():
    """The 1/3 plateau at J2 = 1, h = 3 (Sec. III.A) in equilibrium at 6x6:
    Gibbs averages agree with the exact transfer-matrix values."""
    L, T = 6, 0.8
    inst = oracle.Instance(L, 1.0, 1.0, 3.0, "const", T, id=8)
    S, burn = 1200, 300
    E_means, m_means = [], []
    for ch in range(32):
        _, tr, _ = oracle.run_chain(inst, S, 77, ch, 0, S, trace=True)
        tr = tr[burn:].astype(np.float64)
        E_means.append(((tr[:, 1] + tr[:, 2] - 3 * tr[:, 0]) / 36).mean())
        m_means.append(tr[:, 0].mean() / 36)
    ex = EX.tm_averages(6, 1.0, 1.0, 3.0, T)
    for vals, ref in ((E_means, ex["E"]), (m_means, ex["m"])):
        v = np.array(vals)
        se = v.std(ddof=1) / math.sqrt(len(v))
        assert abs(v.mean() - ref) < 3 * se, (v.mean(), ref, se)


def test_annealing_reaches_paper_phases():
    """Sec. III.A / III.C phase points: annealed chains at 6x6 reach the exact
    ground-state energy (transfer matrix), with the paper's magnetisation for
    the 1/3 plateaus and the FM state, m = 0 in the Neel and dimer phases and
    the dimers antiparallel (B2 = -N/2) in the dimer phase."""
    L = 6
    for pt in GOLD["phase_points"]:
        J2, h = pt["J2"], pt["h"]
        inst = oracle.Instance(L, 1.0, J2, h, "geometric", 3.0, 0.05, id=9)
        best = None
        for ch in range(8):
            s, _, _ = oracle.run_chain(inst, 2000, 31, ch, 0, 2000)
            E = P.energy(s, 1.0, J2, h) / (L * L)
            if best is None or E < best[0]:
                best = (E, s)
        E, s = best
        assert abs(E - EX.tm_ground_energy(L, 1.0, J2, h)) < 1e-12, pt
        if "m" in pt:
            assert abs(s.mean() - pt["m"]) < 1e-12, pt
        if pt["phase"] in ("neel", "dimer"):
            assert s.sum() == 0
        if pt["phase"] == "neel":
            S = P.structure_factor(oracle.corr(L, s), 1, L)
            assert np.argmax(S) == np.ravel_multi_index((L // 2, L // 2), S.shape)
        if pt["phase"] == "dimer":
            assert P.bond_counts(s)[2] == -L * L // 2


def test_critical_point_closed_forms():
    """At the paper's critical point (J2 = 1, h = 2, Sec. III.A) the Neel and
    1/3-plateau energies are degenerate: E/N = -2 J1 + J2/2 = -2 J1/3 - J2/6 - h/3.
    The transfer matrix at 6x6 confirms both closed forms on either side."""
    neel = lambda J2, h: -2 + J2 / 2
    third = lambda J2, h: -2 / 3 - J2 / 6 - h / 3
    assert abs(neel(1.0, 2.0) - third(1.0, 2.0)) < 1e-15
    assert abs(EX.tm_ground_energy(6, 1.0, 1.0, 1.5) - neel(1.0, 1.5)) < 1e-12
    assert abs(EX.tm_ground_energy(6, 1.0, 1.0, 2.5) - third(1.0, 2.5)) < 1e-12


def test_philox_matches_rocrand_engine():
    """Strong pin of the oracle's Philox4x32-10: equal to rocRAND's engine
    (called as a library on the host) on random counters and keys."""
    import ctypes as ct
    path = os.path.join(os.path.dirname(__file__), "librocrand_probe.so")
    if not os.path.exists(path):
        from tests import helpers_build
        helpers_build.build()
    lib = ct.CDLL(path)
    rng = np.random.default_rng(12345)
    for _ in range(2000):
        c = rng.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        c[1] &= (1 << 30) - 1  # the probe reaches word 1 through a 64-bit offset
        k = rng.integers(0, 2 ** 32, 2, dtype=np.uint64).astype(np.uint32)
        o = np.zeros(4, np.uint32)
        lib.rocrand_philox_block(c.ctypes.data_as(ct.c_void_p), k.ctypes.data_as(ct.c_void_p),
                                 o.ctypes.data_as(ct.c_void_p))
        assert np.array_equal(o, oracle.philox(c, k)), (c, k)


# ------------------------------------------------------------ staggered magnetisation and accumulated C

def test_staggered_magnetisation_of_perfect_states():
    """Ms = sum (-1)^(r+c) s: +-N for the two Neel states (the AFM phase of
    Sec. III.A), 0 for the ferromagnet, for row stripes and for the UUD
    plateau state."""
    L = 6
    r, c = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    neel = np.where((r + c) % 2 == 0, 1, -1).astype(np.int8)
    assert oracle.staggered(L, neel) == L * L and oracle.staggered(L, -neel) == -L * L
    assert oracle.staggered(L, np.ones((L, L), np.int8)) == 0
    assert oracle.staggered(L, np.where(r % 2 == 0, 1, -1).astype(np.int8)) == 0
    uud = np.where((c % 3 == 2) & (r % 2 == 0), -1, np.where((c % 3 == 0) & (r % 2 == 1), -1, 1)).astype(np.int8)
    assert oracle.staggered(L, uud) == 0


def test_accumulated_correlation_invariants():
    """C(dr, dc) summed over measured sweeps: C(0, 0) = N per sample,
    sum over all offsets = sum of M^2 over the samples (the accumulator's
    second moment), C(-d) = C(d), |C(d)| <= C(0); and the staggered sums equal
    those of the states at the measured sweeps (the chain rerun sweep by
    sweep); the annealed 6x6 workload ends in Neel states, |Ms| = N."""
    L, S, me, burn = 6, 120, 3, 30
    inst = oracle.Instance(L, 1.0, 0.5, 0.0, "linear", 3.0, 0.1, id=5)
    acc = np.zeros(oracle.N_ACC, np.int64)
    corr = np.zeros(L * L, np.int64)
    s_end, _, _ = oracle.run_chain(inst, S, 17, 2, 0, S, measure_every=me, burn_in=burn, acc=acc, corr=corr)
    C = corr.reshape(L, L)
    n = acc[0]
    assert n == len(range(burn, S, me))
    assert C[0, 0] == L * L * n
    assert C.sum() == acc[4]
    assert np.array_equal(C, np.roll(np.roll(C[::-1, ::-1], 1, axis=0), 1, axis=1))
    assert np.abs(C).max() == C[0, 0]
    ms = []
    s = None
    for sw in range(S):
        s, _, _ = oracle.run_chain(inst, S, 17, 2, sw, sw + 1, spins=s)
        if sw >= burn and (sw - burn) % me == 0:
            ms.append(oracle.staggered(L, s))
    ms = np.array(ms, np.int64)
    assert acc[11] == ms.sum() and acc[12] == (ms * ms).sum() and acc[13] == np.abs(ms).sum()
    assert np.array_equal(s, s_end)
    assert abs(oracle.staggered(L, s_end)) == L * L
