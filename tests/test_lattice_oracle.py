"""Pins of the oracle's general-lattice path (open or periodic axes, one
coupling per filter, a field per column parity: App. A Wrapper Module,
Convoluter-Reverse and Accumulator) against independent statements of the
model: the edge-parity bond rules and enumeration of tests/physics.py, the
row transfer matrix of oracle.exact, and the periodic square-lattice oracle.
"""
import math

import numpy as np
import pytest

import oracle
import physics as P
from oracle import exact as EX

SHAPES = [(4, 4, False, False), (4, 4, True, False), (4, 4, False, True), (4, 4, True, True),
          (6, 8, False, True), (8, 6, True, False), (10, 4, True, True)]


def _lat(Lr, Lc, orr, oc, J, he, ho, T, **kw):
    return oracle.Lattice(Lr, Lc, J, he, ho, open_r=orr, open_c=oc, sched="const", T0=T, **kw)


@pytest.mark.parametrize("Lr,Lc,orr,oc", SHAPES)
def test_bonds_are_the_lattice_edges(Lr, Lc, orr, oc):
    """The cell-window bonds that exist are exactly the square-lattice edges
    and dimers of the lattice, labelled by filter, with those that would
    cross an open edge left out (App. A Wrapper Module, zero padding)."""
    lat = _lat(Lr, Lc, orr, oc, [1.0] * 10, 0, 0, 1)
    got = []
    for k in range(10):
        for i in range(Lr // 2):
            for j in range(Lc // 2):
                b = oracle.lattice_bond(lat, k, i, j)
                if b is not None:
                    got.append((k, b[0], b[1]))
    ref = P.lattice_bonds(Lr, Lc, orr, oc)
    assert sorted(got) == sorted(ref)
    n_per = {k: sum(1 for x in got if x[0] == k) for k in range(10)}
    C = (Lr // 2) * (Lc // 2)
    for k in (0, 2, 4, 6, 8):
        assert n_per[k] == C
    assert n_per[1] == n_per[3] == (Lr // 2) * (Lc // 2 - (1 if oc else 0))
    assert n_per[5] == n_per[7] == (Lr // 2 - (1 if orr else 0)) * (Lc // 2)
    assert n_per[9] == (Lr // 2 - (1 if orr else 0)) * (Lc // 2 - (1 if oc else 0))


@pytest.mark.parametrize("Lr,Lc,orr,oc", SHAPES)
def test_counts_match_independent_geometry(Lr, Lc, orr, oc):
    rng = np.random.default_rng(Lr * 100 + Lc + 7 * orr + 3 * oc)
    lat = _lat(Lr, Lc, orr, oc, [1.0] * 10, 0, 0, 1)
    for _ in range(20):
        s = (2 * rng.integers(0, 2, (Lr, Lc)) - 1).astype(np.int8)
        assert np.array_equal(oracle.lattice_counts(lat, s), P.lattice_counts(s, Lr, Lc, orr, oc))


@pytest.mark.parametrize("orr,oc,seed", [(False, False, 1), (True, False, 2), (False, True, 3), (True, True, 4)])
def test_marginal_is_boltzmann_every_4x4_state(orr, oc, seed):
    """Eq. (4) on a general lattice: summing out the hidden unit of every
    present bond gives exp(-H/T) up to a constant for all 2^16 states, with
    ten different couplings (some negative, one zero) and different even /
    odd column fields.  Slack: the 16.16 rounding of weights and bias."""
    rng = np.random.default_rng(seed)
    J = rng.uniform(-2.0, 2.0, 10)
    J[3] = 0.0
    he, ho, T = 1.3, -0.7, 0.9
    lat = _lat(4, 4, orr, oc, J, he, ho, T)
    st = P.all_states(4)
    Jq = np.array([oracle.quantise(x) for x in J]) / 65536
    heq, hoq = oracle.quantise(he) / 65536, oracle.quantise(ho) / 65536
    E = P.lattice_energy(P.lattice_counts(st, 4, 4, orr, oc), Jq, heq, hoq)
    lm = np.array([oracle.lattice_log_marginal(lat, 1, 0, s) for s in st])
    d = lm + E / T
    nb = len(P.lattice_bonds(4, 4, orr, oc))
    assert d.max() - d.min() < 2 * nb * 2.0 ** -16 + 16 * 2.0 ** -16


def test_periodic_ss_lattice_equals_square_oracle():
    """With both axes periodic, J_k = (J1 x 8, J2 x 2) and one field, the
    general path follows the same conventions as the square-lattice oracle:
    identical trajectories, bit for bit."""
    for L, J2, h, sched, T0, T1 in [(6, 0.5, 0.0, "linear", 3.0, 0.1), (12, 1.0, 3.0, "geometric", 5.0, 0.2),
                                    (36, 1.5, 1.0, "const", 0.7, None)]:
        lat = oracle.Lattice(L, L, oracle.ss_filters(1.0, J2), h, sched=sched, T0=T0, T1=T1, id=11)
        oi = oracle.Instance(L, 1.0, J2, h, sched, T0, T1, id=11)
        for ch in (0, 5):
            s1, t1, _ = oracle.run_chain(oi, 150, 99, ch, 0, 150, trace=True)
            s2, t2, _ = oracle.run_lattice_chain(lat, 150, 99, ch, 0, 150, trace=True)
            assert np.array_equal(s1, s2)
            assert np.array_equal(t1[:, 0], t2[:, 0] + t2[:, 1])
            assert np.array_equal(t1[:, 1], t2[:, 2:10].sum(1)) and np.array_equal(t1[:, 2], t2[:, 10:].sum(1))


@pytest.mark.parametrize("orr,oc,seed,T", [(True, True, 11, 1.1), (False, True, 12, 0.8), (True, False, 13, 1.6)])
def test_gibbs_matches_enumeration_4x4(orr, oc, seed, T):
    """Block Gibbs on general 4x4 lattices samples exp(-H/T): chain averages
    of E/N and m agree with enumeration within 3 standard errors."""
    rng = np.random.default_rng(seed)
    J = rng.uniform(-1.5, 1.5, 10)
    he, ho = rng.uniform(-1.0, 1.0, 2)
    lat = _lat(4, 4, orr, oc, J, he, ho, T, id=5)
    Jq = np.array([oracle.quantise(x) for x in J]) / 65536
    heq, hoq = oracle.quantise(he) / 65536, oracle.quantise(ho) / 65536
    S, burn, n_chains = 1500, 300, 48
    Em, mm = [], []
    for ch in range(n_chains):
        _, tr, _ = oracle.run_lattice_chain(lat, S, 2025, ch, 0, S, trace=True)
        tr = tr[burn:].astype(np.float64)
        Em.append(P.lattice_energy(tr, Jq, heq, hoq).mean() / 16)
        mm.append((tr[:, 0] + tr[:, 1]).mean() / 16)
    ex = P.lattice_exact(4, 4, Jq, heq, hoq, T, orr, oc)
    for vals, ref in ((Em, ex["E"]), (mm, ex["m"])):
        v = np.array(vals)
        se = v.std(ddof=1) / math.sqrt(len(v))
        assert abs(v.mean() - ref) < 3 * se, (v.mean(), ref, se)


def test_gibbs_matches_transfer_matrix_on_a_confined_strip():
    """A laterally confined SS strip (Sec. III.A: open in the lateral
    direction, periodic along the strip) of 8 columns and 12 rows at
    J2/J1 = 1.5, h = 4.5, T = 1: Gibbs averages agree with the row transfer
    matrix within 3 SE."""
    Lr, Lc, T = 12, 8, 1.0
    J = oracle.ss_filters(1.0, 1.5)
    lat = _lat(Lr, Lc, False, True, J, 4.5, 4.5, T, id=6)
    S, burn = 1200, 200
    Em, mm = [], []
    for ch in range(32):
        _, tr, _ = oracle.run_lattice_chain(lat, S, 31, ch, 0, S, trace=True)
        tr = tr[burn:].astype(np.float64)
        Em.append(P.lattice_energy(tr, J, 4.5, 4.5).mean() / (Lr * Lc))
        mm.append((tr[:, 0] + tr[:, 1]).mean() / (Lr * Lc))
    ex = EX.lattice_tm_averages(Lr, Lc, J, 4.5, 4.5, T, open_r=False, open_c=True)
    for vals, ref in ((Em, ex["E"]), (mm, ex["m"])):
        v = np.array(vals)
        se = v.std(ddof=1) / math.sqrt(len(v))
        assert abs(v.mean() - ref) < 3 * se, (v.mean(), ref, se)


@pytest.mark.parametrize("Lr,Lc,orr,oc", [(4, 4, True, True), (4, 4, False, True), (4, 2, True, True),
                                          (4, 4, False, False)])
def test_transfer_matrix_equals_enumeration(Lr, Lc, orr, oc):
    rng = np.random.default_rng(Lr + 10 * Lc + orr + 2 * oc)
    J = rng.uniform(-1.5, 2.0, 10)
    he, ho = rng.uniform(-2.0, 2.0, 2)
    T = 0.7
    a = P.lattice_exact(Lr, Lc, J, he, ho, T, orr, oc)
    b = EX.lattice_tm_averages(Lr, Lc, J, he, ho, T, open_r=orr, open_c=oc)
    assert abs(a["E"] - b["E"]) < 1e-12 and abs(a["m"] - b["m"]) < 1e-12


def test_transfer_matrix_reduces_to_the_square_lattice():
    for L, J2, h, T in [(6, 1.0, 3.0, 0.8), (8, 0.5, 0.0, 1.2)]:
        a = EX.tm_averages(L, 1.0, J2, h, T)
        b = EX.lattice_tm_averages(L, L, oracle.ss_filters(1.0, J2), h, h, T)
        assert abs(a["E"] - b["E"]) < 1e-12 and abs(a["m"] - b["m"]) < 1e-12


@pytest.mark.parametrize("Lr,Lc", [(4, 6), (6, 4), (12, 8)])
def test_displacement_correlation_gives_the_structure_factor(Lr, Lc):
    """Sec. III.B Eq. (13) on any lattice: |sum_r s_r e^{i q.r}|^2 equals the
    sum over displacements d of Cn(d) e^{i q.d} (with Cn(-d) = Cn(d)), for
    arbitrary q; Cn(0) = N."""
    rng = np.random.default_rng(Lr * Lc)
    rr, cc = np.meshgrid(np.arange(Lr), np.arange(Lc), indexing="ij")
    for _ in range(5):
        s = (2 * rng.integers(0, 2, (Lr, Lc)) - 1).astype(np.int8)
        Cn = oracle.lattice_corr(Lr, Lc, s)
        assert Cn[0, Lc - 1] == Lr * Lc
        for q in rng.uniform(-math.pi, math.pi, (6, 2)):
            direct = abs((s * np.exp(1j * (q[0] * rr + q[1] * cc))).sum()) ** 2
            tot = 0.0
            for dr in range(Lr):
                for dc in range(-(Lc - 1), Lc):
                    c = Cn[dr, dc + Lc - 1]
                    if dr == 0 and dc == 0:
                        tot += c
                    elif dr > 0 or dc > 0:
                        tot += 2 * c * math.cos(q[0] * dr + q[1] * dc)
            assert abs(tot - direct) < 1e-8 * max(1.0, direct)


def test_accumulators_and_corr_over_measured_sweeps():
    """The accumulated sums equal a sweep-by-sweep rerun of the same chain."""
    lat = _lat(6, 8, True, False, oracle.ss_filters(1.0, 1.5), 2.0, -1.0, 0.9, id=4)
    S = 60
    corr = np.zeros(6 * 15, np.int64)
    _, _, acc = oracle.run_lattice_chain(lat, S, 3, 2, 0, S, measure_every=3, burn_in=10, corr=corr)
    s = None
    ref = np.zeros(oracle.LATTICE_N_ACC, np.int64)
    cref = np.zeros((6, 15), np.int64)
    rr, cc = np.meshgrid(np.arange(6), np.arange(8), indexing="ij")
    stag = np.where((rr + cc) % 2 == 0, 1, -1)
    for sw in range(S):
        s, _, _ = oracle.run_lattice_chain(lat, S, 3, 2, sw, sw + 1, spins=s)
        if sw >= 10 and (sw - 10) % 3 == 0:
            c = P.lattice_counts(s, 6, 8, True, False)
            M = int(c[0] + c[1])
            ms = int((stag * s).sum())
            ref[0] += 1
            ref[1:13] += c
            ref[13] += M * M
            ref[14] += abs(M)
            ref[15] += ms
            ref[16] += ms * ms
            ref[17] += abs(ms)
            cref += oracle.lattice_corr(6, 8, s)
    assert np.array_equal(acc, ref)
    assert np.array_equal(corr.reshape(6, 15), cref)
