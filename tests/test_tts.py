"""Ground-state search and time-to-solution (Sec. III.C Eq. (14)) without a GPU:
the oracle's ordered-phase ground states against the exact min-plus transfer
matrix and the paper's Fig. 5 phase labels, its minimum-energy definition
against brute force, Eq. (14)'s fixed points, the package's host statistics
against the oracle, and the argument checks of crbm_min_energy."""
import ctypes as ct
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import exact as EX
from oracle import tts as OT
import paper_2511_20911_amd as crbm
from paper_2511_20911_amd import tts as PT

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))

# points in every region of the phase diagram (Neel, dimer, 1/3, FM) and near
# the boundaries between them
POINTS = [(1.0, 0.0), (1.0, 3.0), (1.0, 7.0), (2.5, 0.0), (0.5, 4.0), (1.0, 1.5), (1.0, 2.5), (2.5, 1.0),
          (0.3, 2.0), (3.0, 2.0), (1.5, 4.5), (2.0, 1.0), (2.2, 0.5), (0.5, 1.0), (1.8, 4.0), (2.8, 0.2),
          (0.2, 6.5), (1.2, 5.5), (3.0, 7.5), (0.8, 0.3)]


@pytest.mark.parametrize("J2,h", POINTS)
def test_ordered_ground_state_is_exact_at_6x6(J2, h):
    """The lowest of the four ordered states equals the exact ground-state
    energy of the periodic 6x6 lattice (min-plus row transfer matrix)."""
    _, e = OT.ground_state(1.0, J2, h)
    assert abs(e - EX.tm_ground_energy(6, 1.0, J2, h)) < 1e-12


def test_fig5_phase_points_have_the_papers_phases():
    """The four phase points of Sec. III.C (Fig. 5: FM, dimer, Neel, 1/3) are the
    ground states the oracle names there."""
    seen = set()
    for pt in GOLD["phase_points"]:
        if "III.C" not in pt["cite"]:
            continue
        ph, _ = OT.ground_state(1.0, pt["J2"], pt["h"])
        assert ph == pt["phase"], pt
        seen.add(ph)
    assert seen == {"fm", "dimer", "neel", "one_third"}


def test_ordered_state_bond_counts_are_realised():
    """Each ordered state's (M, B1, B2) is realised by an explicit 6x6 spin
    pattern, counted by the oracle's own bond enumeration."""
    L = 6
    r, c = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    pats = {
        "fm": np.ones((L, L), np.int8),
        "neel": np.where((r + c) % 2 == 0, 1, -1).astype(np.int8),
        # UUD: a ferromagnetic row every third row, two antiferromagnetic rows
        # between them (Sec. III.A)
        "one_third": np.where(r % 3 == 0, 1, 2 * ((c + r % 3) % 2) - 1).astype(np.int8),
    }
    for ph, s in pats.items():
        M, B1, B2 = oracle.counts(L, s)
        N = L * L
        assert (M, B1, B2) == tuple(round(x * N) for x in OT.PHASE_COUNTS[ph]), ph
    # dimer: some state with every dimer antiparallel and B1 = 0 exists at the
    # dimer point (found by the exact ground-state energy: E/N = -J2/2)
    assert abs(EX.tm_ground_energy(L, 1.0, 2.5, 0.0) - OT.phase_energy("dimer", 1.0, 2.5, 0.0)) < 1e-12


def test_oracle_min_energy_equals_brute_force():
    rng = np.random.default_rng(4)
    tr = rng.integers(-40, 40, size=(57, 9, 3)).astype(np.int32)
    tr[10:13, 3] = tr[20, 3]  # repeated minimum: the first sample counts
    w = (-3, 5, 2)
    for sweep0, every in ((0, 1), (100, 3)):
        emin, first = OT.min_energy(tr, w, sweep0, every)
        for c in range(tr.shape[1]):
            best, at = None, None
            for t in range(tr.shape[0]):
                E = w[0] * int(tr[t, c, 0]) + w[1] * int(tr[t, c, 1]) + w[2] * int(tr[t, c, 2])
                if best is None or E < best:
                    best, at = E, sweep0 + (t + 1) * every
            assert emin[c] == best and first[c] == at


def test_eq14_fixed_points():
    """TTS_l = T when p_gnd = l/100 (one run then already reaches the
    confidence level); TTS_100 = T; no success -> inf; more success -> less
    time."""
    for l in (50.0, 90.0, 99.0):
        assert abs(OT.tts(l / 100.0, 7.0, l) - 7.0) < 1e-12
    assert OT.tts(1.0, 3.0) == 3.0 and OT.tts(0.0, 3.0) == math.inf
    ps = [0.01, 0.1, 0.5, 0.9, 0.999]
    vals = [OT.tts(p, 10.0) for p in ps]
    assert all(a > b for a, b in zip(vals, vals[1:]))


@pytest.mark.parametrize("L", [6, 12, 18, 24, 48])
def test_package_ground_state_equals_oracle(L):
    for J2, h in POINTS:
        ph, eq = PT.ordered_ground_state(L, 1.0, J2, h)
        oph, _ = OT.ground_state(1.0, J2, h)
        q = PT.quantise
        assert eq == OT.ground_energy_q(L, q(1.0), q(J2), q(h), oph), (L, J2, h)
    with pytest.raises(ValueError):
        PT.ordered_ground_state(8, 1.0, 1.0, 0.0)


def test_package_tts_statistics_equal_oracle():
    rng = np.random.default_rng(9)
    egs = -1000
    for p_true in (0.0, 0.03, 0.4, 1.0):
        n = 500
        hit = rng.random(n) < p_true
        emin = np.where(hit, egs, egs + rng.integers(1, 50, n))
        first = rng.integers(1, 5000, n)
        r = PT.tts_from_runs(emin, first, egs)
        p = hit.mean()
        assert r["p_gnd"] == p
        if p == 0:
            assert r["tts_sweeps"] == math.inf
        else:
            T = first[hit].mean()
            assert abs(r["T_sweeps"] - T) < 1e-9
            assert abs(r["tts_sweeps"] - OT.tts(p, T)) <= 1e-9 * OT.tts(p, T)
    with pytest.raises(RuntimeError):
        PT.tts_from_runs(np.array([egs - 1, egs]), np.array([3, 4]), egs)


def test_quantise_equals_library_rounding():
    """The package's 16.16 rounding is the library's llround (the instance
    couplings the trace counts are weighted with)."""
    for x in (0.5, 1.0, 2.5, 4.0, 7.0, -3.3, 1e-5, 0.123456, -0.5 / 65536, 1.5 / 65536):
        assert PT.quantise(x) == oracle.quantise(x), x


def test_min_energy_rejects_bad_arguments():
    lib = crbm.lib()
    w = (ct.c_int64 * 3)(1, 2, 3)
    buf = (ct.c_int64 * 4)()
    p = ct.cast(buf, ct.c_void_p)
    bad = [
        (None, 1, 4, 0, 4, w, 0, 1, 1, p, p),      # trace missing with samples
        (p, 1, 4, 0, 4, w, 0, 1, 1, None, p),      # no emin
        (p, 1, 4, 0, 4, w, 0, 1, 1, p, None),      # no first
        (p, 1, 4, 2, 2, w, 0, 1, 1, p, p),         # empty chain range
        (p, 1, 4, 0, 5, w, 0, 1, 1, p, p),         # range beyond the trace
        (p, 1, 4, -1, 2, w, 0, 1, 1, p, p),        # negative c0
        (p, 1, 4, 0, 4, w, -1, 1, 1, p, p),        # negative sweep0
        (p, 1, 4, 0, 4, w, 0, 0, 1, p, p),         # trace_every < 1
        (p, -1, 4, 0, 4, w, 0, 1, 1, p, p),        # negative sample count
        (p, 1, 4, 0, 4, (ct.c_int64 * 3)(1 << 31, 0, 0), 0, 1, 1, p, p),  # |w| too large
        (p, 1, 4, 0, 4, None, 0, 1, 1, p, p),      # no weights
    ]
    for args in bad:
        assert lib.crbm_min_energy(*args, None) == -1, args
        assert "crbm_min_energy" in lib.crbm_last_error().decode()
