"""Host post-processing of the phase-diagram experiments (paper_2511_20911_amd.phase):
the structure factor from displacement sums, the T = 0 transition fields and
step detection on magnetisation curves."""
import math

import numpy as np
import pytest

import oracle
from paper_2511_20911_amd import phase


@pytest.mark.parametrize("rows,cols", [(18, 12), (6, 8)])
def test_structure_factor_equals_direct_sum(rows, cols):
    """Eq. (13) from the displacement sums equals |sum_r s_r e^{i q.r}|^2 / N^2
    averaged over the states, at grid and off-grid wave vectors."""
    rng = np.random.default_rng(rows + cols)
    states = (2 * rng.integers(0, 2, (7, rows, cols)) - 1).astype(np.int8)
    cn = sum(oracle.lattice_corr(rows, cols, s) for s in states)
    qr = np.array([0.0, math.pi, 2 * math.pi / 3, 0.37])
    qc = np.array([0.0, 2 * math.pi / 3, math.pi, 1.91, 5.2])
    S = phase.structure_factor(cn, len(states), rows, cols, qr, qc)
    rr, cc = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    N = rows * cols
    for a, x in enumerate(qr):
        for b, y in enumerate(qc):
            d = np.mean([abs((s * np.exp(1j * (x * rr + y * cc))).sum()) ** 2 for s in states]) / N ** 2
            assert abs(S[a, b] - d) < 1e-12


def test_structure_factor_of_ordered_states():
    """A perfect UUD plateau state (Sec. III.B: peak at (2 pi/3, pi)) and the
    ferromagnet (Gamma) on a 12 x 18 lattice."""
    rows, cols = 18, 12
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    fm = np.ones((rows, cols), np.int8)
    cn = oracle.lattice_corr(rows, cols, fm)
    assert abs(phase.structure_factor(cn, 1, rows, cols, [0.0], [0.0])[0, 0] - 1.0) < 1e-12
    # up-up-down along the rows, alternating along the columns: wave vector (2 pi/3, pi)
    uud = np.where(r % 3 == 2, -1, 1) * np.where(c % 2 == 0, 1, -1)
    cn = oracle.lattice_corr(rows, cols, uud.astype(np.int8))
    qs = 2 * math.pi * np.arange(36) / 36
    S = phase.structure_factor(cn, 1, rows, cols, qs, qs)
    i, j = np.unravel_index(np.argmax(S), S.shape)
    assert abs(qs[i] - 2 * math.pi / 3) < 1e-12 or abs(qs[i] - 4 * math.pi / 3) < 1e-12
    assert abs(qs[j] - math.pi) < 1e-12


def test_boundaries_T0_closed_forms():
    """The four ordered phases of Sec. III.A give the transitions h = 4 - 2 J2
    (Neel | 1/3), h = 4 + J2 (1/3 | FM), h = J2 - 2 (dimer | 1/3) and J2 = 2
    (Neel | dimer at h = 0)."""
    for J2 in (0.5, 1.0, 1.5):
        assert np.allclose(phase.boundaries_T0(J2), [4 - 2 * J2, 4 + J2], atol=1e-4)
    for J2 in (2.5, 3.0):
        assert np.allclose(phase.boundaries_T0(J2), [J2 - 2, 4 + J2], atol=1e-4)
    assert phase.boundaries_T0(0.0, h_max=3.9) == []


def test_transition_fields_of_smoothed_steps():
    hs = np.linspace(0, 8, 65)
    m = (1 / 3) / (1 + np.exp(-(hs - 2.0) / 0.1)) + (2 / 3) / (1 + np.exp(-(hs - 5.0) / 0.1))
    f = phase.transition_fields(hs, m)
    assert len(f) == 2 and abs(f[0] - 2.0) < 0.02 and abs(f[1] - 5.0) < 0.02
    assert phase.transition_fields(hs, np.full_like(hs, 0.3)) == []
