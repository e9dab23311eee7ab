"""The hardware-precision mode (App. A Dimension and Precision; Sigmoid and
LFSR-Forward) without a GPU: the oracle's Q5.4 rounding and 16-bit sigmoid
against their definitions; the oracle's chains in this mode against the exact
law of the effective Ising model that Q5.4 weights encode (row transfer
matrix); the library's tables against the same tables composed from oracle
primitives; argument checks."""
import ctypes as ct
import math

import numpy as np
import pytest

import oracle
from oracle import exact as EX
import paper_2511_20911_amd as crbm

STEP = 4096


def test_q54_rounding_and_saturation():
    assert oracle.q54(0.0) == 0
    assert oracle.q54(1.0 / 32) == STEP           # half a step rounds away from zero
    assert oracle.q54(-1.0 / 32) == -STEP
    assert oracle.q54(0.03) == 0                  # 0.48 of a step
    assert oracle.q54(1.0) == 16 * STEP
    assert oracle.q54(31.9) == 510 * STEP
    assert oracle.q54(31.97) == 511 * STEP        # 511.5 steps saturate at 511
    assert oracle.q54(1e6) == 511 * STEP and oracle.q54(-1e6) == -511 * STEP
    for v in np.linspace(-40, 40, 2001):
        q = oracle.q54(float(v))
        assert q % STEP == 0 and abs(q) <= 511 * STEP
        if abs(v) < 31.9:
            assert abs(q / 65536.0 - v) <= 1.0 / 32 + 1e-12


def test_sigmoid16_is_the_closest_16_bit_value():
    assert oracle.sigmoid16(0) == 32768
    assert oracle.sigmoid16(1 << 30) == 65535
    prev = 0
    for y in np.unique(np.geomspace(1, 2e7, 4000).astype(np.int64)):
        t = oracle.sigmoid16(int(y))
        p = 1.0 / (1.0 + math.exp(-2.0 * y / 65536.0))
        assert t >= prev and 32768 <= t <= 65535
        if t < 65535:
            assert abs(t - 65536.0 * p) <= 0.5 + 1e-9
        prev = t


def _effective(J, T, wq_q54):
    """Coupling whose Ising factor the hidden unit of weight w' encodes:
    summing it out gives cosh(2w') = exp(2|K'|) (Sec. II.A Eq. (4))."""
    w = wq_q54 / 65536.0
    return math.copysign(T * 0.5 * math.log(math.cosh(2.0 * w)), J)


def test_hardware_precision_chain_samples_the_effective_model():
    """At J1 = J2 = 1, h = 3, T = 1 the weights round to 22/16 (from 1.344),
    so the hidden units encode J' = 1.0305; the 6x6 oracle chains in this mode
    reproduce the exact <E'>/N and <m> of (J', J', h) within 3 SE (the 16-bit
    sigmoid changes each probability by at most 2^-17)."""
    L, T, J, h = 6, 1.0, 1.0, 3.0
    wq, _ = oracle.bond_weight_q54(oracle.quantise(J), T)
    assert wq == 22 * STEP
    Jp = _effective(J, T, wq)
    a = oracle.q54(h / T) / 65536.0
    hp = a * T
    assert abs(Jp - 1.0305) < 1e-3 and hp == 3.0
    inst = oracle.Instance(L, J, J, h, "const", T, id=7, precision=1)
    burn, S = 200, 1400
    E_means, m_means = [], []
    for ch in range(48):
        _, tr, _ = oracle.run_chain(inst, S, 0xABC, ch, 0, S, trace=True)
        tr = tr[burn:].astype(np.float64)
        E_means.append(((Jp * tr[:, 1] + Jp * tr[:, 2] - hp * tr[:, 0]) / (L * L)).mean())
        m_means.append(tr[:, 0].mean() / (L * L))
    ex = EX.tm_averages(L, Jp, Jp, hp, T)
    for vals, ref in ((E_means, ex["E"]), (m_means, ex["m"])):
        v = np.array(vals)
        se = v.std(ddof=1) / math.sqrt(len(v))
        assert abs(v.mean() - ref) < 3 * se, (v.mean(), ref, se)


def _oracle_table_q54(J1, J2, h, T):
    wq1, s1 = oracle.bond_weight_q54(oracle.quantise(J1), T)
    wq2, s2 = oracle.bond_weight_q54(oracle.quantise(J2), T)
    aq = oracle.q54(oracle.quantise(h) / 65536.0 / T)
    tab = np.zeros(16, np.uint32)
    tab[0] = oracle.sigmoid16(min(2 * wq1, 511 * STEP)) << 16
    tab[1] = oracle.sigmoid16(min(2 * wq2, 511 * STEP)) << 16
    kge = [5, 5]
    for d in (0, 1):
        for n in range(5):
            x = aq + wq1 * (2 * n - 4) + wq2 * (2 * d - 1)
            x = max(-2047 * STEP, min(2047 * STEP, x))
            tab[3 + 2 * n + d] = oracle.sigmoid16(abs(x)) << 16
            if x >= 0 and kge[d] == 5:
                kge[d] = n
    tab[2] = (s1 < 0) | ((s2 < 0) << 1) | ((wq1 != 0) << 2) | ((wq2 != 0) << 3) | (kge[0] << 8) | (kge[1] << 12)
    return tab


@pytest.mark.parametrize("J1,J2,h", [(1.0, 0.5, 0.0), (1.0, 1.0, 3.0), (1.0, 2.5, -1.25), (-0.5, 0.0, 7.0),
                                     (1.0, 1.5, 4.5), (0.0, 1.0, 0.3), (1.0, 0.02, 0.01)])
def test_hardware_precision_tables_equal_oracle(J1, J2, h):
    """Down to T = 0.005, where the weights, the bias, the hidden field and the
    visible accumulator all saturate."""
    for T in np.geomspace(0.005, 5.0, 41):
        got = crbm.table_for(J1, J2, h, float(T), precision="fpga")
        assert np.array_equal(got, _oracle_table_q54(J1, J2, h, float(T))), T
        assert (got[[0, 1] + list(range(3, 13))] & 0xFFFF).sum() == 0  # 16-bit thresholds
        assert got[0] >= (1 << 31) and got[1] >= (1 << 31)


def test_default_precision_tables_unchanged():
    for T in (0.1, 0.7, 3.0):
        assert np.array_equal(crbm.table_for(1.0, 1.0, 3.0, T), crbm.table_for(1.0, 1.0, 3.0, T, precision="q16"))


def test_precision_argument_checks():
    lib = crbm.lib()
    out = (ct.c_uint32 * 16)()
    assert lib.crbm_table_for_precision(1.0, 1.0, 0.0, 1.0, 2, out) == crbm.CRBM_EINVAL
    assert lib.crbm_table_for_precision(1.0, 1.0, 0.0, 1.0, -1, out) == crbm.CRBM_EINVAL
    assert lib.crbm_table_for_precision(1.0, 1.0, 0.0, 0.0, 1, out) == crbm.CRBM_EINVAL
    assert lib.crbm_table_for_precision(1.0, 1.0, 0.0, 1.0, 1, None) == crbm.CRBM_EINVAL
    # crbm_create checks the config before touching the device
    inst = crbm._Instance(6, 1, 1.0, 1.0, 0.0, 4, 0, 1.0, 1.0, None, 0)
    for bad in (2, -1):
        cfg = crbm._Config(1, 10, 0, 0, None, 0, 0, 0, bad)
        h = ct.c_void_p()
        assert lib.crbm_create(ct.byref(inst), 1, ct.byref(cfg), ct.byref(h)) == crbm.CRBM_EINVAL
        assert "precision" in lib.crbm_last_error().decode()
