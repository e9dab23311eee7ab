"""Host-side checks of the HIP library that need no GPU: it loads, exports
every symbol of include/crbm.h, and its host-built tables equal what the
oracle computes from the same conventions."""
import os
import re

import numpy as np
import pytest

import oracle
import paper_2511_20911_amd as crbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(crbm_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = crbm.lib()
    names = _declared_functions()
    assert "crbm_create" in names and "crbm_sample" in names and "crbm_observables" in names
    for n in sorted(names):
        assert hasattr(lib, n), n


def test_threshold_equals_oracle():
    ys = np.unique(np.concatenate([np.arange(0, 5000), np.geomspace(1, 5e7, 3000).astype(np.int64)]))
    for y in ys:
        assert crbm.threshold(int(y)) == oracle.threshold(int(y)), y


def _oracle_table(J1, J2, h, T):
    wq1, s1 = oracle.bond_weight(oracle.quantise(J1), T)
    wq2, s2 = oracle.bond_weight(oracle.quantise(J2), T)
    aq = oracle.visible_bias(oracle.quantise(h), T)
    tab = np.zeros(16, np.uint32)
    tab[0] = oracle.threshold(2 * wq1)
    tab[1] = oracle.threshold(2 * wq2)
    kge = [5, 5]
    for d in (0, 1):
        for n in range(5):
            x = aq + wq1 * (2 * n - 4) + wq2 * (2 * d - 1)
            tab[3 + 2 * n + d] = oracle.threshold(abs(x))
            if x >= 0 and kge[d] == 5:
                kge[d] = n
    tab[2] = (s1 < 0) | ((s2 < 0) << 1) | ((wq1 != 0) << 2) | ((wq2 != 0) << 3) | (kge[0] << 8) | (kge[1] << 12)
    return tab


@pytest.mark.parametrize("J1,J2,h", [(1.0, 0.5, 0.0), (1.0, 1.0, 3.0), (1.0, 2.5, -1.25), (-0.5, 0.0, 7.0),
                                     (1.0, 1.5, 4.5), (0.0, 1.0, 0.3)])
def test_tables_equal_oracle(J1, J2, h):
    for T in np.geomspace(0.05, 5.0, 37):
        assert np.array_equal(crbm.table_for(J1, J2, h, float(T)), _oracle_table(J1, J2, h, float(T))), T


def test_table_errors():
    with pytest.raises(crbm.CrbmError) as e:
        crbm.table_for(1.0, 0.5, 0.0, 0.0)
    assert e.value.code == crbm.CRBM_EINVAL
    with pytest.raises(crbm.CrbmError) as e:
        crbm.table_for(1.0, 0.5, 0.0, float("nan"))
    assert e.value.code == crbm.CRBM_EINVAL
    with pytest.raises(crbm.CrbmError) as e:
        crbm.table_for(40000.0, 0.5, 0.0, 1.0)
    assert e.value.code == crbm.CRBM_ERANGE
    with pytest.raises(crbm.CrbmError) as e:
        crbm.table_for(1.0, 0.5, 0.0, 1e-6)  # weights beyond int32 in 16.16
    assert e.value.code == crbm.CRBM_ERANGE


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N > 1 exits with a message instead of measuring."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("Lr,Lc,orr,oc,seed", [(6, 8, True, True, 1), (8, 6, False, True, 2), (6, 6, True, False, 3),
                                               (4, 4, False, False, 4)])
def test_lattice_tables_equal_oracle_fields(Lr, Lc, orr, oc, seed):
    """The general-lattice table (crbm_lattice_table, host only): the hidden
    threshold of every filter is t(2 wq_k) from the oracle's weights, and for
    every site the 32 visible entries of its (sublattice, edge) type are the
    thresholds and signs of aq + sum of +-wq over the site's present bonds in
    the oracle's geometry, every sign combination once per value of the bits
    of absent bonds."""
    rng = np.random.default_rng(seed)
    J = list(rng.uniform(-2.0, 2.0, 10))
    J[6] = 0.0
    he, ho, T = 1.7, -0.9, 0.8
    lat = crbm.Lattice(rows=Lr, cols=Lc, J=J, h_even=he, h_odd=ho, open_rows=orr, open_cols=oc)
    tab = crbm.lattice_table(lat, T).astype(np.int64)
    wq, sg = zip(*[oracle.bond_weight(oracle.quantise(x), T) for x in J])
    aq = [oracle.visible_bias(oracle.quantise(he), T), oracle.visible_bias(oracle.quantise(ho), T)]
    for k in range(10):
        assert tab[k] == (oracle.threshold(2 * wq[k]) if wq[k] else 1 << 31)
        assert ((int(tab[10]) >> k) & 1) == (sg[k] < 0) and ((int(tab[11]) >> k) & 1) == (wq[k] != 0)
    ol = oracle.Lattice(Lr, Lc, J, he, ho, open_r=orr, open_c=oc, T0=T)
    inc = {}
    for k in range(10):
        for i in range(Lr // 2):
            for j in range(Lc // 2):
                b = oracle.lattice_bond(ol, k, i, j)
                if b is not None:
                    inc.setdefault(b[0], []).append(wq[k])
                    inc.setdefault(b[1], []).append(wq[k])
    import itertools
    for r in range(Lr):
        for c in range(Lc):
            ws = inc[(r, c)]
            assert len(ws) <= 5
            cls = 2 * (r % 2) + (c % 2)
            redge = orr and (r == 0 if r % 2 == 0 else r == Lr - 1)
            cedge = oc and (c == 0 if c % 2 == 0 else c == Lc - 1)
            typ = (cls * 2 + int(redge)) * 2 + int(cedge)
            want = []
            for signs in itertools.product((-1, 1), repeat=len(ws)):
                x = aq[c % 2] + sum(s * w for s, w in zip(signs, ws))
                want += [(oracle.threshold(abs(x)), int(x >= 0))] * (1 << (5 - len(ws)))
            got = []
            for pat in range(32):
                e = typ * 32 + pat
                t = int(tab[16 + 512 + e])
                hi = t >> 16
                tc = min(0xffff, hi + (1 if t & 0xffff else 0))
                assert int(tab[16 + e]) == (tc | (hi << 16))
                got.append((t, (int(tab[16 + 1024 + e // 32]) >> (e % 32)) & 1))
            assert sorted(got) == sorted(want), (r, c)
