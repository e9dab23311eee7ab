"""CPU oracle for the CRBM Gibbs sampler of the Shastry-Sutherland Ising lattice.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the product path never does.  It wraps
the plain single-threaded C oracle (``crbm_oracle.c``) with ctypes and adds the
numpy parts (autoregressive network, Metropolis-Hastings, autocorrelation
statistics).  Nothing here is shared with the HIP library.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "crbm_oracle.c")

SCHED = {"const": 0, "linear": 1, "geometric": 2, "explicit": 3}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, no intrinsics, single-threaded)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Instance(ct.Structure):
    _fields_ = [
        ("L", ct.c_int32),
        ("J1", ct.c_double),
        ("J2", ct.c_double),
        ("h", ct.c_double),
        ("sched_kind", ct.c_int32),
        ("T0", ct.c_double),
        ("T1", ct.c_double),
        ("T_explicit", ct.POINTER(ct.c_double)),
        ("id", ct.c_uint32),
        ("precision", ct.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ct.CDLL(_LIB_PATH)
        u32, i64, i32, dbl = ct.c_uint32, ct.c_int64, ct.c_int32, ct.c_double
        p = ct.POINTER
        L.oracle_philox4x32_10.argtypes = [p(u32), p(u32), p(u32)]
        L.oracle_uniform_hidden.argtypes = [ct.c_uint64, u32, u32, u32, ct.c_int, ct.c_int, ct.c_int, ct.c_int]
        L.oracle_uniform_hidden.restype = u32
        L.oracle_uniform_visible.argtypes = [ct.c_uint64, u32, u32, u32, ct.c_int, ct.c_int, ct.c_int]
        L.oracle_uniform_visible.restype = u32
        L.oracle_quantise.argtypes = [dbl]
        L.oracle_quantise.restype = i64
        L.oracle_schedule_T.argtypes = [ct.c_int, dbl, dbl, p(dbl), i64, i64]
        L.oracle_schedule_T.restype = dbl
        L.oracle_bond_weight.argtypes = [i64, dbl, p(i64), p(ct.c_int)]
        L.oracle_visible_bias.argtypes = [i64, dbl]
        L.oracle_visible_bias.restype = i64
        L.oracle_threshold.argtypes = [i64]
        L.oracle_threshold.restype = u32
        L.oracle_q54.argtypes = [dbl]
        L.oracle_q54.restype = i64
        L.oracle_sigmoid16.argtypes = [i64]
        L.oracle_sigmoid16.restype = u32
        L.oracle_bond_weight_q54.argtypes = [i64, dbl, p(i64), p(ct.c_int)]
        L.oracle_bond_sites.argtypes = [ct.c_int] * 4 + [p(ct.c_int)] * 5
        L.oracle_counts.argtypes = [ct.c_int, p(ct.c_int8), p(i64), p(i64), p(i64)]
        L.oracle_corr.argtypes = [ct.c_int, p(ct.c_int8), p(i64)]
        L.oracle_order.argtypes = [ct.c_int, p(ct.c_int8), p(i64)]
        L.oracle_init_spins.argtypes = [p(_Instance), ct.c_uint64, u32, p(ct.c_int8)]
        L.oracle_run_chain.argtypes = [p(_Instance), i64, ct.c_uint64, u32, i64, i64,
                                       p(ct.c_int8), p(i32), i32, i64, p(i64), p(i64)]
        L.oracle_staggered.argtypes = [ct.c_int, p(ct.c_int8)]
        L.oracle_staggered.restype = i64
        L.oracle_run_chain.restype = ct.c_int
        L.oracle_log_marginal.argtypes = [p(_Instance), i64, i64, p(ct.c_int8)]
        L.oracle_log_marginal.restype = dbl
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ct.POINTER(ctype))


class Instance:
    """One Hamiltonian point: lattice side L, couplings, schedule, RNG id."""

    def __init__(self, L, J1=1.0, J2=0.5, h=0.0, sched="const", T0=1.0, T1=None,
                 T_explicit=None, id=0, precision=0):
        self.L, self.J1, self.J2, self.h = int(L), float(J1), float(J2), float(h)
        self.sched = sched
        self.T0 = float(T0)
        self.T1 = float(T0 if T1 is None else T1)
        self.T_explicit = None if T_explicit is None else np.ascontiguousarray(T_explicit, np.float64)
        self.id = int(id)
        self.precision = int(precision)  # 0: 16.16 / 32-bit; 1: the hardware's Q5.4 / 16-bit

    def c(self) -> _Instance:
        te = None if self.T_explicit is None else _ptr(self.T_explicit, ct.c_double)
        return _Instance(self.L, self.J1, self.J2, self.h, SCHED[self.sched], self.T0, self.T1, te, self.id,
                         self.precision)


# ------------------------------------------------------------------ primitives

def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_ptr(c, ct.c_uint32), _ptr(k, ct.c_uint32), _ptr(o, ct.c_uint32))
    return o


def uniform_hidden(seed, id, chain, sweep, L, k, i, j) -> int:
    return int(lib().oracle_uniform_hidden(seed, id, chain, sweep, L, k, i, j))


def uniform_visible(seed, id, chain, sweep, L, r, c) -> int:
    return int(lib().oracle_uniform_visible(seed, id, chain, sweep, L, r, c))


def quantise(J) -> int:
    return int(lib().oracle_quantise(float(J)))


def schedule_T(inst: Instance, S: int, s: int) -> float:
    te = None if inst.T_explicit is None else _ptr(inst.T_explicit, ct.c_double)
    return float(lib().oracle_schedule_T(SCHED[inst.sched], inst.T0, inst.T1, te, S, s))


def bond_weight(Jq: int, T: float):
    wq = ct.c_int64()
    sg = ct.c_int()
    lib().oracle_bond_weight(int(Jq), float(T), ct.byref(wq), ct.byref(sg))
    return int(wq.value), int(sg.value)


def visible_bias(hq: int, T: float) -> int:
    return int(lib().oracle_visible_bias(int(hq), float(T)))


def threshold(y: int) -> int:
    return int(lib().oracle_threshold(int(y)))


def q54(v: float) -> int:
    """Hardware fixed point (App. A Dimension and Precision) in 2^-16 units."""
    return int(lib().oracle_q54(float(v)))


def sigmoid16(y: int) -> int:
    """Closest 16-bit value of sigmoid(2 y 2^-16) (App. A Sigmoid module)."""
    return int(lib().oracle_sigmoid16(int(y)))


def bond_weight_q54(Jq: int, T: float):
    wq = ct.c_int64()
    sg = ct.c_int()
    lib().oracle_bond_weight_q54(int(Jq), float(T), ct.byref(wq), ct.byref(sg))
    return int(wq.value), int(sg.value)


def bond_sites(L, k, i, j):
    v = [ct.c_int() for _ in range(5)]
    lib().oracle_bond_sites(L, k, i, j, *[ct.byref(x) for x in v])
    ra, ca, rb, cb, t = (x.value for x in v)
    return (ra, ca), (rb, cb), t


def counts(L, spins) -> tuple[int, int, int]:
    s = np.ascontiguousarray(spins, np.int8).reshape(L * L)
    M, B1, B2 = ct.c_int64(), ct.c_int64(), ct.c_int64()
    lib().oracle_counts(L, _ptr(s, ct.c_int8), ct.byref(M), ct.byref(B1), ct.byref(B2))
    return M.value, B1.value, B2.value


def corr(L, spins) -> np.ndarray:
    s = np.ascontiguousarray(spins, np.int8).reshape(L * L)
    out = np.zeros(L * L, np.int64)
    lib().oracle_corr(L, _ptr(s, ct.c_int8), _ptr(out, ct.c_int64))
    return out.reshape(L, L)


def order(L, spins) -> tuple[int, int, int]:
    """(max, |S(pi, 2pi/3)|^2, |S(2pi/3, pi)|^2) of one configuration (exact integers)."""
    s = np.ascontiguousarray(spins, np.int8).reshape(L * L)
    out = np.zeros(3, np.int64)
    lib().oracle_order(L, _ptr(s, ct.c_int8), _ptr(out, ct.c_int64))
    return int(out[0]), int(out[1]), int(out[2])


def init_spins(inst: Instance, seed: int, chain: int) -> np.ndarray:
    s = np.zeros(inst.L * inst.L, np.int8)
    ci = inst.c()
    lib().oracle_init_spins(ct.byref(ci), seed, chain, _ptr(s, ct.c_int8))
    return s.reshape(inst.L, inst.L)


def log_marginal(inst: Instance, S: int, sweep: int, spins) -> float:
    s = np.ascontiguousarray(spins, np.int8).reshape(inst.L * inst.L)
    ci = inst.c()
    return float(lib().oracle_log_marginal(ct.byref(ci), S, sweep, _ptr(s, ct.c_int8)))


N_ACC = 14  # n, M, B1, B2, MM, B1B1, B2B2, MB1, MB2, B1B2, |M|, Ms, MsMs, |Ms|


def staggered(L, spins) -> int:
    """Staggered magnetisation sum (-1)^(r+c) s(r,c) of one configuration."""
    s = np.ascontiguousarray(spins, np.int8).reshape(L * L)
    return int(lib().oracle_staggered(L, _ptr(s, ct.c_int8)))


def run_chain(inst: Instance, S: int, seed: int, chain: int, sweep_begin: int, sweep_end: int,
              spins=None, trace=False, measure_every=0, burn_in=0, acc=None, corr=None):
    """Run sweeps [sweep_begin, sweep_end) of one chain.

    spins: None -> initialise from the init stream; else an (L, L) int8 array
    of +-1 (copied).  corr: None, or an int64 array of L*L entries to which
    C(dr, dc) of the state after every measured sweep is added.
    Returns (spins, trace or None, acc)."""
    L = inst.L
    if spins is None:
        s = init_spins(inst, seed, chain).reshape(L * L).copy()
    else:
        s = np.ascontiguousarray(spins, np.int8).reshape(L * L).copy()
    n = sweep_end - sweep_begin
    tr = np.zeros((n, 3), np.int32) if trace else None
    a = np.zeros(N_ACC, np.int64) if acc is None else acc
    ci = inst.c()
    rc = lib().oracle_run_chain(
        ct.byref(ci), S, seed, chain, sweep_begin, sweep_end, _ptr(s, ct.c_int8),
        _ptr(tr, ct.c_int32) if trace else None, measure_every, burn_in, _ptr(a, ct.c_int64),
        None if corr is None else _ptr(corr, ct.c_int64))
    if rc != 0:
        raise RuntimeError(f"oracle_run_chain failed: {rc}")
    return s.reshape(L, L), tr, a


# ------------------------------------------------------------- general lattices

class _Lattice(ct.Structure):
    _fields_ = [
        ("Lr", ct.c_int32), ("Lc", ct.c_int32),
        ("open_r", ct.c_int32), ("open_c", ct.c_int32),
        ("J", ct.c_double * 10),
        ("h_even", ct.c_double), ("h_odd", ct.c_double),
        ("sched_kind", ct.c_int32),
        ("T0", ct.c_double), ("T1", ct.c_double),
        ("T_explicit", ct.POINTER(ct.c_double)),
        ("id", ct.c_uint32),
    ]


LATTICE_N_ACC = 18  # n, M_e, M_o, B_0..B_9, sum M^2, sum |M|, sum Ms, sum Ms^2, sum |Ms|


def ss_filters(J1, J2):
    """Per-filter couplings of the Shastry-Sutherland lattice: k0-k7 square edges, k8-k9 dimers."""
    return [float(J1)] * 8 + [float(J2)] * 2


class Lattice:
    """A general lattice: Lr x Lc, open or periodic per axis, one coupling per
    filter (App. A Convoluter-Reverse), a field per column parity (App. A
    Accumulator), a temperature schedule and an RNG id."""

    def __init__(self, Lr, Lc, J, h_even=0.0, h_odd=None, open_r=False, open_c=False, sched="const", T0=1.0,
                 T1=None, T_explicit=None, id=0):
        self.Lr, self.Lc = int(Lr), int(Lc)
        self.open_r, self.open_c = bool(open_r), bool(open_c)
        self.J = [float(x) for x in J]
        assert len(self.J) == 10
        self.h_even = float(h_even)
        self.h_odd = float(h_even if h_odd is None else h_odd)
        self.sched = sched
        self.T0 = float(T0)
        self.T1 = float(T0 if T1 is None else T1)
        self.T_explicit = None if T_explicit is None else np.ascontiguousarray(T_explicit, np.float64)
        self.id = int(id)

    def c(self) -> _Lattice:
        te = None if self.T_explicit is None else _ptr(self.T_explicit, ct.c_double)
        return _Lattice(self.Lr, self.Lc, int(self.open_r), int(self.open_c), (ct.c_double * 10)(*self.J),
                        self.h_even, self.h_odd, SCHED[self.sched], self.T0, self.T1, te, self.id)


def _lattice_lib():
    L = lib()
    if not getattr(L, "_lattice_ready", False):
        i64, i32, u32 = ct.c_int64, ct.c_int32, ct.c_uint32
        p = ct.POINTER
        L.oracle_lattice_bond.argtypes = [p(_Lattice), ct.c_int, ct.c_int, ct.c_int] + [p(ct.c_int)] * 4
        L.oracle_lattice_bond.restype = ct.c_int
        L.oracle_lattice_counts.argtypes = [p(_Lattice), p(ct.c_int8), p(i64)]
        L.oracle_lattice_corr.argtypes = [ct.c_int, ct.c_int, p(ct.c_int8), p(i64)]
        L.oracle_lattice_init_spins.argtypes = [p(_Lattice), ct.c_uint64, u32, p(ct.c_int8)]
        L.oracle_lattice_run_chain.argtypes = [p(_Lattice), i64, ct.c_uint64, u32, i64, i64, p(ct.c_int8), p(i32),
                                               i32, i64, p(i64), p(i64)]
        L.oracle_lattice_run_chain.restype = ct.c_int
        L.oracle_lattice_log_marginal.argtypes = [p(_Lattice), i64, i64, p(ct.c_int8)]
        L.oracle_lattice_log_marginal.restype = ct.c_double
        L._lattice_ready = True
    return L


def lattice_bond(lat: Lattice, k, i, j):
    """((ra, ca), (rb, cb)) of bond k of cell (i, j), or None if it is absent."""
    v = [ct.c_int() for _ in range(4)]
    ci = lat.c()
    if not _lattice_lib().oracle_lattice_bond(ct.byref(ci), k, i, j, *[ct.byref(x) for x in v]):
        return None
    ra, ca, rb, cb = (x.value for x in v)
    return (ra, ca), (rb, cb)


def lattice_counts(lat: Lattice, spins) -> np.ndarray:
    """(M_even, M_odd, B_0, ..., B_9) of one configuration."""
    s = np.ascontiguousarray(spins, np.int8).reshape(lat.Lr * lat.Lc)
    out = np.zeros(12, np.int64)
    ci = lat.c()
    _lattice_lib().oracle_lattice_counts(ct.byref(ci), _ptr(s, ct.c_int8), _ptr(out, ct.c_int64))
    return out


def lattice_corr(Lr, Lc, spins) -> np.ndarray:
    """Cn[dr, dc + Lc - 1] = sum of s(r,c) s(r+dr, c+dc) over pairs inside the lattice (no wrap)."""
    s = np.ascontiguousarray(spins, np.int8).reshape(Lr * Lc)
    out = np.zeros(Lr * (2 * Lc - 1), np.int64)
    _lattice_lib().oracle_lattice_corr(Lr, Lc, _ptr(s, ct.c_int8), _ptr(out, ct.c_int64))
    return out.reshape(Lr, 2 * Lc - 1)


def lattice_init_spins(lat: Lattice, seed: int, chain: int) -> np.ndarray:
    s = np.zeros(lat.Lr * lat.Lc, np.int8)
    ci = lat.c()
    _lattice_lib().oracle_lattice_init_spins(ct.byref(ci), seed, chain, _ptr(s, ct.c_int8))
    return s.reshape(lat.Lr, lat.Lc)


def lattice_log_marginal(lat: Lattice, S: int, sweep: int, spins) -> float:
    s = np.ascontiguousarray(spins, np.int8).reshape(lat.Lr * lat.Lc)
    ci = lat.c()
    return float(_lattice_lib().oracle_lattice_log_marginal(ct.byref(ci), S, sweep, _ptr(s, ct.c_int8)))


def run_lattice_chain(lat: Lattice, S: int, seed: int, chain: int, sweep_begin: int, sweep_end: int,
                      spins=None, trace=False, measure_every=0, burn_in=0, acc=None, corr=None):
    """Sweeps [sweep_begin, sweep_end) of one chain of a general lattice.
    Returns (spins [Lr, Lc], trace [n, 12] of (M_e, M_o, B_0..B_9) or None, acc)."""
    n_sites = lat.Lr * lat.Lc
    if spins is None:
        s = lattice_init_spins(lat, seed, chain).reshape(n_sites).copy()
    else:
        s = np.ascontiguousarray(spins, np.int8).reshape(n_sites).copy()
    n = sweep_end - sweep_begin
    tr = np.zeros((n, 12), np.int32) if trace else None
    a = np.zeros(LATTICE_N_ACC, np.int64) if acc is None else acc
    ci = lat.c()
    rc = _lattice_lib().oracle_lattice_run_chain(
        ct.byref(ci), S, seed, chain, sweep_begin, sweep_end, _ptr(s, ct.c_int8),
        _ptr(tr, ct.c_int32) if trace else None, measure_every, burn_in, _ptr(a, ct.c_int64),
        None if corr is None else _ptr(corr, ct.c_int64))
    if rc != 0:
        raise RuntimeError(f"oracle_lattice_run_chain failed: {rc}")
    return s.reshape(lat.Lr, lat.Lc), tr, a
