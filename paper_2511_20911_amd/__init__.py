"""Python binding of libcrbm.so: CRBM block-Gibbs sampling of the classical
Shastry-Sutherland Ising lattice on MI355X (gfx950).

This module only marshals arguments to the C ABI of ``include/crbm.h``; every
step of the sampler runs in the library's HIP kernels.  PyTorch provides device
memory and the stream.  Importing works without a GPU; creating a sampler
needs the built library and a GPU, and fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcrbm.so")

CRBM_OK, CRBM_EINVAL, CRBM_ERANGE, CRBM_ENOMEM, CRBM_EHIP, CRBM_EUNSUPPORTED, CRBM_ESTATE = 0, -1, -2, -3, -4, -5, -6
SCHED = {"const": 0, "linear": 1, "geometric": 2, "explicit": 3}
N_ACC = 14
MAX_L = 96
SUPPORTED_L = tuple(range(4, 33, 2)) + (36, 40, 48, 64, 72, 96)


class CrbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"crbm error {code}: {msg}")
        self.code = code


class _Instance(ct.Structure):
    _fields_ = [
        ("L", ct.c_int32), ("periodic", ct.c_int32),
        ("J1", ct.c_double), ("J2", ct.c_double), ("h", ct.c_double),
        ("n_chains", ct.c_int32), ("sched_kind", ct.c_int32),
        ("T0", ct.c_double), ("T1", ct.c_double),
        ("T_explicit", ct.POINTER(ct.c_double)),
        ("id", ct.c_uint32),
    ]


class _Config(ct.Structure):
    _fields_ = [
        ("seed", ct.c_uint64), ("n_sweeps", ct.c_int64), ("measure_every", ct.c_int32),
        ("burn_in", ct.c_int64), ("stream", ct.c_void_p), ("tile_rows", ct.c_int32),
        ("launch_mode", ct.c_int32), ("waves_per_block", ct.c_int32), ("precision", ct.c_int32),
        ("flags", ct.c_uint32),
    ]


CRBM_F_CORR = 1


LAUNCH = {"direct": 0, "graph": 1}
PRECISION = {"q16": 0, "fpga": 1}


class _Obs(ct.Structure):
    _fields_ = [
        ("n_samples", ct.c_int64),
        ("sum_M", ct.c_int64), ("sum_B1", ct.c_int64), ("sum_B2", ct.c_int64),
        ("sum_MM", ct.c_int64), ("sum_B1B1", ct.c_int64), ("sum_B2B2", ct.c_int64),
        ("sum_MB1", ct.c_int64), ("sum_MB2", ct.c_int64), ("sum_B1B2", ct.c_int64),
        ("sum_absM", ct.c_int64),
        ("sum_Ms", ct.c_int64), ("sum_MsMs", ct.c_int64), ("sum_absMs", ct.c_int64),
        ("E_per_spin", ct.c_double), ("m", ct.c_double), ("abs_m", ct.c_double),
        ("dimer", ct.c_double), ("E_var_per_spin", ct.c_double), ("abs_stag_m", ct.c_double),
    ]


class _ARConfig(ct.Structure):
    _fields_ = [("L", ct.c_int32), ("channels", ct.c_int32), ("layers", ct.c_int32), ("seed", ct.c_uint64),
                ("stream", ct.c_void_p), ("cond_points", ct.c_int32)]


class _TrainOpts(ct.Structure):
    _fields_ = [("steps", ct.c_int64), ("batch", ct.c_int64), ("lr", ct.c_float), ("lr_late", ct.c_float),
                ("late_from", ct.c_double), ("seed", ct.c_uint64), ("step0", ct.c_int64), ("augment", ct.c_int32)]


class _Lattice(ct.Structure):
    _fields_ = [("rows", ct.c_int32), ("cols", ct.c_int32), ("open_rows", ct.c_int32), ("open_cols", ct.c_int32),
                ("J", ct.c_double * 10), ("h_even", ct.c_double), ("h_odd", ct.c_double),
                ("n_chains", ct.c_int32), ("sched_kind", ct.c_int32), ("T0", ct.c_double), ("T1", ct.c_double),
                ("T_explicit", ct.POINTER(ct.c_double)), ("id", ct.c_uint32)]


LAT_N_ACC = 18
LAT_TAB_WORDS = 1056


_lib = None


def lib() -> ct.CDLL:
    """Load libcrbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2511_20911_amd.build`")
        L = ct.CDLL(LIB_PATH)
        p = ct.POINTER
        L.crbm_create.argtypes = [p(_Instance), ct.c_int32, p(_Config), p(ct.c_void_p)]
        L.crbm_sample.argtypes = [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p]
        L.crbm_sample_thinned.argtypes = [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int32]
        L.crbm_observables.argtypes = [ct.c_void_p, p(_Obs), ct.c_void_p]
        L.crbm_get_state.argtypes = [ct.c_void_p, ct.c_void_p, p(ct.c_int64)]
        L.crbm_set_state.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int64]
        L.crbm_total_chains.argtypes = [ct.c_void_p]
        L.crbm_total_chains.restype = ct.c_int64
        L.crbm_reset_observables.argtypes = [ct.c_void_p]
        L.crbm_destroy.argtypes = [ct.c_void_p]
        L.crbm_destroy.restype = None
        L.crbm_last_error.restype = ct.c_char_p
        L.crbm_threshold.argtypes = [ct.c_int64]
        L.crbm_threshold.restype = ct.c_uint32
        L.crbm_sweep_table.argtypes = [ct.c_void_p, ct.c_int32, ct.c_int64, p(ct.c_uint32)]
        L.crbm_table_for.argtypes = [ct.c_double, ct.c_double, ct.c_double, ct.c_double, p(ct.c_uint32)]
        L.crbm_table_for_precision.argtypes = [ct.c_double, ct.c_double, ct.c_double, ct.c_double, ct.c_int32,
                                               p(ct.c_uint32)]
        L.crbm_autotune.argtypes = [ct.c_int32, ct.c_int32, ct.c_int32, ct.c_void_p, p(ct.c_int32), p(ct.c_int32),
                                    p(ct.c_double)]
        L.crbm_set_tiling.argtypes = [ct.c_int32, ct.c_int32, ct.c_int32]
        L.crbm_min_energy.argtypes = [ct.c_void_p, ct.c_int64, ct.c_int64, ct.c_int64, ct.c_int64, p(ct.c_int64),
                                      ct.c_int64, ct.c_int32, ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.crbm_ar_create.argtypes = [p(_ARConfig), p(ct.c_void_p)]
        L.crbm_ar_num_params.argtypes = [ct.c_void_p]
        L.crbm_ar_num_params.restype = ct.c_int64
        L.crbm_ar_set_params.argtypes = [ct.c_void_p, p(ct.c_float), ct.c_int64]
        L.crbm_ar_get_params.argtypes = [ct.c_void_p, p(ct.c_float), ct.c_int64]
        L.crbm_ar_init_params.argtypes = [ct.c_void_p, ct.c_uint64, ct.c_double]
        L.crbm_ar_grad.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int64, p(ct.c_float), p(ct.c_double)]
        L.crbm_ar_train_step.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_float, p(ct.c_double)]
        L.crbm_ar_logq.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p]
        L.crbm_ar_sample.argtypes = [ct.c_void_p, ct.c_int64, ct.c_uint64, ct.c_int64, ct.c_uint32, ct.c_void_p,
                                     ct.c_void_p]
        L.crbm_sample_mh.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_void_p, ct.c_void_p,
                                     p(ct.c_int64)]
        L.crbm_ar_set_points.argtypes = [ct.c_void_p, ct.c_int32, p(ct.c_double)]
        L.crbm_ar_grad_cond.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, p(ct.c_float),
                                        p(ct.c_double)]
        L.crbm_ar_train_step_cond.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_float,
                                              p(ct.c_double)]
        L.crbm_ar_logq_cond.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p]
        L.crbm_ar_sample_cond.argtypes = [ct.c_void_p, ct.c_int64, ct.c_uint64, ct.c_int64, ct.c_uint32,
                                          ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.crbm_ar_sample_steps.argtypes = [ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_uint64, ct.c_int64, ct.c_uint32,
                                           ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.crbm_ar_train.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, p(_TrainOpts),
                                    p(ct.c_double)]
        L.crbm_ar_batch.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_int64, ct.c_uint64,
                                    ct.c_int64, ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.crbm_ar_destroy.argtypes = [ct.c_void_p]
        L.crbm_ar_destroy.restype = None
        L.crbm_tau_int.argtypes = [ct.c_void_p, ct.c_int64, ct.c_int64, ct.c_int64, ct.c_int64, ct.c_int64,
                                   p(ct.c_double), ct.c_int32, ct.c_double, ct.c_void_p, p(ct.c_double),
                                   p(ct.c_double), p(ct.c_int32), p(ct.c_double)]
        L.crbm_tau_int_noalloc.argtypes = L.crbm_tau_int.argtypes
        L.crbm_get_tiling.argtypes = [ct.c_int32, p(ct.c_int32), p(ct.c_int32)]
        L.crbm_debug_fail_alloc.argtypes = [ct.c_int32]
        L.crbm_debug_tail_cap.argtypes = [ct.c_int32]
        L.crbm_lattice_create.argtypes = [p(_Lattice), ct.c_int32, p(_Config), p(ct.c_void_p)]
        L.crbm_lattice_sample.argtypes = [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_int32]
        L.crbm_lattice_observables.argtypes = [ct.c_void_p, p(ct.c_int64), ct.c_void_p]
        L.crbm_lattice_reset_observables.argtypes = [ct.c_void_p]
        L.crbm_lattice_get_state.argtypes = [ct.c_void_p, ct.c_void_p, p(ct.c_int64)]
        L.crbm_lattice_set_state.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_int64]
        L.crbm_lattice_total_chains.argtypes = [ct.c_void_p]
        L.crbm_lattice_total_chains.restype = ct.c_int64
        L.crbm_lattice_destroy.argtypes = [ct.c_void_p]
        L.crbm_lattice_destroy.restype = None
        L.crbm_lattice_table.argtypes = [p(_Lattice), ct.c_double, p(ct.c_uint32)]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != CRBM_OK:
        raise CrbmError(rc, lib().crbm_last_error().decode())


@dataclass
class Instance:
    """One Hamiltonian point H = J1 sum s s + J2 sum_dimer s s - h sum s on an L x L lattice."""
    L: int
    J1: float = 1.0
    J2: float = 0.5
    h: float = 0.0
    n_chains: int = 1
    sched: str = "const"
    T0: float = 1.0
    T1: Optional[float] = None
    T_explicit: Optional[np.ndarray] = None
    id: int = 0
    periodic: int = 1


def threshold(y: int) -> int:
    """The library's 32-bit sigmoid threshold t(y) (y in 2^16 units)."""
    return int(lib().crbm_threshold(int(y)))


def table_for(J1: float, J2: float, h: float, T: float, precision: str = "q16") -> np.ndarray:
    """The library's 16-word device table for one sweep (host computation)."""
    out = np.zeros(16, np.uint32)
    _check(lib().crbm_table_for_precision(J1, J2, h, T, PRECISION[precision],
                                          out.ctypes.data_as(ct.POINTER(ct.c_uint32))))
    return out


def autotune(L: int, n_chains: int = 4096, n_sweeps: int = 50, stream=None):
    """Time every compiled tiling of lattice side L on this GPU; the fastest
    becomes the process-wide choice.  Returns (rows, waves_per_block, spin-updates/s)."""
    r, w, rate = ct.c_int32(), ct.c_int32(), ct.c_double()
    _check(lib().crbm_autotune(L, n_chains, n_sweeps, _stream_handle(stream), ct.byref(r), ct.byref(w),
                               ct.byref(rate)))
    return int(r.value), int(w.value), float(rate.value)


def tau_int(trace, weights, c0: int = 0, c1: Optional[int] = None, discard: int = 0, max_lag: int = 2000,
            c_window: float = 6.0, stream=None, noalloc: bool = False):
    """tau_int, ESS, window and rho(k) of O = w0 M + w1 B1 + w2 B2 over a
    device counts trace [n_samples, chains, 3] (int32).  noalloc: through
    crbm_tau_int_noalloc (no device allocation; bounded request size)."""
    assert trace.is_cuda and trace.dim() == 3 and trace.shape[2] == 3 and trace.element_size() == 4
    trace = trace.contiguous()
    n, nch = int(trace.shape[0]), int(trace.shape[1])
    c1 = nch if c1 is None else c1
    w = (ct.c_double * 3)(*[float(x) for x in weights])
    K = min(max_lag, n - discard - 1)
    rho = np.zeros(K + 1, np.float64)
    tau, ess, win = ct.c_double(), ct.c_double(), ct.c_int32()
    fn = lib().crbm_tau_int_noalloc if noalloc else lib().crbm_tau_int
    _check(fn(ct.c_void_p(trace.data_ptr()), n, nch, c0, c1, discard, w, max_lag, c_window,
              _stream_handle(stream), ct.byref(tau), ct.byref(ess), ct.byref(win),
              rho.ctypes.data_as(ct.POINTER(ct.c_double))))
    return float(tau.value), float(ess.value), int(win.value), rho


def min_energy(trace, weights, sweep0: int = 0, trace_every: int = 1, c0: int = 0, c1: Optional[int] = None,
               emin=None, first=None, stream=None):
    """Per-chain running minimum of E = w0 M + w1 B1 + w2 B2 over a device
    counts trace [n_samples, chains, 3] (int32) and the number of completed
    sweeps at its first hit (crbm_min_energy).  emin/first: int64 device
    tensors of c1 - c0 entries carrying the minima of earlier traces of the
    same run, or None to start afresh.  Returns (emin, first)."""
    import torch
    assert trace.is_cuda and trace.dim() == 3 and trace.shape[2] == 3 and trace.dtype == torch.int32
    trace = trace.contiguous()
    n, nch = int(trace.shape[0]), int(trace.shape[1])
    c1 = nch if c1 is None else c1
    reset = emin is None
    if reset:
        emin = torch.empty(c1 - c0, dtype=torch.int64, device=trace.device)
        first = torch.empty(c1 - c0, dtype=torch.int64, device=trace.device)
    assert emin.dtype == torch.int64 and first.dtype == torch.int64
    assert emin.numel() >= c1 - c0 and first.numel() >= c1 - c0 and emin.is_contiguous() and first.is_contiguous()
    w = (ct.c_int64 * 3)(*[int(x) for x in weights])
    _check(lib().crbm_min_energy(ct.c_void_p(trace.data_ptr()), n, nch, c0, c1, w, sweep0, trace_every,
                                 1 if reset else 0, ct.c_void_p(emin.data_ptr()), ct.c_void_p(first.data_ptr()),
                                 _stream_handle(stream)))
    return emin, first


def set_tiling(L: int, rows: int, waves_per_block: int = 4):
    _check(lib().crbm_set_tiling(L, rows, waves_per_block))


def get_tiling(L: int):
    r, w = ct.c_int32(), ct.c_int32()
    _check(lib().crbm_get_tiling(L, ct.byref(r), ct.byref(w)))
    return int(r.value), int(w.value)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream)


class Sampler:
    """Handle on crbm_create / crbm_sample / crbm_observables."""

    def __init__(self, instances: Sequence[Instance], seed: int, n_sweeps: int, measure_every: int = 0,
                 burn_in: int = 0, stream=None, tile_rows: int = 0, launch: str = "direct",
                 waves_per_block: int = 0, precision: str = "q16", corr: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the CRBM sampler runs only on the HIP device")
        self.instances = list(instances)
        self._texp = []
        arr = (_Instance * len(self.instances))()
        for k, I in enumerate(self.instances):
            te = None
            if I.sched == "explicit":
                t = np.ascontiguousarray(I.T_explicit, np.float64)
                self._texp.append(t)
                te = t.ctypes.data_as(ct.POINTER(ct.c_double))
            arr[k] = _Instance(I.L, I.periodic, I.J1, I.J2, I.h, I.n_chains, SCHED[I.sched], I.T0,
                               I.T0 if I.T1 is None else I.T1, te, I.id)
        self.stream = stream
        cfg = _Config(seed, n_sweeps, measure_every, burn_in, _stream_handle(stream), tile_rows, LAUNCH[launch],
                      waves_per_block, PRECISION[precision], CRBM_F_CORR if corr else 0)
        h = ct.c_void_p()
        _check(lib().crbm_create(arr, len(self.instances), ct.byref(cfg), ct.byref(h)))
        self._h = h
        self.n_sweeps = n_sweeps
        self.total_chains = int(lib().crbm_total_chains(h))
        self.spin_offsets = np.cumsum([0] + [I.n_chains * I.L * I.L for I in self.instances])
        self.chain_offsets = np.cumsum([0] + [I.n_chains for I in self.instances])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.crbm_destroy(h)
            self._h = None

    def close(self):
        self.__del__()

    @property
    def total_spins(self) -> int:
        return int(self.spin_offsets[-1])

    def sample(self, n_sweeps: int, spins_out=None, trace=None, trace_every: int = 1, order=None):
        """Enqueue n_sweeps sweeps.  spins_out: int8 CUDA tensor of total_spins
        elements; trace: int32 CUDA tensor [n_sweeps // trace_every, total_chains, 3]
        recording the counts after every trace_every-th sweep; order (needs
        trace): same shape, the plateau structure factor (max, |S_A|^2, |S_B|^2)."""
        if spins_out is not None:
            assert spins_out.is_cuda and spins_out.dtype.itemsize == 1 and spins_out.numel() == self.total_spins
        if trace is not None:
            assert trace.is_cuda and trace.element_size() == 4
            assert trace.numel() == (n_sweeps // trace_every) * self.total_chains * 3
        if order is not None:
            assert trace is not None and order.is_cuda and order.element_size() == 4 and order.numel() == trace.numel()
        _check(lib().crbm_sample_thinned(self._h, n_sweeps,
                                         ct.c_void_p(spins_out.data_ptr()) if spins_out is not None else None,
                                         ct.c_void_p(trace.data_ptr()) if trace is not None else None,
                                         ct.c_void_p(order.data_ptr()) if order is not None else None,
                                         int(trace_every)))

    def observables(self, corr: bool = False):
        """Per-instance observables (dicts of the crbm_obs fields); with
        corr, also the per-instance [L, L] int64 sums of C(dr, dc): over the
        measured sweeps for a sampler created with corr=True, else over the
        current state's chains."""
        obs = (_Obs * len(self.instances))()
        cbuf = None
        if corr:
            cbuf = np.zeros(sum(I.L * I.L for I in self.instances), np.int64)
        _check(lib().crbm_observables(self._h, obs, cbuf.ctypes.data_as(ct.c_void_p) if corr else None))
        out = []
        for o in obs:
            out.append({f: getattr(o, f) for f, _ in _Obs._fields_})
        if corr:
            parts, off = [], 0
            for I in self.instances:
                parts.append(cbuf[off:off + I.L * I.L].reshape(I.L, I.L))
                off += I.L * I.L
            return out, parts
        return out

    def reset_observables(self):
        _check(lib().crbm_reset_observables(self._h))

    def get_state(self):
        import torch
        spins = torch.empty(self.total_spins, dtype=torch.int8, device="cuda")
        idx = ct.c_int64()
        _check(lib().crbm_get_state(self._h, ct.c_void_p(spins.data_ptr()), ct.byref(idx)))
        return spins, int(idx.value)

    def set_state(self, spins, sweep_index: int):
        assert spins is None or (spins.is_cuda and spins.numel() == self.total_spins)
        _check(lib().crbm_set_state(self._h, ct.c_void_p(spins.data_ptr()) if spins is not None else None,
                                    int(sweep_index)))

    def split_spins(self, flat):
        """Split a flat [total_spins] tensor into per-instance [n_chains, L, L] views."""
        out = []
        for k, I in enumerate(self.instances):
            a, b = int(self.spin_offsets[k]), int(self.spin_offsets[k + 1])
            out.append(flat[a:b].view(I.n_chains, I.L, I.L))
        return out

    def sweep_table(self, i: int, s: int) -> np.ndarray:
        out = np.zeros(16, np.uint32)
        _check(lib().crbm_sweep_table(self._h, i, s, out.ctypes.data_as(ct.POINTER(ct.c_uint32))))
        return out


def _points_ptr(points, n):
    """Device pointer of an int32 CUDA tensor of n point indices, or None."""
    if points is None:
        return None
    import torch
    assert points.is_cuda and points.dtype == torch.int32 and points.numel() == n and points.is_contiguous()
    return ct.c_void_p(points.data_ptr())


class ARNet:
    """Handle on the learned autoregressive proposal (crbm_ar_*).  With
    cond_points > 0 the network is conditional: set_points() gives each point
    a feature vector of 3 numbers, and the calls take `points`, an int32
    CUDA tensor with one point index per configuration (None = point 0)."""

    def __init__(self, L: int, seed: int = 0, stream=None, cond_points: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the network runs only on the HIP device")
        self.L = L
        self.cond_points = cond_points
        cfg = _ARConfig(L, 32, 12, seed, _stream_handle(stream), cond_points)
        h = ct.c_void_p()
        _check(lib().crbm_ar_create(ct.byref(cfg), ct.byref(h)))
        self._h = h
        self.num_params = int(lib().crbm_ar_num_params(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.crbm_ar_destroy(h)
            self._h = None

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, np.float32)
        assert a.size == self.num_params
        _check(lib().crbm_ar_set_params(self._h, a.ctypes.data_as(ct.POINTER(ct.c_float)), a.size))

    def init_params(self, seed: int, scale: float = 0.5):
        """Seeded fan-in-scaled normal weights, zero biases (library-side)."""
        _check(lib().crbm_ar_init_params(self._h, int(seed), float(scale)))

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.num_params, np.float32)
        _check(lib().crbm_ar_get_params(self._h, a.ctypes.data_as(ct.POINTER(ct.c_float)), a.size))
        return a

    def set_points(self, feats):
        """Feature vectors of the points, [n_points, 3] (conditional network)."""
        f = np.ascontiguousarray(feats, np.float64)
        assert f.ndim == 2 and f.shape[1] == 3
        _check(lib().crbm_ar_set_points(self._h, f.shape[0], f.ctypes.data_as(ct.POINTER(ct.c_double))))

    def grad(self, samples, points=None):
        assert samples.is_cuda and samples.dtype.itemsize == 1
        g = np.zeros(self.num_params, np.float32)
        loss = ct.c_double()
        _check(lib().crbm_ar_grad_cond(self._h, ct.c_void_p(samples.data_ptr()), _points_ptr(points, samples.shape[0]),
                                       samples.shape[0], g.ctypes.data_as(ct.POINTER(ct.c_float)), ct.byref(loss)))
        return g, float(loss.value)

    def train_step(self, samples, lr: float, points=None) -> float:
        loss = ct.c_double()
        _check(lib().crbm_ar_train_step_cond(self._h, ct.c_void_p(samples.data_ptr()),
                                             _points_ptr(points, samples.shape[0]), samples.shape[0], lr,
                                             ct.byref(loss)))
        return float(loss.value)

    def train(self, data, steps: int, batch: int = 1024, lr: float = 1e-3, lr_late: float = 3e-4,
              late_from: float = 0.625, seed: int = 1, step0: int = 0, augment: bool = True, points=None) -> float:
        """A training run in the library (crbm_ar_train): `steps` Adam steps on
        minibatches drawn on the device from data (int8 CUDA [n, L, L]; points:
        int32 CUDA [n] for a conditional network), with random lattice
        symmetries.  Returns the last step's mean loss per configuration."""
        assert data.is_cuda and data.dtype.itemsize == 1 and data.is_contiguous()
        n = int(data.shape[0])
        o = _TrainOpts(int(steps), int(batch), float(lr), float(lr_late), float(late_from), int(seed), int(step0),
                       1 if augment else 0)
        loss = ct.c_double()
        _check(lib().crbm_ar_train(self._h, ct.c_void_p(data.data_ptr()), _points_ptr(points, n), n, ct.byref(o),
                                   ct.byref(loss)))
        return float(loss.value)

    def logq(self, spins, points=None):
        import torch
        out = torch.empty(spins.shape[0], dtype=torch.float64, device="cuda")
        _check(lib().crbm_ar_logq_cond(self._h, ct.c_void_p(spins.data_ptr()), _points_ptr(points, spins.shape[0]),
                                       spins.shape[0], ct.c_void_p(out.data_ptr())))
        return out

    def sample(self, n: int, seed: int, step: int = 0, id: int = 0, points=None):
        import torch
        spins = torch.empty((n, self.L, self.L), dtype=torch.int8, device="cuda")
        lq = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(lib().crbm_ar_sample_cond(self._h, n, seed, step, id, _points_ptr(points, n),
                                         ct.c_void_p(spins.data_ptr()), ct.c_void_p(lq.data_ptr())))
        return spins, lq

    def sample_steps(self, n: int, n_steps: int, seed: int, step0: int = 0, id: int = 0, points=None):
        """n_steps batches of n proposals in one launch; batch k equals
        sample(n, seed, step0 + k, id, points).  Returns spins [n_steps, n, L, L]
        and log q [n_steps, n]."""
        import torch
        if n < 1 or n_steps < 1:  # the library's own argument error
            _check(lib().crbm_ar_sample_steps(self._h, n, n_steps, seed, step0, id, None, None, None))
        spins = torch.empty((n_steps, n, self.L, self.L), dtype=torch.int8, device="cuda")
        lq = torch.empty((n_steps, n), dtype=torch.float64, device="cuda")
        _check(lib().crbm_ar_sample_steps(self._h, n, n_steps, seed, step0, id, _points_ptr(points, n),
                                          ct.c_void_p(spins.data_ptr()), ct.c_void_p(lq.data_ptr())))
        return spins, lq


def train_batch(data, batch: int, seed: int, step: int, augment: bool = True, points=None, stream=None):
    """The minibatch crbm_ar_train draws at `step` (crbm_ar_batch): returns
    (configurations int8 [batch, L, L], their points int32 [batch], the
    indices of the drawn training configurations int64 [batch])."""
    import torch
    assert data.is_cuda and data.dtype.itemsize == 1 and data.is_contiguous() and data.dim() == 3
    n, L = int(data.shape[0]), int(data.shape[1])
    out = torch.empty((batch, L, L), dtype=torch.int8, device="cuda")
    pts = torch.empty(batch, dtype=torch.int32, device="cuda")
    idx = torch.empty(batch, dtype=torch.int64, device="cuda")
    _check(lib().crbm_ar_batch(ct.c_void_p(data.data_ptr()), _points_ptr(points, n), n, L, batch, seed, step,
                               1 if augment else 0, ct.c_void_p(out.data_ptr()), ct.c_void_p(pts.data_ptr()),
                               ct.c_void_p(idx.data_ptr()), _stream_handle(stream)))
    return out, pts, idx


def sample_mh(sampler: Sampler, net: ARNet, n_cycles: int, gibbs_per_mh: int, trace=None, order=None) -> int:
    """n_cycles of gibbs_per_mh Gibbs sweeps then one independent-MH step with
    the network's proposals.  trace / order: int32 CUDA tensors [n_cycles,
    chains, 3] for the counts and the plateau structure factor after each
    cycle.  Returns the number of accepted moves."""
    acc = ct.c_int64()
    _check(lib().crbm_sample_mh(sampler._h, net._h, n_cycles, gibbs_per_mh,
                                ct.c_void_p(trace.data_ptr()) if trace is not None else None,
                                ct.c_void_p(order.data_ptr()) if order is not None else None, ct.byref(acc)))
    return int(acc.value)


# ------------------------------------------------------------- general lattices

def debug_fail_alloc(n: int):
    """Make the library's n-th device allocation from now on fail (n < 0: disarm);
    for tests of the error paths."""
    _check(lib().crbm_debug_fail_alloc(int(n)))


def debug_tail_cap(cap: int):
    """Lanes per round of the Gibbs samplers' compacted hidden tail (64; a
    smaller cap forces several rounds, for tests; trajectories do not change)."""
    _check(lib().crbm_debug_tail_cap(int(cap)))


def ss_filters(J1: float, J2: float):
    """Per-filter couplings of the Shastry-Sutherland lattice: filters k0-k7
    are square edges (J1), k8 and k9 the dimers (J2)."""
    return [float(J1)] * 8 + [float(J2)] * 2


@dataclass
class Lattice:
    """One general lattice for crbm_lattice_create: rows x cols, each axis open
    or periodic, one coupling per filter, fields on even / odd columns."""
    rows: int
    cols: int
    J: Sequence[float]
    h_even: float = 0.0
    h_odd: Optional[float] = None
    open_rows: bool = False
    open_cols: bool = False
    n_chains: int = 64
    sched: str = "const"
    T0: float = 1.0
    T1: Optional[float] = None
    T_explicit: Optional[np.ndarray] = None
    id: int = 0

    def c(self, keep):
        te = None
        if self.sched == "explicit":
            t = np.ascontiguousarray(self.T_explicit, np.float64)
            keep.append(t)
            te = t.ctypes.data_as(ct.POINTER(ct.c_double))
        J = [float(x) for x in self.J]
        assert len(J) == 10
        return _Lattice(self.rows, self.cols, int(self.open_rows), int(self.open_cols), (ct.c_double * 10)(*J),
                        float(self.h_even), float(self.h_even if self.h_odd is None else self.h_odd), self.n_chains,
                        SCHED[self.sched], self.T0, self.T0 if self.T1 is None else self.T1, te, self.id)


def lattice_table(lat: Lattice, T: float) -> np.ndarray:
    """The device table of one sweep at temperature T (host only)."""
    out = np.zeros(LAT_TAB_WORDS, np.uint32)
    keep = []
    c = lat.c(keep)
    _check(lib().crbm_lattice_table(ct.byref(c), float(T), out.ctypes.data_as(ct.POINTER(ct.c_uint32))))
    return out


class LatticeSampler:
    """Handle on crbm_lattice_create / crbm_lattice_sample / crbm_lattice_observables."""

    def __init__(self, lattices: Sequence[Lattice], seed: int, n_sweeps: int, measure_every: int = 0,
                 burn_in: int = 0, stream=None, corr: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the CRBM sampler runs only on the HIP device")
        self.lattices = list(lattices)
        self._keep = []
        arr = (_Lattice * len(self.lattices))()
        for k, I in enumerate(self.lattices):
            arr[k] = I.c(self._keep)
        cfg = _Config(seed, n_sweeps, measure_every, burn_in, _stream_handle(stream), 0, 0, 0, 0,
                      CRBM_F_CORR if corr else 0)
        h = ct.c_void_p()
        _check(lib().crbm_lattice_create(arr, len(self.lattices), ct.byref(cfg), ct.byref(h)))
        self._h = h
        self.corr = corr
        self.n_sweeps = n_sweeps
        self.total_chains = int(lib().crbm_lattice_total_chains(h))
        self.spin_offsets = np.cumsum([0] + [I.n_chains * I.rows * I.cols for I in self.lattices])
        self.chain_offsets = np.cumsum([0] + [I.n_chains for I in self.lattices])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.crbm_lattice_destroy(h)
            self._h = None

    def close(self):
        self.__del__()

    @property
    def total_spins(self) -> int:
        return int(self.spin_offsets[-1])

    def sample(self, n_sweeps: int, spins_out=None, trace=None, trace_every: int = 1):
        """Enqueue n_sweeps sweeps.  spins_out: int8 CUDA tensor of total_spins
        elements; trace: int32 CUDA tensor [n_sweeps // trace_every, total_chains, 12]
        of (M_even, M_odd, B_0..B_9) after every trace_every-th sweep."""
        if spins_out is not None:
            assert spins_out.is_cuda and spins_out.dtype.itemsize == 1 and spins_out.numel() == self.total_spins
        if trace is not None:
            assert trace.is_cuda and trace.element_size() == 4
            assert trace.numel() == (n_sweeps // trace_every) * self.total_chains * 12
        _check(lib().crbm_lattice_sample(self._h, n_sweeps,
                                         ct.c_void_p(spins_out.data_ptr()) if spins_out is not None else None,
                                         ct.c_void_p(trace.data_ptr()) if trace is not None else None,
                                         int(trace_every)))

    def observables(self):
        """Per-lattice int64 accumulator sums [n, 18] and, for a sampler created
        with corr=True, the per-lattice [rows, 2 cols - 1] displacement
        correlation sums (else None)."""
        acc = np.zeros((len(self.lattices), LAT_N_ACC), np.int64)
        cbuf = None
        if self.corr:
            cbuf = np.zeros(sum(I.rows * (2 * I.cols - 1) for I in self.lattices), np.int64)
        _check(lib().crbm_lattice_observables(self._h, acc.ctypes.data_as(ct.POINTER(ct.c_int64)),
                                              cbuf.ctypes.data_as(ct.c_void_p) if cbuf is not None else None))
        if cbuf is None:
            return acc, None
        parts, off = [], 0
        for I in self.lattices:
            n = I.rows * (2 * I.cols - 1)
            parts.append(cbuf[off:off + n].reshape(I.rows, 2 * I.cols - 1))
            off += n
        return acc, parts

    def reset_observables(self):
        _check(lib().crbm_lattice_reset_observables(self._h))

    def get_state(self):
        import torch
        spins = torch.empty(self.total_spins, dtype=torch.int8, device="cuda")
        idx = ct.c_int64()
        _check(lib().crbm_lattice_get_state(self._h, ct.c_void_p(spins.data_ptr()), ct.byref(idx)))
        return spins, int(idx.value)

    def set_state(self, spins, sweep_index: int):
        assert spins is None or (spins.is_cuda and spins.numel() == self.total_spins)
        _check(lib().crbm_lattice_set_state(self._h, ct.c_void_p(spins.data_ptr()) if spins is not None else None,
                                            int(sweep_index)))

    def split_spins(self, flat):
        """Split a flat [total_spins] tensor into per-lattice [n_chains, rows, cols] views."""
        out = []
        for k, I in enumerate(self.lattices):
            a, b = int(self.spin_offsets[k]), int(self.spin_offsets[k + 1])
            out.append(flat[a:b].view(I.n_chains, I.rows, I.cols))
        return out
