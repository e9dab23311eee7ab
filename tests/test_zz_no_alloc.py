"""The allocation-free entry point crbm_tau_int_noalloc (for callers that
cannot allocate device memory) against crbm_tau_int on the same traces: two
calls in a row, the second smaller, through the C ABI; results bit-identical
(same kernels, same summation order); requests beyond the scratch bound are
refused before any work is enqueued."""
import ctypes as ct

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
crbm = pytest.importorskip("paper_2511_20911_amd")


def _call(fn, trace, w, c0, c1, discard, max_lag):
    n, nch = int(trace.shape[0]), int(trace.shape[1])
    K = min(max_lag, n - discard - 1)
    rho = np.zeros(K + 1, np.float64)
    tau, ess, win = ct.c_double(), ct.c_double(), ct.c_int32()
    wv = (ct.c_double * 3)(*w)
    rc = fn(ct.c_void_p(trace.data_ptr()), n, nch, c0, c1, discard, wv, max_lag, 6.0, None, ct.byref(tau),
            ct.byref(ess), ct.byref(win), rho.ctypes.data_as(ct.POINTER(ct.c_double)))
    return rc, tau.value, ess.value, win.value, rho


def _trace(L, J2, h, T, chains, sweeps, seed, ident):
    inst = crbm.Instance(L=L, J1=1.0, J2=J2, h=h, n_chains=chains, sched="const", T0=T, id=ident)
    smp = crbm.Sampler([inst], seed=seed, n_sweeps=sweeps)
    tr = torch.empty((sweeps, chains, 3), dtype=torch.int32, device="cuda")
    smp.sample(sweeps, trace=tr)
    torch.cuda.synchronize()
    return tr


def test_noalloc_tau_int_equals_the_allocating_one():
    lib = crbm.lib()
    cases = [
        # (L, J2, h, T, chains, sweeps, c0, c1, discard, max_lag): the second is smaller
        (12, 1.0, 3.0, 0.8, 2048, 600, 0, 2048, 100, 400),
        (6, 0.5, 0.0, 1.5, 300, 200, 17, 250, 20, 60),
    ]
    for k, (L, J2, h, T, chains, sweeps, c0, c1, discard, max_lag) in enumerate(cases):
        print(f"case {k}: L={L} chains={chains} sweeps={sweeps}", flush=True)
        tr = _trace(L, J2, h, T, chains, sweeps, 40 + k, 7 + k)
        Jq = [int(round(x * 65536)) for x in (1.0, J2, h)]
        for w in ((-Jq[2], Jq[0], Jq[1]), (1.0, 0.0, 0.0)):
            w = tuple(float(x) for x in w)
            ref = _call(lib.crbm_tau_int, tr, w, c0, c1, discard, max_lag)
            got = _call(lib.crbm_tau_int_noalloc, tr, w, c0, c1, discard, max_lag)
            assert ref[0] == 0 and got[0] == 0, lib.crbm_last_error().decode()
            assert got[1] == ref[1] and got[2] == ref[2] and got[3] == ref[3], (got[1:4], ref[1:4])
            assert np.array_equal(got[4], ref[4])
            assert ref[1] >= 1.0 or ref[1] > 0.0


def test_noalloc_tau_int_refuses_oversized_requests():
    lib = crbm.lib()
    tr = torch.zeros((8, 4, 3), dtype=torch.int32, device="cuda")
    # a trace header claiming more chains x samples than the scratch holds (the pointer is never read)
    n, nch = 1 << 20, 16
    wv = (ct.c_double * 3)(1.0, 0.0, 0.0)
    tau = ct.c_double()
    rc = lib.crbm_tau_int_noalloc(ct.c_void_p(tr.data_ptr()), n, nch, 0, nch, 0, wv, 10, 6.0, None, ct.byref(tau),
                                  None, None, None)
    assert rc == crbm.CRBM_ERANGE and "scratch" in lib.crbm_last_error().decode()
    rc = lib.crbm_tau_int_noalloc(ct.c_void_p(tr.data_ptr()), 8, 4, 0, 4, 0, wv, 0, 6.0, None, ct.byref(tau),
                                  None, None, None)
    assert rc == crbm.CRBM_EINVAL
    # the lag bound
    tr2 = torch.zeros((6000, 2, 3), dtype=torch.int32, device="cuda")
    rc = lib.crbm_tau_int_noalloc(ct.c_void_p(tr2.data_ptr()), 6000, 2, 0, 2, 0, wv, 5000, 6.0, None,
                                  ct.byref(tau), None, None, None)
    assert rc == crbm.CRBM_ERANGE
    # a good call still works afterwards
    rc = lib.crbm_tau_int_noalloc(ct.c_void_p(tr2.data_ptr()), 6000, 2, 0, 2, 0, wv, 100, 6.0, None,
                                  ct.byref(tau), None, None, None)
    assert rc == 0 and tau.value == 1.0
