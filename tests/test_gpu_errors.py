"""Error paths of the library under injected device-allocation failures
(crbm_debug_fail_alloc): every allocation of every entry point that
allocates is made to fail in turn; the call must return CRBM_ENOMEM with a
message and leave nothing behind, and the same call must then succeed and
give the same results as a handle that never saw a failure."""
import numpy as np
import pytest

import oracle
from oracle import ar

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
crbm = pytest.importorskip("paper_2511_20911_amd")

ENOMEM = -3
MAX_ALLOCS = 40  # more than any entry point makes


def _each_failure(make):
    """Call make() with the k-th allocation failing, k = 0, 1, ... until a
    call succeeds; return that call's result and the number of failures seen."""
    fails = 0
    for k in range(MAX_ALLOCS):
        crbm.debug_fail_alloc(k)
        try:
            out = make()
        except crbm.CrbmError as e:
            assert e.code == ENOMEM, (k, e.code, str(e))
            assert "crbm error -3" in str(e) and len(str(e)) > len("crbm error -3: ")
            fails += 1
            continue
        finally:
            crbm.debug_fail_alloc(-1)
        return out, fails
    raise AssertionError("no call succeeded")


def test_sampler_create_and_observables_survive_allocation_failures():
    insts = [crbm.Instance(L=6, J1=1.0, J2=0.5, h=0.0, n_chains=40, sched="linear", T0=3.0, T1=0.1, id=3),
             crbm.Instance(L=36, J1=1.0, J2=1.0, h=2.0, n_chains=9, sched="const", T0=0.8, id=4)]
    S, seed = 60, 0x5EED00000000E001
    smp, fails = _each_failure(lambda: crbm.Sampler(insts, seed=seed, n_sweeps=S, measure_every=1, launch="graph",
                                                    corr=True))
    assert fails >= 5  # state, tables, accumulators, items, correlation sums, queue
    spins = torch.empty(smp.total_spins, dtype=torch.int8, device="cuda")
    smp.sample(S, spins_out=spins)
    torch.cuda.synchronize()
    got = smp.split_spins(spins)[0].cpu().numpy()
    oi = oracle.Instance(6, 1.0, 0.5, 0.0, "linear", 3.0, 0.1, id=3)
    for ch in (0, 39):
        s, _, _ = oracle.run_chain(oi, S, seed, ch, 0, S)
        assert np.array_equal(got[ch], s)
    # the snapshot correlation of a handle without CRBM_F_CORR allocates on the fly
    plain = crbm.Sampler(insts, seed=seed, n_sweeps=S)
    plain.sample(10)
    (obs, corr), fails = _each_failure(lambda: plain.observables(corr=True))
    assert fails == 1 and corr[0][0, 0] == 40 * 36


def test_lattice_create_survives_allocation_failures():
    lats = [crbm.Lattice(rows=12, cols=8, J=crbm.ss_filters(1.0, 1.5), h_even=4.5, open_cols=True, n_chains=70,
                         T0=0.9, id=5),
            crbm.Lattice(rows=6, cols=40, J=crbm.ss_filters(1.0, 0.5), open_rows=True, n_chains=3, T0=1.2, id=6)]
    S, seed = 40, 0x5EED00000000E002
    smp, fails = _each_failure(lambda: crbm.LatticeSampler(lats, seed=seed, n_sweeps=S, measure_every=1, corr=True))
    assert fails >= 6  # state, tables, accumulators, correlation sums, items of both widths
    spins = torch.empty(smp.total_spins, dtype=torch.int8, device="cuda")
    smp.sample(S, spins_out=spins)
    torch.cuda.synchronize()
    got = smp.split_spins(spins)[0].cpu().numpy()
    ol = oracle.Lattice(12, 8, oracle.ss_filters(1.0, 1.5), 4.5, 4.5, open_c=True, T0=0.9, id=5)
    s, _, _ = oracle.run_lattice_chain(ol, S, seed, 69, 0, S)
    assert np.array_equal(got[69], s)


def test_learned_proposal_survives_allocation_failures():
    """Creation (conditional network), the training buffers, the sampler and
    scorer buffers, training runs and the MH buffers: each fails once at every
    allocation, then gives exactly what an undisturbed network gives."""
    L = 6
    params = ar.init_params(seed=7, scale=0.5)
    flat = np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)
    rng = np.random.default_rng(1)
    data = torch.from_numpy((2 * rng.integers(0, 2, (300, L, L)) - 1).astype(np.int8)).cuda()

    ref = crbm.ARNet(L)
    ref.set_params(flat)
    g_ref, loss_ref = ref.grad(data[:64].contiguous())
    p_ref, lq_ref = ref.sample(48, seed=9, step=2, id=1)
    s_ref = ref.logq(p_ref)

    net, fails = _each_failure(lambda: crbm.ARNet(L, cond_points=2))
    assert fails >= 8
    net = crbm.ARNet(L)
    net.set_params(flat)
    (g, loss), fails = _each_failure(lambda: net.grad(data[:64].contiguous()))
    assert fails >= 10 and np.array_equal(g, g_ref) and loss == loss_ref
    (p, lq), fails = _each_failure(lambda: net.sample(48, seed=9, step=2, id=1))
    assert fails >= 2 and torch.equal(p, p_ref) and torch.equal(lq, lq_ref)
    s, fails = _each_failure(lambda: net.logq(p))
    assert torch.equal(s, s_ref)
    # a whole training run: its minibatch buffers fail, then the run matches an undisturbed one
    a = crbm.ARNet(L)
    a.set_params(flat)
    b = crbm.ARNet(L)
    b.set_params(flat)
    la = a.train(data, 5, batch=32, seed=3)
    lb, fails = _each_failure(lambda: b.train(data, 5, batch=32, seed=3))
    assert fails >= 2 and la == lb and np.array_equal(a.get_params(), b.get_params())
    # MH buffers
    def mh(net_):
        smp = crbm.Sampler([crbm.Instance(L=L, J1=1.0, J2=1.0, h=3.0, n_chains=50, sched="const", T0=1.0, id=2)],
                           seed=11, n_sweeps=40)
        acc = crbm.sample_mh(smp, net_, 3, 2)
        st, _ = smp.get_state()
        return acc, st
    acc_ref, st_ref = mh(ref)
    (acc, st), fails = _each_failure(lambda: mh(net))
    assert fails >= 3 and acc == acc_ref and torch.equal(st, st_ref)


def test_tau_int_survives_allocation_failures():
    rng = np.random.default_rng(2)
    tr = torch.from_numpy(rng.integers(-50, 50, (400, 16, 3)).astype(np.int32)).cuda()
    ref = crbm.tau_int(tr, (1, 0, 0), max_lag=100)
    got, fails = _each_failure(lambda: crbm.tau_int(tr, (1, 0, 0), max_lag=100))
    assert fails == 3
    for a, b in zip(got, ref):
        assert np.array_equal(np.asarray(a), np.asarray(b))
