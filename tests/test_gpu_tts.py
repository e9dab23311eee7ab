"""GPU: per-chain minimum energy and first-hit sweep (crbm_min_energy) against
the oracle's definition over the oracle's own trajectories, bit for bit; and
the ground states of the four phase points of Sec. III.C reached by the
time-to-solution runs, never undercut."""
import numpy as np
import pytest

import oracle
from oracle import tts as OT

torch = pytest.importorskip("torch")
crbm = pytest.importorskip("paper_2511_20911_amd")
from paper_2511_20911_amd import tts as PT  # noqa: E402

pytestmark = pytest.mark.gpu


def _weights(J1, J2, h):
    return (-oracle.quantise(h), oracle.quantise(J1), oracle.quantise(J2))


def _oracle_traces(I, S, seed, chains):
    oi = oracle.Instance(I.L, I.J1, I.J2, I.h, I.sched, I.T0, I.T1, id=I.id)
    return np.stack([oracle.run_chain(oi, S, seed, c, 0, S, trace=True)[1] for c in range(chains)], axis=1)


@pytest.mark.parametrize("L,chains", [(6, 48), (12, 24)])
def test_min_energy_matches_oracle_in_chunks(L, chains):
    """Two sample calls (100 + 140 sweeps) folded into one running minimum
    equal the oracle's minimum and first hit over its whole 240-sweep trace."""
    S, seed = 240, 0x77
    I = crbm.Instance(L=L, J1=1.0, J2=1.0, h=0.0, n_chains=chains, sched="geometric", T0=3.0, T1=0.1, id=5)
    print(f"case L={L} chains={chains} seed={seed}", flush=True)
    smp = crbm.Sampler([I], seed=seed, n_sweeps=S)
    w = _weights(1.0, 1.0, 0.0)
    emin = first = None
    for s0, n in ((0, 100), (100, 140)):
        tr = torch.empty((n, chains, 3), dtype=torch.int32, device="cuda")
        smp.sample(n, trace=tr)
        emin, first = crbm.min_energy(tr, w, sweep0=s0, emin=emin, first=first)
    torch.cuda.synchronize()
    otr = _oracle_traces(I, S, seed, chains)
    oe, of = OT.min_energy(otr, w)
    assert np.array_equal(emin.cpu().numpy(), oe)
    assert np.array_equal(first.cpu().numpy(), of)


@pytest.mark.parametrize("every", [3, 8])
def test_min_energy_of_thinned_trace(every):
    """A thinned trace (every k-th sweep) gives the oracle's minimum over the
    same recorded sweeps, with first hits counted in completed sweeps."""
    L, chains, S, seed = 6, 40, 240, 0x99
    I = crbm.Instance(L=L, J1=1.0, J2=2.5, h=0.0, n_chains=chains, sched="const", T0=0.6, T1=0.6, id=11)
    print(f"case every={every} seed={seed}", flush=True)
    smp = crbm.Sampler([I], seed=seed, n_sweeps=S)
    tr = torch.empty((S // every, chains, 3), dtype=torch.int32, device="cuda")
    smp.sample(S, trace=tr, trace_every=every)
    w = _weights(1.0, 2.5, 0.0)
    emin, first = crbm.min_energy(tr, w, sweep0=0, trace_every=every)
    torch.cuda.synchronize()
    otr = _oracle_traces(I, S, seed, chains)[every - 1::every]
    oe, of = OT.min_energy(otr, w, 0, every)
    assert np.array_equal(emin.cpu().numpy(), oe)
    assert np.array_equal(first.cpu().numpy(), of)


def test_min_energy_chain_range_and_reset():
    """Chains [c0, c1) of a trace give the same values as the full fold; a
    zero-sample fold leaves the minima untouched; reset ignores stale contents."""
    L, chains, S, seed = 12, 64, 150, 0x31
    I = crbm.Instance(L=L, J1=1.0, J2=0.5, h=4.0, n_chains=chains, sched="geometric", T0=3.0, T1=0.2, id=3)
    smp = crbm.Sampler([I], seed=seed, n_sweeps=S)
    tr = torch.empty((S, chains, 3), dtype=torch.int32, device="cuda")
    smp.sample(S, trace=tr)
    w = _weights(1.0, 0.5, 4.0)
    e_all, f_all = crbm.min_energy(tr, w)
    e_sub, f_sub = crbm.min_energy(tr, w, c0=17, c1=50)
    assert torch.equal(e_sub, e_all[17:50]) and torch.equal(f_sub, f_all[17:50])
    e2, f2 = crbm.min_energy(tr[:0], w, sweep0=S, emin=e_all.clone(), first=f_all.clone())
    assert torch.equal(e2, e_all) and torch.equal(f2, f_all)
    stale_e = torch.full_like(e_all, -(1 << 60))
    stale_f = torch.full_like(f_all, 7)
    # the Python binding resets when no running minima are passed; pass stale
    # arrays through the C entry point with reset = 1
    import ctypes as ct
    wv = (ct.c_int64 * 3)(*w)
    rc = crbm.lib().crbm_min_energy(ct.c_void_p(tr.data_ptr()), S, chains, 0, chains, wv, 0, 1, 1,
                                    ct.c_void_p(stale_e.data_ptr()), ct.c_void_p(stale_f.data_ptr()),
                                    ct.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    assert torch.equal(stale_e, e_all) and torch.equal(stale_f, f_all)


@pytest.mark.parametrize("L", [6, 12])
def test_tts_runs_reach_the_phase_ground_states(L):
    """Constant-T runs at the four Sec. III.C phase points never go below the
    oracle's ground-state energy and reach it (at 12x12 the ordered Neel and
    1/3 phases may need longer runs: there only the bound is asserted), and
    the package's TTS statistics follow Eq. (14) from the runs' minima."""
    for pt, T in (((1.0, 7.0), 0.5), ((2.5, 0.0), 0.5), ((1.0, 0.0), 0.6), ((0.5, 4.0), 0.5)):
        J2, h = pt
        print(f"case L={L} J2={J2} h={h} T={T}", flush=True)
        ph, _ = OT.ground_state(1.0, J2, h)
        egs = OT.ground_energy_q(L, oracle.quantise(1.0), oracle.quantise(J2), oracle.quantise(h), ph)
        emin, first, sec = PT.runs(L, 1.0, J2, h, T, n_chains=512, n_sweeps=3000, seed=21, id=40, chunk=1000)
        assert (emin >= egs).all(), (pt, L)
        hit = emin == egs
        if L == 6 or ph in ("fm", "dimer"):
            assert hit.any(), (pt, L, emin.min() - egs)
        r = PT.tts_from_runs(emin, first, egs)
        assert r["p_gnd"] == hit.mean()
        if hit.any():
            assert (first[hit] >= 1).all() and (first[hit] <= 3000).all()
            assert abs(r["tts_sweeps"] - OT.tts(hit.mean(), first[hit].mean())) <= 1e-9 * r["tts_sweeps"]
        assert sec > 0.0
