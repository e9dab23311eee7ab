"""GPU parity: the HIP sampler equals the CPU oracle bit for bit, trajectory by
trajectory, from the same seed (spins and exact int64 counts), through the C ABI.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
crbm = pytest.importorskip("paper_2511_20911_amd")


def _oi(I: "crbm.Instance"):
    return oracle.Instance(I.L, I.J1, I.J2, I.h, I.sched, I.T0, I.T1, I.T_explicit, id=I.id)


def _run_gpu(insts, seed, S, n_run=None, trace=True, tile_rows=0, measure_every=0, burn_in=0):
    n_run = S if n_run is None else n_run
    smp = crbm.Sampler(insts, seed=seed, n_sweeps=S, measure_every=measure_every, burn_in=burn_in,
                       tile_rows=tile_rows)
    spins = torch.empty(smp.total_spins, dtype=torch.int8, device="cuda")
    tr = torch.empty((n_run, smp.total_chains, 3), dtype=torch.int32, device="cuda") if trace else None
    smp.sample(n_run, spins_out=spins, trace=tr)
    torch.cuda.synchronize()
    parts = [p.cpu().numpy() for p in smp.split_spins(spins)]
    return smp, parts, (tr.cpu().numpy() if trace else None)


def _check_chains(I, parts_k, trace, chain_off, seed, S, chains, n_run=None):
    n_run = S if n_run is None else n_run
    oi = _oi(I)
    for ch in chains:
        s, t, _ = oracle.run_chain(oi, S, seed, ch, 0, n_run, trace=trace is not None)
        assert np.array_equal(parts_k[ch], s), f"L={I.L} chain {ch}: spins differ"
        if trace is not None:
            assert np.array_equal(trace[:, chain_off + ch, :], t), f"L={I.L} chain {ch}: trace differs"


def test_config1_all_chains_bit_exact():
    """6x6, J2/J1 = 0.5, h = 0, 256 chains, linear anneal 3.0 -> 0.1 over 2000
    sweeps: every chain's final spins and per-sweep (M, B1, B2) equal the oracle."""
    I = crbm.Instance(L=6, J1=1.0, J2=0.5, h=0.0, n_chains=256, sched="linear", T0=3.0, T1=0.1, id=0)
    seed = 0x5EED000000000001
    S = 2000
    smp, parts, tr = _run_gpu([I], seed, S)
    _check_chains(I, parts[0], tr, 0, seed, S, range(256))
    # every chain ends in the Neel state of this point (E/N = -1.75)
    M, B1, B2 = tr[-1, :, 0], tr[-1, :, 1], tr[-1, :, 2]
    E = (B1 + 0.5 * B2) / 36
    assert np.all(M == 0) and np.all(np.abs(E + 1.75) < 1e-12)


@pytest.mark.parametrize("tile_rows", [1, 3, 9])
def test_18x18_geometric_bit_exact_any_tiling(tile_rows):
    """18x18 (the paper's 324 spins), geometric anneal 5.0 -> 0.05 over 10^4
    sweeps at two (J2/J1, h) points: sampled chains equal the oracle for every
    lanes-per-chain tiling (G = 9, 3, 1)."""
    S = 10000
    seed = 0x5EED000000000002
    insts = [crbm.Instance(L=18, J1=1.0, J2=1.0, h=3.0, n_chains=32, sched="geometric", T0=5.0, T1=0.05, id=5),
             crbm.Instance(L=18, J1=1.0, J2=2.0, h=0.6, n_chains=21, sched="geometric", T0=5.0, T1=0.05, id=61)]
    n_run = 1500
    smp, parts, tr = _run_gpu(insts, seed, S, n_run=n_run, tile_rows=tile_rows)
    _check_chains(insts[0], parts[0], tr, 0, seed, S, [0, 7, 31], n_run)
    _check_chains(insts[1], parts[1], tr, 32, seed, S, [0, 20], n_run)


def test_18x18_full_schedule_sampled_chains():
    """Full 10^4-sweep schedule at 18x18, J2/J1 = 1, h = 3 (the plateau point):
    two sampled chains equal the oracle at the end."""
    S = 10000
    seed = 0x5EED000000000002
    I = crbm.Instance(L=18, J1=1.0, J2=1.0, h=3.0, n_chains=64, sched="geometric", T0=5.0, T1=0.05, id=9)
    smp, parts, _ = _run_gpu([I], seed, S, trace=False)
    _check_chains(I, parts[0], None, 0, seed, S, [0, 63])


def test_mixed_sizes_in_one_handle():
    """Instances of different L, couplings and schedules in one handle; ragged
    chain counts (not multiples of the chains per wavefront)."""
    seed = 77
    S = 300
    insts = [
        crbm.Instance(L=4, J1=1.0, J2=0.5, h=0.0, n_chains=5, sched="const", T0=1.0, id=1),
        crbm.Instance(L=6, J1=1.0, J2=2.5, h=0.0, n_chains=70, sched="linear", T0=3.0, T1=0.2, id=2),
        crbm.Instance(L=12, J1=1.0, J2=1.0, h=3.0, n_chains=33, sched="geometric", T0=5.0, T1=0.1, id=3),
        crbm.Instance(L=24, J1=1.0, J2=1.5, h=-1.0, n_chains=17, sched="const", T0=0.7, id=4),
        crbm.Instance(L=32, J1=-1.0, J2=0.0, h=0.25, n_chains=3, sched="const", T0=2.0, id=5),
        crbm.Instance(L=10, J1=1.0, J2=1.0, h=2.0, n_chains=9, sched="explicit",
                      T_explicit=np.linspace(4.0, 0.3, S), id=6),
    ]
    smp, parts, tr = _run_gpu(insts, seed, S)
    off = smp.chain_offsets
    for k, I in enumerate(insts):
        chains = sorted({0, I.n_chains // 2, I.n_chains - 1})
        _check_chains(I, parts[k], tr, int(off[k]), seed, S, chains)


@pytest.mark.parametrize("every", [1, 4, 25])
def test_thinned_trace_is_every_kth_row(every):
    """crbm_sample_thinned records (M, B1, B2) after sweeps k, 2k, ... of the
    call: exactly rows k-1, 2k-1, ... of the oracle's per-sweep trace, across
    two calls (the second starting mid-schedule); the spins are unchanged."""
    seed, S = 0x5EED000000000004, 200
    I = crbm.Instance(L=18, J1=1.0, J2=1.0, h=3.0, n_chains=40, sched="const", T0=0.4, id=9)
    smp = crbm.Sampler([I], seed=seed, n_sweeps=S)
    spins = torch.empty(smp.total_spins, dtype=torch.int8, device="cuda")
    tr1 = torch.empty((100 // every, 40, 3), dtype=torch.int32, device="cuda")
    tr2 = torch.empty((100 // every, 40, 3), dtype=torch.int32, device="cuda")
    smp.sample(100, trace=tr1, trace_every=every)
    smp.sample(100, spins_out=spins, trace=tr2, trace_every=every)
    torch.cuda.synchronize()
    got = np.concatenate([tr1.cpu().numpy(), tr2.cpu().numpy()])
    sp = spins.cpu().numpy().reshape(40, 18, 18)
    oi = _oi(I)
    for ch in (0, 17, 39):
        s, t, _ = oracle.run_chain(oi, S, seed, ch, 0, S, trace=True)
        assert np.array_equal(sp[ch], s)
        assert np.array_equal(got[:, ch, :], t[every - 1::every]), (every, ch)
    with pytest.raises(crbm.CrbmError) as e:
        smp2 = crbm.Sampler([I], seed=seed, n_sweeps=S)
        smp2.sample(10, trace=torch.empty((3, 40, 3), dtype=torch.int32, device="cuda"), trace_every=3)
    assert e.value.code == crbm.CRBM_EINVAL


@pytest.mark.parametrize("L,every,rows", [(18, 5, 1), (18, 5, 3), (18, 5, 9), (12, 1, 2), (8, 3, 4), (36, 4, 1),
                                          (36, 4, 3)])
def test_order_trace_matches_oracle(L, every, rows):
    """The plateau structure-factor trace (max, |S_A|^2, |S_B|^2) of
    crbm_sample_thinned equals the oracle's definition (cos/sin sums) on the
    oracle's own trajectory at every recorded sweep, for every lanes-per-chain
    tiling (the sums are reduced across the chain's lanes); L = 8 (not a
    multiple of 3) and 36 (two words per row) included."""
    seed, S = 0x5EED000000000007, 60
    I = crbm.Instance(L=L, J1=1.0, J2=1.0, h=3.0, n_chains=10, sched="linear", T0=2.0, T1=0.3, id=11)
    smp = crbm.Sampler([I], seed=seed, n_sweeps=S, tile_rows=rows)
    tr = torch.empty((S // every, 10, 3), dtype=torch.int32, device="cuda")
    od = torch.empty_like(tr)
    smp.sample(S, trace=tr, trace_every=every, order=od)
    torch.cuda.synchronize()
    got, tgot = od.cpu().numpy(), tr.cpu().numpy()
    oi = _oi(I)
    for ch in (0, 3, 9):
        sp = None
        for k in range(S // every):
            sp, t, _ = oracle.run_chain(oi, S, seed, ch, k * every, (k + 1) * every, spins=sp, trace=True)
            assert np.array_equal(tgot[k, ch], t[-1])
            assert tuple(got[k, ch]) == oracle.order(L, sp), (L, ch, k)


def test_batch_composition_invariance():
    """An instance gives the same chains alone or inside a batch (the random
    stream depends on the instance id, not on its position)."""
    seed = 99
    S = 200
    A = crbm.Instance(L=12, J1=1.0, J2=1.0, h=2.0, n_chains=40, sched="const", T0=0.8, id=17)
    B = crbm.Instance(L=18, J1=1.0, J2=0.5, h=0.0, n_chains=30, sched="const", T0=1.5, id=4)
    _, p1, _ = _run_gpu([A], seed, S, trace=False)
    _, p2, _ = _run_gpu([B, A], seed, S, trace=False)
    assert np.array_equal(p1[0], p2[1])


def test_resume_is_bit_exact():
    """get_state / set_state at any sweep: 2 x 150 sweeps == 300 sweeps."""
    seed = 5
    S = 300
    I = crbm.Instance(L=18, J1=1.0, J2=1.5, h=1.0, n_chains=50, sched="linear", T0=3.0, T1=0.3, id=2)
    _, full, _ = _run_gpu([I], seed, S, trace=False)
    smp = crbm.Sampler([I], seed=seed, n_sweeps=S)
    smp.sample(150)
    st, idx = smp.get_state()
    assert idx == 150
    smp2 = crbm.Sampler([I], seed=seed, n_sweeps=S)
    smp2.set_state(st, 150)
    out = torch.empty(smp2.total_spins, dtype=torch.int8, device="cuda")
    smp2.sample(150, spins_out=out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(50, 18, 18), full[0])
    with pytest.raises(crbm.CrbmError) as e:
        smp2.sample(1)
    assert e.value.code == crbm.CRBM_ESTATE


def test_accumulators_and_structure_factor_match_oracle():
    """Exact int64 sums of (M, B1, B2) and their second moments, and the summed
    correlation C(dr, dc) of the final state, equal the oracle's."""
    seed = 31
    S = 400
    I = crbm.Instance(L=12, J1=1.0, J2=1.0, h=3.0, n_chains=24, sched="const", T0=0.6, id=8)
    smp = crbm.Sampler([I], seed=seed, n_sweeps=S, measure_every=3, burn_in=100)
    smp.sample(S)
    obs, corr = smp.observables(corr=True)
    acc = np.zeros(oracle.N_ACC, np.int64)
    csum = np.zeros((12, 12), np.int64)
    oi = _oi(I)
    for ch in range(24):
        s, _, a = oracle.run_chain(oi, S, seed, ch, 0, S, measure_every=3, burn_in=100)
        acc += a
        csum += oracle.corr(12, s)
    assert [obs[0][k] for k in ACC_KEYS] == acc.tolist()
    assert np.array_equal(corr[0], csum)
    n = acc[0]
    E = (acc[2] + acc[3] - 3 * acc[1]) / n / 144
    assert abs(obs[0]["E_per_spin"] - E) < 1e-12
    assert abs(obs[0]["abs_stag_m"] - acc[13] / n / 144) < 1e-12


ACC_KEYS = ["n_samples", "sum_M", "sum_B1", "sum_B2", "sum_MM", "sum_B1B1", "sum_B2B2", "sum_MB1", "sum_MB2",
            "sum_B1B2", "sum_absM", "sum_Ms", "sum_MsMs", "sum_absMs"]


@pytest.mark.parametrize("launch", ["direct", "graph"])
def test_accumulated_structure_factor_matches_oracle(launch):
    """Sampler created with CRBM_F_CORR: C(dr, dc) summed over the chains and
    every measured sweep (Sec. III.B Eq. (13) averages it over the sampled
    states), for two lattice sizes in one handle (a one-word and a two-word
    row); every accumulator, the thinned counts trace written across the
    per-measured-sweep launches and the final states equal the oracle's; a
    reset zeroes the sums, which then restart."""
    seed, S, me, burn, te = 44, 90, 4, 13, 5
    insts = [crbm.Instance(L=12, J1=1.0, J2=1.0, h=2.0, n_chains=10, sched="geometric", T0=3.0, T1=0.5, id=3),
             crbm.Instance(L=36, J1=1.0, J2=1.5, h=1.0, n_chains=3, sched="const", T0=0.9, id=4)]
    smp = crbm.Sampler(insts, seed=seed, n_sweeps=S, measure_every=me, burn_in=burn, corr=True, launch=launch)
    n_tot = smp.total_chains
    tr = torch.zeros((60 // te, n_tot, 3), dtype=torch.int32, device="cuda")
    smp.sample(60, trace=tr, trace_every=te)
    obs, corr = smp.observables(corr=True)
    trn = tr.cpu().numpy()
    states = {}
    for k, I in enumerate(insts):
        acc = np.zeros(oracle.N_ACC, np.int64)
        csum = np.zeros(I.L * I.L, np.int64)
        for ch in range(I.n_chains):
            s, t, a = oracle.run_chain(_oi(I), S, seed, ch, 0, 60, trace=True, measure_every=me, burn_in=burn,
                                       corr=csum)
            acc += a
            states[(k, ch)] = s
            assert np.array_equal(trn[:, int(smp.chain_offsets[k]) + ch], t[te - 1::te]), (k, ch)
        assert [obs[k][key] for key in ACC_KEYS] == acc.tolist(), k
        assert np.array_equal(corr[k].reshape(-1), csum), k
        assert corr[k][0, 0] == I.L * I.L * acc[0]  # C(0, 0) = N per sample
    # the rest of the schedule after a reset: sums restart from zero
    smp.reset_observables()
    smp.sample(S - 60)
    obs2, corr2 = smp.observables(corr=True)
    for k, I in enumerate(insts):
        acc = np.zeros(oracle.N_ACC, np.int64)
        csum = np.zeros(I.L * I.L, np.int64)
        for ch in range(I.n_chains):
            oracle.run_chain(_oi(I), S, seed, ch, 60, S, spins=states[(k, ch)], measure_every=me, burn_in=burn,
                             acc=acc, corr=csum)
        assert [obs2[k][key] for key in ACC_KEYS] == acc.tolist(), k
        assert np.array_equal(corr2[k].reshape(-1), csum), k


def test_degenerate_couplings_bit_exact():
    """Edge cases of the mapping in one handle: zero J1 (no square bonds),
    zero J2, a pure field, ferromagnetic (negative) couplings, a temperature
    low enough to saturate every threshold, a very high one (near fair coins),
    and a single chain on the smallest lattice; every chain and trace equals
    the oracle."""
    seed, S = 0x5EED000000000006, 120
    insts = [
        crbm.Instance(L=6, J1=0.0, J2=1.0, h=0.5, n_chains=9, sched="const", T0=0.7, id=1),
        crbm.Instance(L=12, J1=1.0, J2=0.0, h=-1.0, n_chains=9, sched="linear", T0=2.0, T1=0.3, id=2),
        crbm.Instance(L=6, J1=0.0, J2=0.0, h=2.0, n_chains=9, sched="const", T0=1.5, id=3),
        crbm.Instance(L=18, J1=-1.0, J2=-0.5, h=0.0, n_chains=9, sched="geometric", T0=4.0, T1=0.5, id=4),
        crbm.Instance(L=12, J1=1.0, J2=1.0, h=3.0, n_chains=9, sched="const", T0=0.01, id=5),
        crbm.Instance(L=6, J1=1.0, J2=2.0, h=1.0, n_chains=9, sched="const", T0=1e4, id=6),
        crbm.Instance(L=4, J1=1.0, J2=0.5, h=0.2, n_chains=1, sched="const", T0=1.0, id=7),
    ]
    smp, parts, tr = _run_gpu(insts, seed, S)
    for k, I in enumerate(insts):
        _check_chains(I, parts[k], tr, int(smp.chain_offsets[k]), seed, S, range(I.n_chains))
    # zero sweeps is a no-op that still returns the state
    out = torch.empty(smp.total_spins, dtype=torch.int8, device="cuda")
    with pytest.raises(crbm.CrbmError):
        smp.sample(1)  # the schedule is exhausted
    smp2 = crbm.Sampler(insts, seed=seed, n_sweeps=S)
    smp2.sample(0, spins_out=out)
    st, idx = smp2.get_state()
    torch.cuda.synchronize()
    assert idx == 0 and torch.equal(out, st)


def test_every_compiled_tiling_bit_exact():
    """Every compiled (L, rows-per-lane) kernel variant -- whichever one the
    autotuner picks for a workload -- gives the oracle's trajectories: first
    and last chain of a ragged chain count, per-sweep counts and final spins."""
    seed, S = 0x5EED000000000008, 24
    tried = 0
    for L in crbm.SUPPORTED_L:
        for R in range(1, L // 2 + 1):
            if (L // 2) % R:
                continue
            I = crbm.Instance(L=L, J1=1.0, J2=1.25, h=1.5, n_chains=13, sched="linear", T0=3.0, T1=0.4,
                              id=(L * 7 + R) % 1000)
            try:
                smp, parts, tr = _run_gpu([I], seed, S, tile_rows=R)
            except crbm.CrbmError as e:
                assert e.code == crbm.CRBM_EUNSUPPORTED
                continue
            _check_chains(I, parts[0], tr, 0, seed, S, [0, 12])
            tried += 1
    assert tried >= 68, tried


def test_invalid_arguments_fail_cleanly():
    bad = [
        (crbm.Instance(L=7, n_chains=1), crbm.CRBM_EINVAL),
        (crbm.Instance(L=6, n_chains=0), crbm.CRBM_EINVAL),
        (crbm.Instance(L=6, n_chains=1, T0=-1.0), crbm.CRBM_EINVAL),
        (crbm.Instance(L=34, n_chains=1), crbm.CRBM_EUNSUPPORTED),
        (crbm.Instance(L=98, n_chains=1), crbm.CRBM_EUNSUPPORTED),
        (crbm.Instance(L=6, n_chains=1, periodic=0), crbm.CRBM_EUNSUPPORTED),
        (crbm.Instance(L=6, n_chains=1, T0=1e-7), crbm.CRBM_ERANGE),
    ]
    for I, code in bad:
        with pytest.raises(crbm.CrbmError) as e:
            crbm.Sampler([I], seed=1, n_sweeps=10)
        assert e.value.code == code, I


@pytest.mark.parametrize("tile_rows", [0, 1])
def test_multiword_lattices_bit_exact(tile_rows):
    """Rows wider than one 32-bit word (partial last word at L = 36, 40, 48, 72;
    full words at L = 64, 96): sampled chains equal the oracle."""
    seed = 0x5EED000000000005
    S = 40
    insts = [
        crbm.Instance(L=36, J1=1.0, J2=1.0, h=3.0, n_chains=11, sched="const", T0=0.9, id=21),
        crbm.Instance(L=40, J1=1.0, J2=2.5, h=0.5, n_chains=7, sched="linear", T0=3.0, T1=0.5, id=22),
        crbm.Instance(L=48, J1=1.0, J2=1.5, h=4.5, n_chains=9, sched="geometric", T0=5.0, T1=0.2, id=23),
        crbm.Instance(L=64, J1=1.0, J2=0.5, h=0.0, n_chains=3, sched="const", T0=1.2, id=24),
        crbm.Instance(L=72, J1=-1.0, J2=1.0, h=1.0, n_chains=5, sched="const", T0=2.0, id=25),
        crbm.Instance(L=96, J1=1.0, J2=1.0, h=2.0, n_chains=6, sched="linear", T0=4.0, T1=0.4, id=26),
    ]
    smp, parts, tr = _run_gpu(insts, seed, S, tile_rows=0 if tile_rows == 0 else 1)
    off = smp.chain_offsets
    for k, I in enumerate(insts):
        _check_chains(I, parts[k], tr, int(off[k]), seed, S, sorted({0, I.n_chains - 1}))


def test_multiword_observables_and_corr():
    seed = 3
    S = 30
    I = crbm.Instance(L=48, J1=1.0, J2=1.0, h=3.0, n_chains=4, sched="const", T0=0.7, id=31)
    smp = crbm.Sampler([I], seed=seed, n_sweeps=S, measure_every=2, burn_in=5)
    smp.sample(S)
    obs, corr = smp.observables(corr=True)
    acc = np.zeros(oracle.N_ACC, np.int64)
    csum = np.zeros((48, 48), np.int64)
    for ch in range(4):
        s, _, a = oracle.run_chain(_oi(I), S, seed, ch, 0, S, measure_every=2, burn_in=5)
        acc += a
        csum += oracle.corr(48, s)
    assert [obs[0][k] for k in ACC_KEYS] == acc.tolist()
    assert np.array_equal(corr[0], csum)


def _to_inst(p):
    return crbm.Instance(L=p.L, J1=p.J1, J2=p.J2, h=p.h, n_chains=p.n_chains, sched=p.sched, T0=p.T0, T1=p.T1,
                         id=p.id)


def test_graph_launch_equals_direct_and_replays():
    """One hipGraph launch (persistent kernels per lattice size) gives exactly
    the direct launches' result; replayed several times with eager work in
    between, every replay matches."""
    from paper_2511_20911_amd import workloads
    pts = workloads.batched_uneven(n_instances=24, chains=70)
    insts = [_to_inst(p) for p in pts]
    seed = 0x5EED000000000003
    S = 60
    d = crbm.Sampler(insts, seed=seed, n_sweeps=S, measure_every=1)
    g = crbm.Sampler(insts, seed=seed, n_sweeps=S, measure_every=1, launch="graph")
    for rep in range(4):
        n = 15
        sd = torch.empty(d.total_spins, dtype=torch.int8, device="cuda")
        sg = torch.empty(g.total_spins, dtype=torch.int8, device="cuda")
        td = torch.empty((n, d.total_chains, 3), dtype=torch.int32, device="cuda")
        tg = torch.empty((n, g.total_chains, 3), dtype=torch.int32, device="cuda")
        d.sample(n, spins_out=sd, trace=td)
        g.sample(n, spins_out=sg, trace=tg)
        torch.cuda.synchronize()
        _ = g.get_state()  # eager work between replays
        assert torch.equal(sd, sg), rep
        assert torch.equal(td, tg), rep
    assert d.observables() == g.observables()


def test_batched_uneven_full_size_graph():
    """The full uneven batch (2048 instances, L in {6..48}, 256 chains each,
    5000 sweeps at fixed T) in one graph launch; chains sampled from the small
    lattices equal the oracle."""
    from paper_2511_20911_amd import workloads
    pts = workloads.batched_uneven()
    insts = [_to_inst(p) for p in pts]
    seed = 0x5EED000000000003
    S = 5000
    smp = crbm.Sampler(insts, seed=seed, n_sweeps=S, launch="graph")
    out = torch.empty(smp.total_spins, dtype=torch.int8, device="cuda")
    smp.sample(S, spins_out=out)
    torch.cuda.synchronize()
    parts = smp.split_spins(out)
    picked = [k for k, p in enumerate(pts) if p.L <= 12][:3] + [k for k, p in enumerate(pts) if p.L == 18][:1]
    for k in picked:
        I = insts[k]
        for ch in (0, I.n_chains - 1):
            s, _, _ = oracle.run_chain(_oi(I), S, seed, ch, 0, S)
            assert np.array_equal(parts[k][ch].cpu().numpy(), s), (k, ch)


def test_autotune_picks_a_valid_tiling():
    r, w, rate = crbm.autotune(18, n_chains=1024, n_sweeps=20)
    assert 9 % r == 0 and 1 <= w <= 4 and rate > 0
    assert crbm.get_tiling(18) == (r, w)


@pytest.mark.parametrize("cap", [1, 5])
def test_compacted_tail_in_several_rounds_is_bit_exact(cap):
    """The hidden comparison finishes the words still tied after two random
    blocks on at most `cap` lanes per round (crbm_debug_tail_cap); with 64
    lanes a second round almost never happens, so here the cap forces several
    per launch.  Square lattices of one, two and three words per row and a
    general lattice with open edges still equal the oracle bit for bit."""
    seed, S = 0x5EED0000000000C1, 60
    insts = [crbm.Instance(L=18, J1=1.0, J2=1.0, h=3.0, n_chains=64, sched="geometric", T0=5.0, T1=0.2, id=1),
             crbm.Instance(L=48, J1=1.0, J2=0.5, h=1.0, n_chains=20, sched="linear", T0=3.0, T1=0.3, id=2),
             crbm.Instance(L=96, J1=1.0, J2=2.0, h=0.5, n_chains=5, sched="const", T0=0.8, id=3)]
    lat = crbm.Lattice(rows=12, cols=18, J=[1.0, 0.8, -0.6, 1.2, 0.9, -1.1, 0.5, 1.4, 1.3, -0.7], h_even=0.4,
                       h_odd=-0.2, open_cols=True, n_chains=70, sched="const", T0=0.9, id=4)
    crbm.debug_tail_cap(cap)
    try:
        smp, parts, tr = _run_gpu(insts, seed, S)
        lsmp = crbm.LatticeSampler([lat], seed=seed, n_sweeps=S)
        lspins = torch.empty(lsmp.total_spins, dtype=torch.int8, device="cuda")
        lsmp.sample(S, spins_out=lspins)
        # the same instances in one graph launch, built while the cap is set
        gsmp = crbm.Sampler(insts, seed=seed, n_sweeps=S, launch="graph")
        gspins = torch.empty(gsmp.total_spins, dtype=torch.int8, device="cuda")
        gsmp.sample(S, spins_out=gspins)
        torch.cuda.synchronize()
    finally:
        crbm.debug_tail_cap(64)
    for k, I in enumerate(insts):
        _check_chains(I, parts[k], tr, int(smp.chain_offsets[k]), seed, S, (0, I.n_chains - 1))
    gparts = [p.cpu().numpy() for p in gsmp.split_spins(gspins)]
    for k in range(len(insts)):
        assert np.array_equal(gparts[k], parts[k]), k
    got = lsmp.split_spins(lspins)[0].cpu().numpy()
    ol = oracle.Lattice(12, 18, lat.J, 0.4, -0.2, open_c=True, T0=0.9, id=4)
    for ch in (0, 69):
        s, _, _ = oracle.run_lattice_chain(ol, S, seed, ch, 0, S)
        assert np.array_equal(got[ch], s), ch
    with pytest.raises(crbm.CrbmError):
        crbm.debug_tail_cap(0)
    with pytest.raises(crbm.CrbmError):
        crbm.debug_tail_cap(65)
