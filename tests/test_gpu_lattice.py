"""GPU parity of the general-lattice sampler (crbm_lattice_*): open or
periodic axes, one coupling per filter, odd/even column fields (App. A
Wrapper Module, Convoluter-Reverse, Accumulator).  Trajectories (final spins
and every sweep's 12 counts), accumulators and the displacement correlation
equal the CPU oracle's bit for bit; a periodic square SS lattice equals the
square-lattice sampler."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
crbm = pytest.importorskip("paper_2511_20911_amd")


def _ol(I):
    return oracle.Lattice(I.rows, I.cols, I.J, I.h_even, I.h_even if I.h_odd is None else I.h_odd,
                          open_r=I.open_rows, open_c=I.open_cols, sched=I.sched, T0=I.T0, T1=I.T1,
                          T_explicit=I.T_explicit, id=I.id)


def _run(lats, seed, S, n_run=None):
    n_run = S if n_run is None else n_run
    smp = crbm.LatticeSampler(lats, seed=seed, n_sweeps=S)
    spins = torch.empty(smp.total_spins, dtype=torch.int8, device="cuda")
    tr = torch.empty((n_run, smp.total_chains, 12), dtype=torch.int32, device="cuda")
    smp.sample(n_run, spins_out=spins, trace=tr)
    torch.cuda.synchronize()
    return smp, [p.cpu().numpy() for p in smp.split_spins(spins)], tr.cpu().numpy()


def _check(lats, smp, parts, tr, seed, S, n_run, picks):
    for k, I in enumerate(lats):
        ol = _ol(I)
        for ch in picks(I):
            s, t, _ = oracle.run_lattice_chain(ol, S, seed, ch, 0, n_run, trace=True)
            assert np.array_equal(parts[k][ch], s), f"lattice {k} chain {ch}: spins differ"
            assert np.array_equal(tr[:, int(smp.chain_offsets[k]) + ch, :], t), f"lattice {k} chain {ch}: counts differ"


def _picks(I):
    return sorted({0, I.n_chains // 2, I.n_chains - 1})


def test_open_and_mixed_boundaries_bit_exact():
    """Strips, open squares and rectangles in one handle (one and two words per
    row), each with its own couplings, fields and schedule; ragged chain
    counts."""
    rng = np.random.default_rng(3)
    S = 200
    lats = [
        crbm.Lattice(rows=18, cols=12, J=crbm.ss_filters(1.0, 1.5), h_even=4.5, open_cols=True, n_chains=70,
                     sched="const", T0=0.8, id=1),
        crbm.Lattice(rows=6, cols=6, J=list(rng.uniform(-1.5, 1.5, 10)), h_even=0.7, h_odd=-0.4, open_rows=True,
                     open_cols=True, n_chains=33, sched="linear", T0=3.0, T1=0.3, id=2),
        crbm.Lattice(rows=10, cols=36, J=crbm.ss_filters(1.0, 1.0), h_even=3.0, open_rows=True, n_chains=65,
                     sched="geometric", T0=5.0, T1=0.2, id=3),
        crbm.Lattice(rows=4, cols=64, J=list(rng.uniform(-2.0, 2.0, 10)), h_even=-1.0, h_odd=2.0, open_rows=True,
                     open_cols=True, n_chains=9, sched="const", T0=0.5, id=4),
        crbm.Lattice(rows=64, cols=8, J=crbm.ss_filters(-1.0, 2.0), h_even=0.3, open_cols=True, n_chains=5,
                     sched="explicit", T_explicit=np.linspace(4.0, 0.5, S), id=5),
    ]
    smp, parts, tr = _run(lats, 0x5EED0000000000F1, S)
    _check(lats, smp, parts, tr, 0x5EED0000000000F1, S, S, _picks)


def test_every_compiled_width_bit_exact():
    """The sampler is compiled once per even column count 4 .. 64: one handle
    holds a lattice of every width (4 or 6 rows, the four boundary kinds in
    turn, random couplings and even/odd fields, 3 chains each), and every
    instance's first and last chains equal the oracle, spins and counts of
    every sweep."""
    rng = np.random.default_rng(17)
    S, seed = 40, 0x5EED0000000000F6
    lats = []
    for k, cols in enumerate(range(4, 66, 2)):
        lats.append(crbm.Lattice(rows=4 + 2 * (k % 2), cols=cols, J=list(rng.uniform(-1.5, 1.5, 10)),
                                 h_even=float(rng.uniform(-1, 1)), h_odd=float(rng.uniform(-1, 1)),
                                 open_rows=bool(k & 1), open_cols=bool(k & 2), n_chains=3,
                                 sched="linear", T0=2.0, T1=0.4, id=40 + k))
    smp, parts, tr = _run(lats, seed, S)
    _check(lats, smp, parts, tr, seed, S, S, lambda I: (0, I.n_chains - 1))


@pytest.mark.parametrize("L", [6, 18, 36])
def test_periodic_square_equals_square_sampler(L):
    """Both axes periodic, J_k = (J1 x 8, J2 x 2), one field: the same
    trajectories as crbm_create / crbm_sample, spins and (M, B1, B2) alike."""
    S, seed = 150, 0x5EED0000000000F2
    lat = crbm.Lattice(rows=L, cols=L, J=crbm.ss_filters(1.0, 1.5), h_even=1.0, n_chains=130, sched="geometric",
                       T0=4.0, T1=0.3, id=7)
    smp, parts, tr = _run([lat], seed, S)
    sq = crbm.Sampler([crbm.Instance(L=L, J1=1.0, J2=1.5, h=1.0, n_chains=130, sched="geometric", T0=4.0, T1=0.3,
                                     id=7)], seed=seed, n_sweeps=S)
    sp = torch.empty(sq.total_spins, dtype=torch.int8, device="cuda")
    trs = torch.empty((S, 130, 3), dtype=torch.int32, device="cuda")
    sq.sample(S, spins_out=sp, trace=trs)
    torch.cuda.synchronize()
    assert np.array_equal(parts[0].reshape(-1), sp.cpu().numpy())
    trs = trs.cpu().numpy()
    assert np.array_equal(trs[..., 0], tr[..., 0] + tr[..., 1])
    assert np.array_equal(trs[..., 1], tr[..., 2:10].sum(-1))
    assert np.array_equal(trs[..., 2], tr[..., 10:].sum(-1))


def test_confined_strip_full_run_bit_exact():
    """The laterally confined lattice of Sec. III.A (12 columns open, 18 rows
    periodic, J2/J1 = 1.5, h = 4.5): a geometric anneal to T = 0.1 over 3000
    sweeps, 512 chains; sampled chains equal the oracle at the end."""
    S, seed = 3000, 0x5EED0000000000F3
    lat = crbm.Lattice(rows=18, cols=12, J=crbm.ss_filters(1.0, 1.5), h_even=4.5, open_cols=True, n_chains=512,
                       sched="geometric", T0=5.0, T1=0.1, id=11)
    smp = crbm.LatticeSampler([lat], seed=seed, n_sweeps=S)
    spins = torch.empty(smp.total_spins, dtype=torch.int8, device="cuda")
    smp.sample(S, spins_out=spins)
    torch.cuda.synchronize()
    got = smp.split_spins(spins)[0].cpu().numpy()
    ol = _ol(lat)
    for ch in (0, 200, 511):
        s, _, _ = oracle.run_lattice_chain(ol, S, seed, ch, 0, S)
        assert np.array_equal(got[ch], s), ch


def test_accumulators_and_correlation_match_oracle():
    """Accumulated counts, M^2, |M|, staggered sums and the displacement
    correlation Cn over measured sweeps equal the oracle's sums; a sampling
    run split over two calls and a reset behave as documented."""
    S, seed = 60, 0x5EED0000000000F4
    lats = [crbm.Lattice(rows=8, cols=12, J=crbm.ss_filters(1.0, 1.5), h_even=2.0, h_odd=1.0, open_cols=True,
                         n_chains=40, sched="const", T0=0.9, id=21),
            crbm.Lattice(rows=6, cols=40, J=crbm.ss_filters(1.0, 0.5), h_even=0.0, open_rows=True, n_chains=3,
                         sched="linear", T0=2.0, T1=0.5, id=22)]
    smp = crbm.LatticeSampler(lats, seed=seed, n_sweeps=S, measure_every=4, burn_in=10, corr=True)
    smp.sample(25)
    smp.sample(35)
    acc, cn = smp.observables()
    for k, I in enumerate(lats):
        ol = _ol(I)
        ref = np.zeros(oracle.LATTICE_N_ACC, np.int64)
        cref = np.zeros(I.rows * (2 * I.cols - 1), np.int64)
        for ch in range(I.n_chains):
            oracle.run_lattice_chain(ol, S, seed, ch, 0, S, measure_every=4, burn_in=10, acc=ref, corr=cref)
        assert np.array_equal(acc[k], ref), k
        assert np.array_equal(cn[k].reshape(-1), cref), k
    smp.reset_observables()
    acc2, cn2 = smp.observables()
    assert not acc2.any() and not any(c.any() for c in cn2)


def test_state_round_trip_and_resume():
    S, seed = 80, 0x5EED0000000000F5
    lat = crbm.Lattice(rows=12, cols=10, J=crbm.ss_filters(1.0, 1.0), h_even=3.0, open_rows=True, open_cols=True,
                       n_chains=20, sched="geometric", T0=3.0, T1=0.4, id=31)
    a = crbm.LatticeSampler([lat], seed=seed, n_sweeps=S)
    a.sample(S)
    full, idx = a.get_state()
    assert idx == S
    b = crbm.LatticeSampler([lat], seed=seed, n_sweeps=S)
    b.sample(30)
    mid, _ = b.get_state()
    c = crbm.LatticeSampler([lat], seed=seed, n_sweeps=S)
    c.set_state(mid, 30)
    c.sample(S - 30)
    out, _ = c.get_state()
    assert torch.equal(full, out)


def test_invalid_arguments_fail_cleanly():
    good = dict(rows=8, cols=8, J=crbm.ss_filters(1.0, 1.0), h_even=0.0, n_chains=4, T0=1.0)
    for bad in (dict(rows=7), dict(cols=66), dict(rows=2), dict(n_chains=0), dict(T0=0.0), dict(T0=float("nan")),
                dict(J=[1.0] * 9 + [float("inf")])):
        kw = dict(good)
        kw.update(bad)
        with pytest.raises(crbm.CrbmError):
            crbm.LatticeSampler([crbm.Lattice(**kw)], seed=1, n_sweeps=10)
    with pytest.raises(crbm.CrbmError):  # a field past int32 at a low temperature
        crbm.LatticeSampler([crbm.Lattice(**dict(good, h_even=1000.0, T0=0.01))], seed=1, n_sweeps=10)
    s = crbm.LatticeSampler([crbm.Lattice(**good)], seed=1, n_sweeps=10)
    with pytest.raises(crbm.CrbmError):
        s.sample(11)
    s.sample(10)
    with pytest.raises(crbm.CrbmError):
        s.sample(1)


def _ref_cases():
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lattice_reference.json")) as f:
        return {c["name"]: c for c in json.load(f)["cases"]}


@pytest.mark.parametrize("name", ["strip12x18_h4.5_T1.0", "strip12x18_h4.5_T0.7", "strip12x18_h3.5_T1.0",
                                  "strip12x18_h2.5_T1.0", "periodic12_oddeven_T0.8", "raw_filters_8x12_T0.8"])
def test_equilibrium_matches_transfer_matrix(name):
    """In equilibrium the general-lattice sampler reproduces the exact <E>/N
    and <m> of the row transfer matrix (tests/golden/lattice_reference.json)
    within 3 standard errors: the confined 12 x 18 strip of Sec. III.A on
    both sides of its transition, a periodic lattice with different even and
    odd column fields, and ten different filter couplings."""
    c = _ref_cases()[name]
    # The confined strip relaxes slowly at low T and at its transition (h = 3.5):
    # the oracle's own 12 x 18 chains, run from a random start, have 5000-sweep
    # block means of E/N that scatter by ~0.01 between chains (T = 0.7, h = 3.5;
    # T = 0.5, h = 4.5) and reach the transfer matrix only after tens of
    # thousands of sweeps.  Agreement within 3 SE of 2048 chains is therefore
    # tested where the chains relax within this run: T = 1 on both sides of the
    # transition, T = 0.7 deep in the confined phase.
    chains, anneal, measure = 2048, 10000, 5000
    sched = np.concatenate([5.0 * (c["T"] / 5.0) ** (np.arange(anneal) / (anneal - 1)), np.full(measure, c["T"])])
    lat = crbm.Lattice(rows=c["rows"], cols=c["cols"], J=c["J"], h_even=c["h_even"], h_odd=c["h_odd"],
                       open_rows=c["open_rows"], open_cols=c["open_cols"], n_chains=chains, sched="explicit",
                       T_explicit=sched, id=40)
    smp = crbm.LatticeSampler([lat], seed=0x5EED0000000000F6, n_sweeps=anneal + measure)
    smp.sample(anneal)
    every = 10
    tr = torch.empty((measure // every, chains, 12), dtype=torch.int32, device="cuda")
    smp.sample(measure, trace=tr, trace_every=every)
    t = tr.cpu().numpy().astype(np.float64)
    N = c["rows"] * c["cols"]
    Jq = np.array([oracle.quantise(x) for x in c["J"]], np.float64)
    E = (t[..., 2:] @ Jq - oracle.quantise(c["h_even"]) * t[..., 0] - oracle.quantise(c["h_odd"]) * t[..., 1]) / 65536 / N
    m = (t[..., 0] + t[..., 1]) / N
    for vals, ref in ((E.mean(0), c["E_per_spin"]), (m.mean(0), c["m"])):
        se = vals.std(ddof=1) / np.sqrt(len(vals))
        assert abs(vals.mean() - ref) < 3 * se, (name, vals.mean(), ref, se)
