"""GPU: the hardware-precision mode (Q5.4 weights and bias, saturating 10-bit
hidden field and 12-bit visible accumulator, 16-bit sigmoid against 16-bit
uniforms; App. A Dimension and Precision) equals the oracle's own
implementation of it bit for bit, trajectory by trajectory, including
schedules that drive every quantity into saturation; MH refuses such
handles."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
crbm = pytest.importorskip("paper_2511_20911_amd")


def _run(insts, seed, S, tile_rows=0, launch="direct"):
    smp = crbm.Sampler(insts, seed=seed, n_sweeps=S, tile_rows=tile_rows, launch=launch, precision="fpga")
    spins = torch.empty(smp.total_spins, dtype=torch.int8, device="cuda")
    tr = torch.empty((S, smp.total_chains, 3), dtype=torch.int32, device="cuda")
    smp.sample(S, spins_out=spins, trace=tr)
    torch.cuda.synchronize()
    return smp, [p.cpu().numpy() for p in smp.split_spins(spins)], tr.cpu().numpy()


def _check(I, part, tr, off, seed, S, chains):
    oi = oracle.Instance(I.L, I.J1, I.J2, I.h, I.sched, I.T0, I.T1, id=I.id, precision=1)
    for ch in chains:
        s, t, _ = oracle.run_chain(oi, S, seed, ch, 0, S, trace=True)
        assert np.array_equal(part[ch], s), f"L={I.L} chain {ch}: spins differ"
        assert np.array_equal(tr[:, off + ch, :], t), f"L={I.L} chain {ch}: trace differs"


def test_hardware_precision_6x6_all_chains_bit_exact():
    """Geometric anneal 3.0 -> 0.01: below T ~ 0.03 the weights, the bias
    (h/T up to 300) and the visible accumulator saturate."""
    seed, S = 0x5EED00000000F001, 600
    print(f"case L=6 seed={seed}", flush=True)
    I = crbm.Instance(L=6, J1=1.0, J2=1.0, h=3.0, n_chains=96, sched="geometric", T0=3.0, T1=0.01, id=3)
    smp, parts, tr = _run([I], seed, S)
    _check(I, parts[0], tr, 0, seed, S, range(96))


@pytest.mark.parametrize("tile_rows", [1, 3, 9])
def test_hardware_precision_18x18_bit_exact_any_tiling(tile_rows):
    seed, S = 0x5EED00000000F002, 300
    print(f"case L=18 R={tile_rows} seed={seed}", flush=True)
    insts = [crbm.Instance(L=18, J1=1.0, J2=0.5, h=4.0, n_chains=10, sched="geometric", T0=5.0, T1=0.02, id=4),
             crbm.Instance(L=18, J1=1.0, J2=2.5, h=0.0, n_chains=7, sched="const", T0=0.7, id=5)]
    smp, parts, tr = _run(insts, seed, S, tile_rows=tile_rows)
    off = smp.chain_offsets
    for k, I in enumerate(insts):
        _check(I, parts[k], tr, int(off[k]), seed, S, sorted({0, 3, I.n_chains - 1}))


def test_hardware_precision_multiword_and_graph():
    """Rows of two and three words, in the persistent graph launch."""
    seed, S = 0x5EED00000000F003, 40
    print(f"case multiword seed={seed}", flush=True)
    insts = [crbm.Instance(L=36, J1=1.0, J2=1.0, h=3.0, n_chains=5, sched="const", T0=0.3, id=6),
             crbm.Instance(L=96, J1=1.0, J2=1.0, h=2.0, n_chains=4, sched="linear", T0=4.0, T1=0.02, id=7)]
    smp, parts, tr = _run(insts, seed, S, launch="graph")
    off = smp.chain_offsets
    for k, I in enumerate(insts):
        _check(I, parts[k], tr, int(off[k]), seed, S, sorted({0, I.n_chains - 1}))


def test_hardware_precision_tables_reach_the_device():
    """The handle's per-sweep tables are the host builder's, and differ from
    the default precision's."""
    I = crbm.Instance(L=6, J1=1.0, J2=1.0, h=3.0, n_chains=4, sched="geometric", T0=3.0, T1=0.05, id=1)
    smp = crbm.Sampler([I], seed=1, n_sweeps=50, precision="fpga")
    ref = crbm.Sampler([I], seed=1, n_sweeps=50)
    for s in (0, 25, 49):
        T = 3.0 * (0.05 / 3.0) ** (s / 49)
        got = smp.sweep_table(0, s)
        assert np.array_equal(got, crbm.table_for(1.0, 1.0, 3.0, T, precision="fpga"))
        assert not np.array_equal(got, ref.sweep_table(0, s))


def test_mh_refuses_hardware_precision():
    I = crbm.Instance(L=6, J1=1.0, J2=1.0, h=3.0, n_chains=16, sched="const", T0=0.5, id=2)
    smp = crbm.Sampler([I], seed=1, n_sweeps=100, precision="fpga")
    net = crbm.ARNet(6)
    net.init_params(seed=1)
    with pytest.raises(crbm.CrbmError) as e:
        crbm.sample_mh(smp, net, 1, 1)
    assert e.value.code == crbm.CRBM_EUNSUPPORTED
