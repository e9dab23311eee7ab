"""The learned-proposal pipeline: the training run's lattice symmetries keep
every bond count (CPU); the library's minibatches are the documented ones and
a training run equals its steps one by one (GPU); the parameter initialiser
has the stated statistics, and on a 6x6 plateau lattice the trained proposal
samples the exact law with high acceptance (GPU)."""
import math

import numpy as np
import pytest

import physics as P

torch = pytest.importorskip("torch")
crbm = pytest.importorskip("paper_2511_20911_amd")
from paper_2511_20911_amd import learned  # noqa: E402


@pytest.mark.parametrize("L", [6, 12, 18])
def test_training_symmetries_preserve_every_bond_count(L):
    """The symmetries crbm_ar_batch applies (translations by even vectors,
    the transpose) map the SS lattice onto itself: (M, B1, B2) of every drawn
    configuration equals that of the training configuration it came from,
    and both transposed and untransposed draws occur."""
    import oracle
    from ar_helpers import documented_batch
    rng = np.random.default_rng(L)
    s = (2 * rng.integers(0, 2, (40, L, L)) - 1).astype(np.int8)
    out, _, idx = documented_batch(oracle, s, 64, seed=0x1234 + L, step=3)
    before = P.bond_counts(s[idx])
    after = P.bond_counts(out)
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    transposed = [any(np.array_equal(o, np.roll(s[i], (a, c), (0, 1)).T) for a in range(0, L, 2) for c in range(0, L, 2))
                  and not any(np.array_equal(o, np.roll(s[i], (a, c), (0, 1))) for a in range(0, L, 2)
                              for c in range(0, L, 2)) for o, i in zip(out, idx)]
    assert 0 < sum(transposed) < len(transposed)
    assert len(set(idx.tolist())) > 20  # the draws spread over the training set


def test_odd_translation_is_not_a_symmetry():
    """Control: shifting by one site moves dimers onto empty plaquettes, so B2
    changes for generic configurations (the augmentation must use even shifts)."""
    rng = np.random.default_rng(1)
    s = (2 * rng.integers(0, 2, (64, 6, 6)) - 1).astype(np.int8)
    assert not np.array_equal(P.bond_counts(s)[2], P.bond_counts(np.roll(s, 1, 2))[2])


@pytest.mark.gpu
def test_init_params_statistics():
    net = crbm.ARNet(6)
    net.init_params(seed=9, scale=0.5)
    th = net.get_params()
    # layer 2 (taps 5, cin 32, cout 32) follows layer 1 (4*1*32 weights + 32 biases)
    off = 4 * 32 + 32
    w = th[off:off + 5 * 32 * 32].astype(np.float64)
    b = th[off + 5 * 32 * 32:off + 5 * 32 * 32 + 32]
    sd = 0.5 * math.sqrt(2.0 / (5 * 32))
    assert abs(w.mean()) < 4 * sd / math.sqrt(w.size)
    assert abs(w.std() / sd - 1) < 0.06
    assert np.all(b == 0)
    net2 = crbm.ARNet(6)
    net2.init_params(seed=9, scale=0.5)
    assert np.array_equal(net2.get_params(), th)


@pytest.mark.gpu
def test_learned_mh_moves_between_degenerate_plateau_states_12x12():
    """12x12 on the 1/3 plateau at T = 0.2: from the same ordered states,
    learned MH moves most chains between the six degenerate ground states
    (sectors of learned.plateau_sectors) within 60 cycles, while 600 plain
    Gibbs sweeps move at most a tenth as many: what the trained proposal
    gains where E and O_1/3 cannot tell the states apart."""
    L, T = 12, 0.2
    data = learned.training_set(L, 1.0, 1.0, 3.0, T, n_chains=1024, anneal_sweeps=4000, snapshots=64)
    net = crbm.ARNet(L, seed=4)
    net.init_params(seed=4, scale=0.5)
    learned.train(net, data, steps=400, batch=512)
    del data
    r = learned.sector_moves(net, L, 1.0, 1.0, 3.0, T, n_chains=512, warm_cycles=30, steps=60)
    lm, gb = r["learned"], r["gibbs"]
    assert lm["ordered_fraction"] > 0.9 and gb["ordered_fraction"] > 0.9, r
    assert lm["chains_changed"] > 0.5 and lm["changes_per_chain_step"] > 0.1, r
    assert gb["changes_per_chain_step"] <= 0.1 * lm["changes_per_chain_step"], r


@pytest.mark.gpu
def test_trained_proposal_samples_plateau_6x6():
    """6x6 at (J2, h, T) = (1, 3, 0.4): trained on Gibbs samples, learned MH
    (1 MH : 10 Gibbs) reproduces the exact <E>/N of the transfer matrix within
    3 SE with acceptance above 0.3."""
    from oracle import exact
    L, T = 6, 0.4
    data = learned.training_set(L, 1.0, 1.0, 3.0, T, n_chains=1024, anneal_sweeps=2000, snapshots=64)
    net = crbm.ARNet(L, seed=3)
    net.init_params(seed=3, scale=0.5)
    learned.train(net, data, steps=300, batch=512)
    r = learned.compare(net, L, 1.0, 1.0, 3.0, T, n_chains=1024, cycles=300)
    ref = exact.tm_averages(L, 1.0, 1.0, 3.0, T)["E"]
    lm = r["learned"]
    assert lm["acceptance"] > 0.3, lm
    assert abs(lm["E_per_spin"] - ref) < 3 * lm["se"] + 1e-12, (lm, ref)
    assert r["gibbs"]["ess_per_s"] > 0 and lm["ess_per_s"] > 0


@pytest.mark.gpu
@pytest.mark.parametrize("L,augment", [(6, True), (18, True), (12, False)])
def test_library_minibatches_are_the_documented_ones(L, augment):
    import oracle
    from ar_helpers import documented_batch
    rng = np.random.default_rng(5 + L)
    s = (2 * rng.integers(0, 2, (300, L, L)) - 1).astype(np.int8)
    pts = rng.integers(0, 7, 300).astype(np.int32)
    got, gp, gi = crbm.train_batch(torch.from_numpy(s).cuda(), 96, seed=0xABCDEF0123, step=41, augment=augment,
                                   points=torch.from_numpy(pts).cuda())
    ref, rp, ri = documented_batch(oracle, s, 96, seed=0xABCDEF0123, step=41, augment=augment, points=pts)
    assert np.array_equal(gi.cpu().numpy(), ri)
    assert np.array_equal(gp.cpu().numpy(), rp)
    assert np.array_equal(got.cpu().numpy(), ref)


@pytest.mark.gpu
@pytest.mark.parametrize("cond", [False, True])
def test_training_run_equals_its_steps(cond):
    """crbm_ar_train over 7 steps (learning rate switching after 3.5 steps)
    leaves the same parameters, bit for bit, as 7 calls of
    crbm_ar_train_step_cond on the minibatches crbm_ar_batch draws."""
    L, n, B = 6, 500, 64
    rng = np.random.default_rng(9)
    data = torch.from_numpy((2 * rng.integers(0, 2, (n, L, L)) - 1).astype(np.int8)).cuda()
    pts = torch.from_numpy(rng.integers(0, 3, n).astype(np.int32)).cuda() if cond else None
    feats = np.array([[1.0, 0.5, -1.0], [0.5, 0.2, 0.0], [2.0, 0.9, 0.3]])

    def fresh():
        net = crbm.ARNet(L, cond_points=3 if cond else 0)
        if cond:
            net.set_points(feats)
        net.init_params(seed=4, scale=0.5)
        return net

    a = fresh()
    loss_a = a.train(data, 7, batch=B, lr=2e-3, lr_late=5e-4, late_from=0.5, seed=77, step0=3, points=pts)
    b = fresh()
    for k in range(7):
        x, p, _ = crbm.train_batch(data, B, seed=77, step=3 + k, points=pts)
        loss_b = b.train_step(x, 2e-3 if k < 4 else 5e-4, points=p if cond else None)
    assert np.array_equal(a.get_params(), b.get_params())
    assert loss_a == loss_b
    assert not np.array_equal(a.get_params(), fresh().get_params())


@pytest.mark.gpu
def test_learned_mh_beats_gibbs_on_the_plateau_18x18():
    """The learned part's claim at 18x18 on the 1/3 plateau (Sec. III.A point
    J2/J1 = 1, h/J1 = 3), T = 0.2: a proposal trained on 2^20 Gibbs samples,
    run as 1 MH : 10 Gibbs sweeps on 8192 chains, gives more energy and
    order-parameter effective samples per second than plain Gibbs run for the
    same wall time from the same seeded start; its <E>/N lies within 3 SE of
    the exact transfer-matrix value, and it is at least as close to that value
    as plain Gibbs (whose chains freeze into domains of different plateau
    translations at this temperature)."""
    import json
    import os
    L, T = 18, 0.2
    ref_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "plateau_reference.json")
    with open(ref_path) as f:
        ref = [v["E_per_spin"] for v in json.load(f)["values"] if v["L"] == 12 and v["T"] == T][0]
    data = learned.training_set(L, 1.0, 1.0, 3.0, T)
    net = crbm.ARNet(L, seed=5)
    net.init_params(seed=5, scale=0.5)
    learned.train(net, data, steps=800)
    del data
    r = learned.compare(net, L, 1.0, 1.0, 3.0, T, cycles=500)
    lm, gb = r["learned"], r["gibbs"]
    assert lm["acceptance"] > 0.3, lm
    assert lm["ess_per_s"] > gb["ess_per_s"] and lm["ess_min_per_s"] > gb["ess_min_per_s"], (lm, gb)
    assert abs(lm["E_per_spin"] - ref) <= 3 * lm["se"] + 1e-12, (lm["E_per_spin"], ref, lm["se"])
    assert abs(lm["E_per_spin"] - ref) <= abs(gb["E_per_spin"] - ref) + 1e-12, (lm["E_per_spin"], gb["E_per_spin"], ref)
