"""GPU tests of the conditional learned proposal: one network whose biases
are shifted per Hamiltonian point by an MLP of the point's features.  Scorer,
gradient and sampler against the oracle, sampler self-consistency across
points, and multi-instance MH reproducing two exact 4x4 laws at once."""
import math

import numpy as np
import pytest

import oracle
import physics as P
from oracle import ar
from ar_helpers import (GRAD_ATOL_OF_BLOCK_MAX, GRAD_REL_L2, assert_grad_blocks, decisions_follow_rule, flatten,
                        proposal_uniforms)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
crbm = pytest.importorskip("paper_2511_20911_amd")

LOGQ_TOL_PER_SITE = 1e-3  # as for the unconditional network (same kernels, same rounding points)
INIT_SCALE = 0.5
FEATS = np.array([[1.0, 0.0, math.log(0.4)], [0.5, 1.2, math.log(0.2)], [2.0, -0.5, 0.0]])


def _cond_params(seed, w2_scale=0.3):
    base = ar.init_params(seed=seed, scale=INIT_SCALE)
    c = ar.init_cond(seed=seed + 1)
    rng = np.random.default_rng(seed + 2)
    c["b1"] = rng.standard_normal(c["b1"].shape) * 0.2
    c["W2"] = rng.standard_normal(c["W2"].shape) * w2_scale
    return base, c


def _flat(base, c):
    return np.concatenate([flatten(base), c["W1"].ravel(), c["b1"].ravel(), c["W2"].ravel()]).astype(np.float32)


def _net(L, base, c, feats=FEATS):
    net = crbm.ARNet(L, cond_points=len(feats))
    net.set_points(feats)
    net.set_params(_flat(base, c))
    return net


def _spins(n, L, seed):
    return (2 * np.random.default_rng(seed).integers(0, 2, (n, L, L)) - 1).astype(np.int8)


def _pts(idx):
    return torch.from_numpy(np.asarray(idx, np.int32)).cuda()


def test_parameter_count():
    net = crbm.ARNet(6, cond_points=3)
    assert net.num_params == flatten(ar.init_params()).size + 3 * 32 + 32 + 32 * 12 * 32


@pytest.mark.parametrize("L", [6, 36])
def test_cond_scorer_matches_oracle(L):
    """Mixed points in one batch (fused scorer at 6x6, layer-by-layer scorer
    at 36x36): log q within tolerance of the oracle with each sample's offsets;
    scoring the same states at other points changes log q."""
    base, c = _cond_params(40 + L)
    net = _net(L, base, c)
    n = 24
    s = _spins(n, L, L)
    idx = np.arange(n) % 3
    got = net.logq(torch.from_numpy(s).cuda(), points=_pts(idx)).cpu().numpy()
    _, cache = ar.forward(base, s, bias_add=ar.cond_bias(c, FEATS)[idx])
    ref = ar.proposal_logq(cache["logit"], s)
    assert np.all(np.abs(got - ref) < LOGQ_TOL_PER_SITE * L * L), np.abs(got - ref).max()
    other = net.logq(torch.from_numpy(s).cuda(), points=_pts((idx + 1) % 3)).cpu().numpy()
    assert np.abs(other - got).min() > 1e-3


def test_fresh_conditional_network_scores_like_its_base():
    """crbm_ar_init_params zeroes W2: every point scores like the base network."""
    L = 6
    net = crbm.ARNet(L, cond_points=3)
    net.set_points(FEATS)
    net.init_params(seed=9)
    flat = net.get_params()
    base_only = crbm.ARNet(L)
    base_only.set_params(flat[:base_only.num_params])
    s = torch.from_numpy(_spins(12, L, 3)).cuda()
    a = net.logq(s, points=_pts(np.arange(12) % 3))
    b = base_only.logq(s)
    assert torch.equal(a, b)


@pytest.mark.parametrize("L,B", [(4, 16), (18, 64)])
def test_cond_gradient_matches_oracle(L, B):
    """Gradient of the mean NLL with respect to the network and the MLP,
    mixed points, against the oracle's backward plus the MLP backward:
    element by element per block (each layer's weights and biases, W1, b1,
    W2), with the bf16 bound of the unconditional gradient test."""
    base, c = _cond_params(50, w2_scale=0.2)
    net = _net(L, base, c)
    s = _spins(B, L, 7)
    idx = (np.arange(B) * 5 + np.arange(B) // 3) % 3
    g, loss = net.grad(torch.from_numpy(s).cuda(), points=_pts(idx))
    ref_loss, ref_grads, gb = ar.loss_and_grad(base, s, bias_add=ar.cond_bias(c, FEATS)[idx], per_sample_bias=True)
    gc = ar.cond_grad(c, FEATS, idx, gb)
    ref = np.concatenate([flatten(ref_grads).astype(np.float64), gc["W1"].ravel(), gc["b1"].ravel(), gc["W2"].ravel()])
    assert abs(loss - ref_loss) < 1e-5 * L * L  # a mean of per-sample log q: the log q bound's scale
    n_net = flatten(ref_grads).size
    assert_grad_blocks(g[:n_net], ref_grads, base)
    off = n_net
    for name in ("W1", "b1", "W2"):
        b = gc[name].ravel()
        a = g[off:off + b.size].astype(np.float64)
        off += b.size
        np.testing.assert_allclose(a, b, rtol=0, atol=GRAD_ATOL_OF_BLOCK_MAX * np.abs(b).max(), err_msg=name)
        assert np.linalg.norm(a - b) / np.linalg.norm(b) < GRAD_REL_L2, name
    assert off == g.size


@pytest.mark.parametrize("L,n", [(6, 40), (36, 24)])
def test_cond_sampler(L, n):
    """Proposals at mixed points: sampler log q == scorer log q bit for bit; a
    chain's proposal depends on its own point only; picked chains match the
    oracle's log q and follow the documented uniforms."""
    base, c = _cond_params(60 + L)
    net = _net(L, base, c)
    idx = (np.arange(n) * 7) % 3
    s, lq = net.sample(n, seed=3, step=1, id=2, points=_pts(idx))
    assert torch.equal(lq, net.logq(s, points=_pts(idx)))
    s1, lq1 = net.sample(n, seed=3, step=1, id=2, points=_pts(np.ones(n, np.int32)))
    sel = torch.from_numpy(idx == 1).cuda()
    assert torch.equal(s[sel], s1[sel]) and torch.equal(lq[sel], lq1[sel])
    pick = [0, n // 2 + 1, n - 1]
    sn = s.cpu().numpy()[pick]
    off = ar.cond_bias(c, FEATS)[idx[pick]]
    _, cache = ar.forward(base, sn, bias_add=off)
    ref = ar.proposal_logq(cache["logit"], sn)
    assert np.all(np.abs(lq.cpu().numpy()[pick] - ref) < LOGQ_TOL_PER_SITE * L * L)
    for k, ch in enumerate(pick):
        ok, _ = decisions_follow_rule(ar, sn[k], cache["logit"][k], proposal_uniforms(oracle, L * L, 3, 1, ch, 2))
        assert ok, ch


def _exact_law(L, J2, h, T):
    st = P.all_states(L)
    J1q, J2q, hq = (oracle.quantise(x) / 65536 for x in (1.0, J2, h))
    E = P.energy(st, J1q, J2q, hq)
    w = np.exp(-(E - E.min()) / T)
    return st, w / w.sum()


@pytest.mark.parametrize("gibbs_per_mh", [0, 1])
def test_cond_mh_two_instances_reproduce_exact_4x4(gibbs_per_mh):
    """One handle with two Hamiltonian points, one conditional network trained
    on exact samples of both: MH (pure, and interleaved with Gibbs), started
    from Gibbs-equilibrated states, keeps each point's exact 4x4 averages of E
    and m within 3 SE, each chain accepting on its own point's target.  (An
    independence sampler started far from equilibrium can stay stuck where
    the proposal's tails are lighter than the target's, so the chains start
    equilibrated: what is tested is that MH leaves each law invariant.)"""
    L = 4
    pts = [(1.0, 3.0, 1.0), (0.5, 0.5, 0.8)]  # (J2, h, T)
    feats = np.array([[J2, h / 4.0, math.log(T)] for J2, h, T in pts])
    laws = [_exact_law(L, *p) for p in pts]
    net = crbm.ARNet(L, cond_points=2)
    net.set_points(feats)
    net.init_params(seed=71, scale=INIT_SCALE)
    rng = np.random.default_rng(72)
    for _ in range(200):
        batch, where = [], []
        for k, (st, pr) in enumerate(laws):
            batch.append(st[rng.choice(len(pr), size=512, p=pr)])
            where.append(np.full(512, k, np.int32))
        net.train_step(torch.from_numpy(np.concatenate(batch)).cuda(), 3e-3,
                       points=torch.from_numpy(np.concatenate(where)).cuda())
    n_chains, cycles = 256, 300
    insts = [crbm.Instance(L=L, J1=1.0, J2=J2, h=h, n_chains=n_chains, sched="const", T0=T, id=3 + k)
             for k, (J2, h, T) in enumerate(pts)]
    burn = 200
    smp = crbm.Sampler(insts, seed=11, n_sweeps=burn + cycles * max(gibbs_per_mh, 1) + 10)
    smp.sample(burn)
    tr = torch.empty((cycles, 2 * n_chains, 3), dtype=torch.int32, device="cuda")
    acc = crbm.sample_mh(smp, net, cycles, gibbs_per_mh, trace=tr)
    assert 0.3 * cycles * 2 * n_chains < acc <= cycles * 2 * n_chains, acc
    t = tr.cpu().numpy().astype(np.float64)[50:]
    for k, (J2, h, T) in enumerate(pts):
        tk = t[:, k * n_chains:(k + 1) * n_chains]
        J1q, J2q, hq = (oracle.quantise(x) for x in (1.0, J2, h))
        E = (J1q * tk[:, :, 1] + J2q * tk[:, :, 2] - hq * tk[:, :, 0]) / 65536 / 16
        m = tk[:, :, 0] / 16
        ex = P.exact_averages(4, J1q / 65536, J2q / 65536, hq / 65536, T)
        for vals, ref in ((E.mean(axis=0), ex["E"]), (m.mean(axis=0), ex["m"])):
            se = vals.std(ddof=1) / math.sqrt(len(vals))
            assert abs(vals.mean() - ref) < 3 * se, (k, vals.mean(), ref, se)


def test_unconditional_mh_on_two_instances():
    """An unconditional network also drives MH over a two-instance handle:
    started from Gibbs-equilibrated states, pure MH keeps each instance's own
    exact 4x4 law although the proposal was trained for the first one only."""
    L = 4
    pts = [(1.0, 3.0, 1.0), (1.0, 3.0, 1.3)]
    net = crbm.ARNet(L)
    net.init_params(seed=81, scale=INIT_SCALE)
    st, pr = _exact_law(L, *pts[0])
    rng = np.random.default_rng(82)
    for _ in range(150):
        net.train_step(torch.from_numpy(st[rng.choice(len(pr), size=1024, p=pr)]).cuda(), 3e-3)
    n_chains, cycles = 256, 300
    insts = [crbm.Instance(L=L, J1=1.0, J2=J2, h=h, n_chains=n_chains, sched="const", T0=T, id=5 + k)
             for k, (J2, h, T) in enumerate(pts)]
    smp = crbm.Sampler(insts, seed=13, n_sweeps=210)
    smp.sample(200)
    tr = torch.empty((cycles, 2 * n_chains, 3), dtype=torch.int32, device="cuda")
    crbm.sample_mh(smp, net, cycles, 0, trace=tr)
    t = tr.cpu().numpy().astype(np.float64)[50:]
    exs, ses = [], []
    for k, (J2, h, T) in enumerate(pts):
        tk = t[:, k * n_chains:(k + 1) * n_chains]
        J1q, J2q, hq = (oracle.quantise(x) for x in (1.0, J2, h))
        E = (J1q * tk[:, :, 1] + J2q * tk[:, :, 2] - hq * tk[:, :, 0]) / 65536 / 16
        ex = P.exact_averages(4, J1q / 65536, J2q / 65536, hq / 65536, T)
        exs.append(ex["E"])
        vals = E.mean(axis=0)
        se = vals.std(ddof=1) / math.sqrt(len(vals))
        ses.append(se)
        assert abs(vals.mean() - ex["E"]) < 3 * se, (k, vals.mean(), ex["E"], se)
    # the two laws are far apart on this scale: a shared target would fail one of them
    assert abs(exs[0] - exs[1]) > 8 * max(ses), (exs, ses)


# ---------------------------------------------------------------- error paths (host-side checks, no kernel fault)

def _code(fn):
    try:
        fn()
    except crbm.CrbmError as e:
        return e.code
    return crbm.CRBM_OK


def test_conditional_errors():
    assert _code(lambda: crbm.ARNet(6, cond_points=129)) == crbm.CRBM_EINVAL
    assert _code(lambda: crbm.ARNet(6, cond_points=-1)) == crbm.CRBM_EINVAL
    net = crbm.ARNet(6, cond_points=2)
    s = torch.from_numpy(_spins(4, 6, 1)).cuda()
    # no points yet: every conditional computation refuses
    assert _code(lambda: net.logq(s)) == crbm.CRBM_ESTATE
    assert _code(lambda: net.sample(4, seed=1)) == crbm.CRBM_ESTATE
    assert _code(lambda: net.train_step(s, 1e-3)) == crbm.CRBM_ESTATE
    assert _code(lambda: net.set_points(np.zeros((3, 3)))) == crbm.CRBM_EINVAL       # more than cond_points
    assert _code(lambda: net.set_points(np.array([[0.0, np.nan, 1.0]]))) == crbm.CRBM_EINVAL
    plain = crbm.ARNet(6)
    assert _code(lambda: plain.set_points(np.zeros((1, 3)))) == crbm.CRBM_EINVAL     # not conditional
    net.set_points(FEATS[:2])
    assert _code(lambda: net.logq(s)) == crbm.CRBM_OK
    # out-of-range point indices are clamped, not read out of bounds
    a = net.logq(s, points=_pts([5, -3, 1, 0]))
    b = net.logq(s, points=_pts([1, 0, 1, 0]))
    assert torch.equal(a, b)


def test_mh_handle_checks():
    L = 4
    net = crbm.ARNet(L, cond_points=2)
    net.set_points(FEATS[:1])  # one point, two instances below
    two = crbm.Sampler([crbm.Instance(L=L, J2=1.0, h=3.0, n_chains=8, T0=1.0, id=k) for k in range(2)], seed=1,
                       n_sweeps=10)
    assert _code(lambda: crbm.sample_mh(two, net, 1, 0)) == crbm.CRBM_EINVAL
    plain = crbm.ARNet(L)
    mixed = crbm.Sampler([crbm.Instance(L=L, n_chains=8, T0=1.0, id=0), crbm.Instance(L=6, n_chains=8, T0=1.0, id=1)],
                         seed=1, n_sweeps=10)
    assert _code(lambda: crbm.sample_mh(mixed, plain, 1, 0)) == crbm.CRBM_EUNSUPPORTED
    anneal = crbm.Sampler([crbm.Instance(L=L, n_chains=8, sched="linear", T0=2.0, T1=1.0, id=0)], seed=1, n_sweeps=10)
    assert _code(lambda: crbm.sample_mh(anneal, plain, 1, 0)) == crbm.CRBM_EUNSUPPORTED
    other_L = crbm.ARNet(6)
    single = crbm.Sampler([crbm.Instance(L=L, n_chains=8, T0=1.0, id=0)], seed=1, n_sweeps=10)
    assert _code(lambda: crbm.sample_mh(single, other_L, 1, 0)) == crbm.CRBM_EINVAL


def test_cond_sample_steps_equal_separate_calls():
    """Batched proposals of a conditional network (every batch on the same
    per-chain points) equal separate launches bit for bit."""
    base, c = _cond_params(77)
    net = _net(6, base, c)
    n = 40
    idx = _pts((np.arange(n) * 5) % 3)
    s, lq = net.sample_steps(n, 3, seed=8, step0=4, id=1, points=idx)
    for k in range(3):
        s1, lq1 = net.sample(n, seed=8, step=4 + k, id=1, points=idx)
        assert torch.equal(s[k], s1) and torch.equal(lq[k], lq1), k
