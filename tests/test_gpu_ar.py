"""GPU tests of the learned proposal: the bf16 matrix-core kernels against the
oracle (which rounds to bf16 at the same points), sampler self-consistency,
MH reproducing exact 4x4 averages, and what training gains."""
import ctypes as ct
import math

import numpy as np
import pytest

import oracle
import physics as P
from oracle import ar
from ar_helpers import (assert_grad_blocks, decisions_follow_rule, flatten, proposal_uniforms,
                        unflatten)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
crbm = pytest.importorskip("paper_2511_20911_amd")

# Kernel and oracle round the same values to bf16; their fp32 / fp64 sums
# differ in the last bits, which flips an occasional bf16 rounding (2^-8
# relative) that then propagates through the remaining layers.  With weights
# of the scale training produces (|logit| of order 1) the oracle run with its
# pre-rounding sums perturbed at the fp32 level moves log q by at most
# ~3e-6 per site; the bound below leaves a wide margin.  (With weights large
# enough that |logit| reaches hundreds the network amplifies such flips
# chaotically and no fixed tolerance holds, so the tests use scale 0.5.)
LOGQ_TOL_PER_SITE = 1e-3
INIT_SCALE = 0.5


def _rand_spins(n, L, seed):
    rng = np.random.default_rng(seed)
    return (2 * rng.integers(0, 2, (n, L, L)) - 1).astype(np.int8)


@pytest.mark.parametrize("L", [4, 6, 18])
def test_scorer_matches_oracle(L):
    params = ar.init_params(seed=10 + L, scale=INIT_SCALE)
    net = crbm.ARNet(L)
    net.set_params(flatten(params))
    s = _rand_spins(40, L, L)
    got = net.logq(torch.from_numpy(s).cuda()).cpu().numpy()
    _, c = ar.forward(unflatten(flatten(params), params), s)
    ref = ar.proposal_logq(c["logit"], s)
    assert np.all(np.abs(got - ref) < LOGQ_TOL_PER_SITE * L * L), np.abs(got - ref).max()


@pytest.mark.parametrize("L,B", [(4, 16), (6, 16), (18, 64), (18, 512)])
def test_gradient_matches_oracle(L, B):
    """The training gradient element by element, per layer, weights and
    biases separately.  At 18x18, 64 samples run 41 weight-gradient chunks of
    512 pixels with both wavefronts of a chunk active and a ragged last chunk;
    512 samples give the convolutions several 32-pixel tiles per wavefront
    (operands loaded a tile ahead, ReLU gates and bias sums carried across
    tiles): the path of the benchmark's training steps."""
    print(f"case L={L} B={B}", flush=True)
    params = ar.init_params(seed=20 + L, scale=INIT_SCALE)
    net = crbm.ARNet(L)
    flat = flatten(params)
    net.set_params(flat)
    s = _rand_spins(B, L, 100 + L)
    g, loss = net.grad(torch.from_numpy(s).cuda())
    p64 = unflatten(flat, params)
    ref_loss, ref_grads = ar.loss_and_grad(p64, s)
    assert abs(loss - ref_loss) < 1e-5 * L * L  # a mean of per-sample log q: the log q bound's scale
    assert_grad_blocks(g, ref_grads, params)


def _plateau_net(L=18, T=0.4, steps=300):
    """A network trained by the library on its own Gibbs samples at the 1/3
    plateau point (J2/J1 = 1, h/J1 = 3), and held-out Gibbs samples."""
    from paper_2511_20911_amd import learned
    data = learned.training_set(L, 1.0, 1.0, 3.0, T, n_chains=1024, anneal_sweeps=4000, snapshots=64, spacing=20)
    net = crbm.ARNet(L)
    net.init_params(seed=5, scale=0.5)
    learned.train(net, data[:-1024], steps=steps, batch=512)
    return net, data[-1024:]


def test_trained_network_matches_oracle_18x18():
    """At weights trained on plateau samples (logits up to |x| ~ 14, the
    regime of the learned-MH runs): log q of held-out Gibbs samples and of
    the network's own proposals, and the gradient on 64 Gibbs samples, against
    the oracle.  Most configurations agree to ~1e-6 (no bf16 rounding falls
    differently); a flipped rounding moves a confident site's log-probability
    by up to ~1e-2: measured at most 7e-5 per site over a configuration, so
    the bound is 2.5e-4 per site, and the median must stay below 1e-4."""
    L = 18
    net, held = _plateau_net(L)
    flat = net.get_params()
    like = ar.init_params(seed=0)
    p64 = unflatten(flat, like)
    idx = torch.arange(0, 1024, 16, device="cuda")
    for name, S in (("gibbs", held[idx].contiguous()), ("proposals", net.sample(64, seed=3, step=1, id=1)[0])):
        got = net.logq(S).cpu().numpy()
        sn = S.cpu().numpy()
        _, c = ar.forward(p64, sn)
        assert np.abs(c["logit"]).max() > 8.0  # a confident, trained network
        d = np.abs(got - ar.proposal_logq(c["logit"], sn))
        assert d.max() < 2.5e-4 * L * L, (name, d.max())
        assert np.median(d) < 1e-4, (name, np.median(d))
    S = held[idx].contiguous()
    g, loss = net.grad(S)
    ref_loss, ref_grads = ar.loss_and_grad(p64, S.cpu().numpy())
    assert abs(loss - ref_loss) < 1e-5 * L * L
    assert_grad_blocks(g, ref_grads, like)


def test_gradient_of_a_large_batch_is_the_mean_of_its_parts():
    """At 1024 samples of 18 x 18 the convolution launches give each wavefront
    several 32-pixel tiles (operands loaded a tile ahead, ReLU gate and bias
    sums carried across tiles); at 64 samples each wavefront has at most one
    tile.  The mean-loss gradient is linear in the samples, so the big batch's
    gradient must equal the mean of its 16 parts' gradients up to fp32
    summation order."""
    L, n, parts = 18, 1024, 16
    params = ar.init_params(seed=77, scale=INIT_SCALE)
    net = crbm.ARNet(L)
    net.set_params(flatten(params))
    s = torch.from_numpy(_rand_spins(n, L, 78)).cuda()
    g, loss = net.grad(s)
    ref = np.zeros_like(g, dtype=np.float64)
    ref_loss = 0.0
    m = n // parts
    for k in range(parts):
        gk, lk = net.grad(s[k * m:(k + 1) * m].contiguous())
        ref += gk.astype(np.float64) / parts
        ref_loss += lk / parts
    assert abs(loss - ref_loss) < 1e-5 * L * L  # a mean of per-sample log q: the log q bound's scale, (loss, ref_loss)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    assert rel < 1e-4, rel
    assert np.abs(g - ref).max() < 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("L,n", [(6, 96), (18, 40), (36, 24)])
def test_sampler_logq_equals_scorer_and_follows_logits(L, n):
    """Ancestral sampler vs scorer: identical log q (the fused one-workgroup
    scorer for L <= 32, the layer-by-layer one above), both within tolerance
    of the oracle, and every decision follows the documented uniforms."""
    params = ar.init_params(seed=31, scale=INIT_SCALE)
    net = crbm.ARNet(L)
    net.set_params(flatten(params))
    s, lq = net.sample(n, seed=7, step=3, id=2)
    lq2 = net.logq(s)
    assert torch.equal(lq, lq2)  # same per-site arithmetic in both kernels: identical
    sn = s.cpu().numpy()
    _, c = ar.forward(unflatten(flatten(params), params), sn)
    ref = ar.proposal_logq(c["logit"], sn)
    assert np.all(np.abs(lq.cpu().numpy() - ref) < LOGQ_TOL_PER_SITE * L * L)
    # the decisions used the documented uniforms and the integer rule, up to near-ties
    near_share = []
    for ch in range(n):
        u = proposal_uniforms(oracle, L * L, 7, 3, ch, 2)
        ok, near = decisions_follow_rule(ar, sn[ch], c["logit"][ch], u)
        assert ok, ch
        near_share.append(near)
    assert np.mean(near_share) < 0.01


@pytest.mark.parametrize("L", [6, 18])
def test_sampler_chains_independent_of_batch_size(L):
    """A chain's configuration and log q depend only on (network, seed, step,
    id, chain index): batches that launch one, two or four wavefronts per
    workgroup, with ragged last workgroups, agree chain by chain, and sampled
    chains at the batch edges match the oracle's log q and uniforms."""
    params = ar.init_params(seed=37, scale=INIT_SCALE)
    net = crbm.ARNet(L)
    net.set_params(flatten(params))
    runs = {n: net.sample(n, seed=5, step=1, id=4) for n in (16, 40, 4100, 8200)}
    s_ref, lq_ref = runs[16]
    for n, (s, lq) in runs.items():
        assert torch.equal(s[:16], s_ref), n
        assert torch.equal(lq[:16], lq_ref), n
        assert torch.equal(lq, net.logq(s)), n
    s40, lq40 = runs[40]
    assert torch.equal(runs[8200][0][:40], s40) and torch.equal(runs[8200][1][:40], lq40)
    s, lq = runs[8200]
    pick = [4095, 4099, 8191, 8199]
    sn = s.cpu().numpy()[pick]
    _, c = ar.forward(unflatten(flatten(params), params), sn)
    ref = ar.proposal_logq(c["logit"], sn)
    assert np.all(np.abs(lq.cpu().numpy()[pick] - ref) < LOGQ_TOL_PER_SITE * L * L)
    for k, ch in enumerate(pick):
        ok, _ = decisions_follow_rule(ar, sn[k], c["logit"][k], proposal_uniforms(oracle, L * L, 5, 1, ch, 4))
        assert ok, ch


def test_training_reduces_loss():
    L = 6
    net = crbm.ARNet(L)
    net.set_params(flatten(ar.init_params(seed=41)))
    # a structured target: striped configurations with noise
    rng = np.random.default_rng(3)
    base = np.where(np.arange(L)[None, :, None] % 2 == 0, 1, -1) * np.ones((512, L, L))
    flip = rng.random((512, L, L)) < 0.05
    s = torch.from_numpy(np.where(flip, -base, base).astype(np.int8)).cuda()
    first = net.train_step(s, 3e-3)
    for _ in range(60):
        last = net.train_step(s, 3e-3)
    assert last < 0.5 * first, (first, last)


def _exact_law(L, J2, h, T):
    """All 2^(L*L) states and their probabilities under exp(-H_q / T)."""
    st = P.all_states(L)
    J1q, J2q, hq = (oracle.quantise(x) / 65536 for x in (1.0, J2, h))
    E = P.energy(st, J1q, J2q, hq)
    w = np.exp(-(E - E.min()) / T)
    return st, w / w.sum()


def _trained_net(L, J2, h, T, steps=150, batch=1024, seed=61):
    """A network fitted to exact samples of the 4x4 law (maximum likelihood)."""
    st, p = _exact_law(L, J2, h, T)
    rng = np.random.default_rng(seed)
    net = crbm.ARNet(L)
    net.set_params(flatten(ar.init_params(seed=seed, scale=INIT_SCALE)))
    for _ in range(steps):
        idx = rng.choice(len(p), size=batch, p=p)
        net.train_step(torch.from_numpy(st[idx]).cuda(), 3e-3)
    return net


def _mh_run(net, L, J2, h, T, gibbs_per_mh, cycles, n_chains=256, seed=11, with_order=False, burn=0):
    inst = crbm.Instance(L=L, J1=1.0, J2=J2, h=h, n_chains=n_chains, sched="const", T0=T, id=3)
    smp = crbm.Sampler([inst], seed=seed, n_sweeps=burn + cycles * max(gibbs_per_mh, 1) + 10)
    if burn:
        smp.sample(burn)  # Gibbs burn-in: start the MH chains from equilibrium
    tr = torch.empty((cycles, n_chains, 3), dtype=torch.int32, device="cuda")
    od = torch.empty_like(tr) if with_order else None
    acc = crbm.sample_mh(smp, net, cycles, gibbs_per_mh, trace=tr, order=od)
    if with_order:
        st, _ = smp.get_state()
        return acc, tr.cpu().numpy().astype(np.float64), od.cpu().numpy(), st.cpu().numpy().reshape(n_chains, L, L)
    return acc, tr.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("gibbs_per_mh", [0, 1])
def test_mh_reproduces_exact_4x4(gibbs_per_mh):
    """Independent MH with a trained network's proposals (pure, and
    interleaved with Gibbs) samples the CRBM's law: 4x4 averages of E and m
    within 3 SE (over chains) of exact enumeration."""
    L, J2, h, T = 4, 1.0, 3.0, 1.0
    net = _trained_net(L, J2, h, T)
    cycles, n_chains = 300, 256
    acc, t = _mh_run(net, L, J2, h, T, gibbs_per_mh, cycles, n_chains)
    assert 0 < acc <= cycles * n_chains
    t = t[50:]
    J1q, J2q, hq = (oracle.quantise(x) for x in (1.0, J2, h))
    E = (J1q * t[:, :, 1] + J2q * t[:, :, 2] - hq * t[:, :, 0]) / 65536 / 16
    m = t[:, :, 0] / 16
    ex = P.exact_averages(4, J1q / 65536, J2q / 65536, hq / 65536, T)
    for vals, ref in ((E.mean(axis=0), ex["E"]), (m.mean(axis=0), ex["m"])):
        se = vals.std(ddof=1) / math.sqrt(len(vals))
        assert abs(vals.mean() - ref) < 3 * se, (vals.mean(), ref, se)


def test_training_gains_over_untrained_proposal():
    """Pure MH at 4x4 on the 1/3 plateau, from Gibbs-equilibrated states: the
    trained proposal is accepted far more often than the untrained one, and
    the energy trace of the trained sampler decorrelates within a few cycles.
    (From the random start, chains can stay in high-energy states whose q is
    far below pi for hundreds of cycles: an independence sampler's burn-in is
    not what this test measures.)"""
    L, J2, h, T = 4, 1.0, 3.0, 0.7
    cycles = 400
    untrained = crbm.ARNet(L)
    untrained.set_params(flatten(ar.init_params(seed=61, scale=INIT_SCALE)))
    a0, _ = _mh_run(untrained, L, J2, h, T, 0, cycles, burn=200)
    a1, t1 = _mh_run(_trained_net(L, J2, h, T), L, J2, h, T, 0, cycles, burn=200)
    r0, r1 = a0 / (cycles * 256), a1 / (cycles * 256)
    assert r1 > 0.5 and r1 > 5 * r0, (r0, r1)
    from oracle import stats
    J1q, J2q, hq = (oracle.quantise(x) for x in (1.0, J2, h))
    e = J1q * t1[100:, :, 1] + J2q * t1[100:, :, 2] - hq * t1[100:, :, 0]
    tau1 = stats.tau_int(e, max_lag=200)[0]
    assert tau1 < 5.0, tau1


def test_mh_order_trace_is_the_states_structure_factor():
    """The order trace of crbm_sample_mh after the last cycle equals the
    oracle's plateau structure factor of the final states, and its counts
    trace equals their bond counts."""
    L, J2, h, T = 6, 1.0, 3.0, 0.7
    net = crbm.ARNet(L)
    net.set_params(flatten(ar.init_params(seed=61, scale=INIT_SCALE)))
    acc, tr, od, st = _mh_run(net, L, J2, h, T, 2, 20, n_chains=64, with_order=True)
    for ch in range(64):
        assert tuple(od[-1, ch]) == oracle.order(L, st[ch])
        assert tuple(tr[-1, ch].astype(int)) == oracle.counts(L, st[ch])


def test_full_size_proposals_18x18():
    """The benchmark's proposal batch: 8192 configurations at 18x18.  Sampler
    and scorer log q are identical for all of them; sampled chains (first,
    last, a middle one in a ragged position) match the oracle's log q within
    tolerance and follow the documented uniforms."""
    L, n = 18, 8192
    params = ar.init_params(seed=77, scale=INIT_SCALE)
    net = crbm.ARNet(L)
    net.set_params(flatten(params))
    s, lq = net.sample(n, seed=99, step=5, id=0)
    assert torch.equal(lq, net.logq(s))
    pick = [0, 4097, n - 1]
    sn = s.cpu().numpy()[pick]
    _, c = ar.forward(unflatten(flatten(params), params), sn)
    ref = ar.proposal_logq(c["logit"], sn)
    assert np.all(np.abs(lq.cpu().numpy()[pick] - ref) < LOGQ_TOL_PER_SITE * L * L)
    for k, ch in enumerate(pick):
        ok, _ = decisions_follow_rule(ar, sn[k], c["logit"][k], proposal_uniforms(oracle, L * L, 99, 5, ch, 0))
        assert ok, ch


@pytest.mark.parametrize("L,n,steps", [(6, 40, 3), (18, 17, 2), (6, 8192, 2), (6, 8192, 4), (18, 8192, 4)])
def test_sample_steps_equal_separate_calls(L, n, steps):
    """crbm_ar_sample_steps: batch k of one launch equals a launch of that batch
    alone with step step0 + k, bit for bit (spins and log q), for ragged
    batches and for the launches of two and four 8192-chain MH cycles (16384
    and 32768 proposals: one and two rounds of one wavefront per SIMD)."""
    print(f"case L={L} n={n} steps={steps}", flush=True)
    net = crbm.ARNet(L)
    net.set_params(flatten(ar.init_params(seed=17, scale=INIT_SCALE)))
    s, lq = net.sample_steps(n, steps, seed=0x51, step0=9, id=3)
    for k in range(steps):
        s1, lq1 = net.sample(n, seed=0x51, step=9 + k, id=3)
        assert torch.equal(s[k], s1) and torch.equal(lq[k], lq1), k


def test_mh_cycles_do_not_depend_on_batching():
    """One call of 5 MH cycles (proposals drawn together) equals 5 calls of one
    cycle each: same accepted count, same traces, same final states."""
    L, n = 4, 64

    def run(split):
        net = _trained_net(L, 1.0, 3.0, 0.5, steps=40)
        inst = crbm.Instance(L=L, J1=1.0, J2=1.0, h=3.0, n_chains=n, sched="const", T0=0.5, id=3)
        smp = crbm.Sampler([inst], seed=12, n_sweeps=100)
        tr = torch.empty((5, n, 3), dtype=torch.int32, device="cuda")
        if split:
            acc = sum(crbm.sample_mh(smp, net, 1, 2, trace=tr[k:k + 1]) for k in range(5))
        else:
            acc = crbm.sample_mh(smp, net, 5, 2, trace=tr)
        st, _ = smp.get_state()
        return acc, tr.cpu().numpy(), st.cpu().numpy()

    a1, t1, s1 = run(False)
    a2, t2, s2 = run(True)
    assert a1 == a2 and np.array_equal(t1, t2) and np.array_equal(s1, s2)
    assert a1 > 0


def test_batches_beyond_32_bit_pixel_indices_are_refused():
    """Training and scoring batches of 2^31 pixels or more are refused before
    any buffer is sized or any kernel runs (the pointer is never read)."""
    L = 18
    net = crbm.ARNet(L)
    x = torch.ones((1, L, L), dtype=torch.int8, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    big = (2**31 - 1) // (L * L) + 1
    lib = crbm.lib()
    loss = ct.c_double()
    assert lib.crbm_ar_train_step_cond(net._h, ct.c_void_p(x.data_ptr()), None, big, 1e-3,
                                       ct.byref(loss)) == crbm.CRBM_EINVAL
    assert "2^31" in lib.crbm_last_error().decode()
    assert lib.crbm_ar_grad_cond(net._h, ct.c_void_p(x.data_ptr()), None, big, None, None) == crbm.CRBM_EINVAL
    assert lib.crbm_ar_logq_cond(net._h, ct.c_void_p(x.data_ptr()), None, big,
                                 ct.c_void_p(out.data_ptr())) == crbm.CRBM_EINVAL
    assert torch.isfinite(net.logq(x)).all()  # the handle still works


def test_batched_sampler_and_mh_edge_cases():
    """crbm_ar_sample_steps rejects empty requests; zero MH cycles accept
    nothing and leave the state as it was; a one-chain handle runs."""
    net = crbm.ARNet(6)
    net.set_params(flatten(ar.init_params(seed=3, scale=INIT_SCALE)))
    for n, k in ((0, 2), (4, 0), (-1, 1)):
        with pytest.raises(crbm.CrbmError) as e:
            net.sample_steps(n, k, seed=1)
        assert e.value.code == crbm.CRBM_EINVAL, (n, k)
    inst = crbm.Instance(L=6, J1=1.0, J2=1.0, h=3.0, n_chains=1, sched="const", T0=0.5, id=4)
    smp = crbm.Sampler([inst], seed=2, n_sweeps=50)
    smp.sample(5)
    before, _ = smp.get_state()
    assert crbm.sample_mh(smp, net, 0, 3) == 0
    after, _ = smp.get_state()
    assert torch.equal(before, after)
    tr = torch.empty((3, 1, 3), dtype=torch.int32, device="cuda")
    crbm.sample_mh(smp, net, 3, 1, trace=tr)
    st, _ = smp.get_state()
    assert tuple(tr[-1, 0].cpu().numpy().astype(int)) == oracle.counts(6, st.cpu().numpy().reshape(6, 6))


def _confident_params(seed, bias):
    """Random weights at the test scale with the logit layer's bias shifted,
    so that most sites' logits sit near `bias`: their minority value has a
    probability of a few times 2^-32 (|bias| = 20), below the 2^-24 resolution
    of a 24-bit uniform."""
    params = ar.init_params(seed=seed, scale=INIT_SCALE)
    W, b = params[-1]
    params[-1] = (W, b + bias)
    return params


@pytest.mark.parametrize("bias", [-20.0, 20.0])
def test_scorer_uses_the_integer_law_at_confident_logits(bias):
    """log q of configurations full of minority values under an over-confident
    network is the integer law's, sum log(t / 2^32) with t = 9 or so per site,
    not the sigmoid's (which differs by ~0.02 per such site: 0.7 per 6x6
    configuration, over 10 times the tolerance)."""
    L = 6
    params = _confident_params(91, bias)
    net = crbm.ARNet(L)
    net.set_params(flatten(params))
    s = _rand_spins(16, L, 5)
    s[0] = 1
    s[1] = -1
    got = net.logq(torch.from_numpy(s).cuda()).cpu().numpy()
    _, c = ar.forward(unflatten(flatten(params), params), s)
    ref = ar.proposal_logq(c["logit"], s)
    sig = ar.forward(unflatten(flatten(params), params), s)[0]
    t = ar.minority_threshold(c["logit"])
    assert np.median(t) < 20  # the regime below 2^-24
    assert np.all(np.abs(got - ref) < LOGQ_TOL_PER_SITE * L * L), np.abs(got - ref).max()
    assert np.abs(ref - sig).max() > 10 * LOGQ_TOL_PER_SITE * L * L


def test_confident_proposals_follow_the_integer_rule():
    """Proposals of an over-confident network: every decision follows the
    documented uniform and the integer rule, and sampler log q == scorer log q
    == the oracle's integer law (a sampler still on the old sigmoid rule would
    give log q values off by the sigmoid-vs-integer gap at these logits)."""
    L, n = 6, 64
    params = _confident_params(92, -20.0)
    p64 = unflatten(flatten(params), params)
    net = crbm.ARNet(L)
    net.set_params(flatten(params))
    s, lq = net.sample(n, seed=21, step=4, id=1)
    assert torch.equal(lq, net.logq(s))
    sn = s.cpu().numpy()
    _, c = ar.forward(p64, sn)
    assert np.all(np.abs(lq.cpu().numpy() - ar.proposal_logq(c["logit"], sn)) < 1e-6 * L * L)
    for ch in range(n):
        ok, _ = decisions_follow_rule(ar, sn[ch], c["logit"][ch], proposal_uniforms(oracle, L * L, 21, 4, ch, 1))
        assert ok, ch


def test_mh_keeps_the_exact_law_with_an_overconfident_proposal():
    """1 Gibbs sweep : 1 MH step on 4x4 in the ferromagnetic phase (J2/J1 = 1,
    h = 7, T = 1: the all-up state holds most of the weight) with a proposal
    so confident (logit bias +20) that it proposes all spins up nearly always
    and every minority value at a few times 2^-32: moves are accepted (from
    the all-up state) and E and m stay within 3 SE of exact enumeration."""
    L, J2, h, T = 4, 1.0, 7.0, 1.0
    net = crbm.ARNet(L)
    net.set_params(flatten(_confident_params(93, 20.0)))
    cycles, n_chains = 400, 1024
    acc, t = _mh_run(net, L, J2, h, T, 1, cycles, n_chains, seed=31)
    assert 0 < acc < cycles * n_chains
    t = t[50:]
    J1q, J2q, hq = (oracle.quantise(x) for x in (1.0, J2, h))
    E = (J1q * t[:, :, 1] + J2q * t[:, :, 2] - hq * t[:, :, 0]) / 65536 / 16
    m = t[:, :, 0] / 16
    ex = P.exact_averages(4, J1q / 65536, J2q / 65536, hq / 65536, T)
    for vals, ref in ((E.mean(axis=0), ex["E"]), (m.mean(axis=0), ex["m"])):
        se = vals.std(ddof=1) / math.sqrt(len(vals))
        assert abs(vals.mean() - ref) < 3 * se, (vals.mean(), ref, se)


def test_proposal_frequencies_match_scorer_law_4x4():
    """2^22 proposals at 4x4 against the scorer's law over all 2^16 states: a
    chi-square statistic (expected counts >= 5, the rest pooled) below its
    99.9 % quantile, and the scorer's law sums to 1."""
    from scipy import stats
    L = 4
    params = ar.init_params(seed=94, scale=1.0)
    params = [(W, b + 0.1) for W, b in params]
    net = crbm.ARNet(L)
    net.set_params(flatten(params))
    states = torch.from_numpy(P.all_states(L)).cuda()
    q = torch.exp(net.logq(states)).cpu().numpy()
    assert abs(q.sum() - 1.0) < 1e-9
    weights = torch.tensor([1 << k for k in range(L * L)], dtype=torch.int64, device="cuda")
    counts = torch.zeros(1 << (L * L), dtype=torch.int64, device="cuda")
    n, steps = 16384, 32
    for k in range(8):
        s, _ = net.sample_steps(n, steps, seed=0x77, step0=k * steps, id=5)
        code = ((s.reshape(-1, L * L) > 0).to(torch.int64) * weights).sum(dim=1)
        counts += torch.bincount(code, minlength=1 << (L * L))
    obs = counts.cpu().numpy().astype(np.float64)
    total = obs.sum()
    assert total == 8 * n * steps
    exp = q * total
    # state k of P.all_states has spin j = bit j of k, the same code as above
    big = exp >= 5
    o = np.append(obs[big], obs[~big].sum())
    e = np.append(exp[big], exp[~big].sum())
    chi2 = ((o - e) ** 2 / e).sum()
    assert big.sum() > 500  # many cells tested individually
    assert chi2 < stats.chi2.ppf(0.999, len(o) - 1), (chi2, len(o))
