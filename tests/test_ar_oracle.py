"""Pins of the learned-proposal oracle: exact normalisation, causality,
finite-difference gradients, the bf16 rounding against torch's, the
bf16-emulating backward against autograd, the proposal's integer law, and the
MH target equal to the CRBM marginal."""
import math

import numpy as np
import pytest

import oracle
import physics as P
from oracle import ar


def _forward_all(params, states, chunk=2048, **kw):
    """The oracle's forward pass over many states, a chunk of states at a time
    (samples are independent; small chunks keep the temporaries in reused
    memory).  Returns (sigmoid-law log q, logits)."""
    lq, lg = [], []
    for k in range(0, states.shape[0], chunk):
        extra = {key: (v[k:k + chunk] if key == "bias_add" else v) for key, v in kw.items()}
        a, c = ar.forward(params, states[k:k + chunk], **extra)
        lq.append(a)
        lg.append(c["logit"])
    return np.concatenate(lq), np.concatenate(lg)


@pytest.mark.parametrize("emulate", [False, True])
def test_normalised_over_all_4x4_states(emulate):
    """sum over all 2^16 configurations of q = 1 (an autoregressive model is
    normalised only if every logit depends on earlier sites alone)."""
    params = ar.init_params(C=8, seed=1, scale=1.5)  # normalisation is a property of the masks, not the width
    states = P.all_states(4)
    lq, _ = _forward_all(params, states, emulate_bf16=emulate)
    assert abs(np.logaddexp.reduce(lq)) < 1e-9


def test_causality():
    params = ar.init_params(seed=2)
    rng = np.random.default_rng(0)
    s = (2 * rng.integers(0, 2, (1, 6, 6)) - 1).astype(np.int8)
    _, c0 = ar.forward(params, s)
    for j in (0, 7, 20, 35):
        t = s.copy()
        t.reshape(-1)[j] *= -1
        _, c1 = ar.forward(params, t)
        a, b = c0["logit"].reshape(-1), c1["logit"].reshape(-1)
        assert np.array_equal(a[: j + 1], b[: j + 1]), j


def test_gradient_matches_finite_differences():
    params = ar.init_params(seed=3, scale=1.2)
    rng = np.random.default_rng(1)
    # non-zero biases: with zero bias the first site's layer-1 pre-activation is
    # exactly 0 (all its taps are padding), a ReLU kink where differences fail
    params = [(W, rng.normal(scale=0.3, size=b.shape)) for W, b in params]
    s = (2 * rng.integers(0, 2, (3, 4, 4)) - 1).astype(np.int8)
    _, grads = ar.loss_and_grad(params, s, emulate_bf16=False)
    eps = 1e-6
    for (l, kind, idx) in [(0, 0, (0, 0, 3)), (0, 1, (5,)), (3, 0, (4, 7, 2)), (3, 1, (11,)), (11, 0, (4, 9, 0)),
                           (11, 1, (0,)), (6, 0, (0, 31, 31)), (10, 0, (2, 1, 30))]:
        def f(delta):
            p2 = [(W.copy(), b.copy()) for W, b in params]
            arr = p2[l][kind]
            arr[idx] += delta
            return ar.loss_and_grad(p2, s, emulate_bf16=False)[0]
        fd = (f(eps) - f(-eps)) / (2 * eps)
        an = grads[l][kind][idx]
        assert abs(fd - an) < 1e-6 + 1e-5 * abs(fd), (l, kind, idx, fd, an)


def test_bf16_rounding_equals_torch():
    """The oracle's bf16 rounding (round to nearest, ties to even, through
    float32) equals torch's float32 -> bfloat16 conversion on random values,
    exact ties in both directions, subnormals, signed zeros, values that round
    to infinity and the largest finite ones."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(11)
    bits = rng.integers(0, 1 << 32, 200000, dtype=np.uint64).astype(np.uint32)
    special = []
    for hi in (0x0000, 0x0001, 0x0080, 0x3F80, 0x3F81, 0x7F7F, 0x8001, 0xBF80, 0xFF7F):
        for lo in (0x0000, 0x0001, 0x7FFF, 0x8000, 0x8001, 0xFFFF):
            special.append((hi << 16) | lo)
    bits = np.concatenate([bits, np.array(special, np.uint32)])
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).to(torch.float64).numpy()
    got = ar.bf16(x)
    same = (got == ref) | (np.isnan(got) & np.isnan(ref))
    assert same.all(), x[~same][:5]
    assert np.array_equal(np.signbit(got), np.signbit(ref))
    # the pin has teeth: truncation or ties away from zero would differ
    tie = np.array([np.uint32(0x3F808000)], np.uint32).view(np.float32)
    assert ar.bf16(tie)[0] == 1.0 and ar.bf16(np.nextafter(tie, np.float32(2)))[0] > 1.0


def _torch_loss(params, spins, emulate):
    """Mean negative log-likelihood written with torch modules (masked 3x3
    convolutions via conv2d, ReLU, residuals), so that autograd derives the
    backward independently of the oracle's hand-written one.  With emulate,
    the same bf16 rounding points as the kernels: weights and stored
    activations rounded in the forward pass (straight through), and the
    gradient reaching each convolution's output rounded before it is used for
    that convolution's weight and input gradients."""
    import torch

    def rnd(v):
        return v.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    class ST(torch.autograd.Function):
        @staticmethod
        def forward(ctx, v):
            return rnd(v)

        @staticmethod
        def backward(ctx, g):
            return g

    class GR(torch.autograd.Function):
        @staticmethod
        def forward(ctx, v):
            return v.clone()

        @staticmethod
        def backward(ctx, g):
            return rnd(g)

    st = ST.apply if emulate else (lambda v: v)
    gr = GR.apply if emulate else (lambda v: v)
    s = torch.from_numpy(np.asarray(spins, np.float64))
    h = s[:, None]
    ts = []
    for l, (W, b) in enumerate(params):
        taps = ar.TAPS_A if l == 0 else ar.TAPS_B
        Wt = torch.tensor(W, dtype=torch.float64, requires_grad=True)
        bt = torch.tensor(b, dtype=torch.float64, requires_grad=True)
        ts.append((Wt, bt))
        K = torch.zeros((W.shape[2], W.shape[1], 3, 3), dtype=torch.float64)
        Wr = st(Wt)
        for k, (dr, dc) in enumerate(taps):
            K[:, :, dr + 1, dc + 1] = Wr[k].T
        z = gr(torch.nn.functional.conv2d(h, K, padding=1)) + bt[None, :, None, None]
        if l == len(params) - 1:
            logit = z[:, 0]
        elif l == 0:
            h = st(torch.relu(z))
        else:
            h = st(h + torch.relu(z))
    loss = -torch.nn.functional.logsigmoid(s * logit).sum(dim=(1, 2)).mean()
    loss.backward()
    return float(loss.detach()), [(W.grad.numpy(), b.grad.numpy()) for W, b in ts]


@pytest.mark.parametrize("emulate", [False, True])
def test_backward_equals_autograd(emulate):
    """The hand-derived backward (both with and without the kernels' bf16
    rounding points) equals autograd through a torch formulation of the same
    network, per layer, for weights and biases separately."""
    pytest.importorskip("torch")
    params = ar.init_params(seed=21, scale=1.0)
    rng = np.random.default_rng(12)
    params = [(W, rng.normal(scale=0.1, size=b.shape)) for W, b in params]
    s = (2 * rng.integers(0, 2, (6, 6, 6)) - 1).astype(np.int8)
    loss, grads = ar.loss_and_grad(params, s, emulate_bf16=emulate)
    tloss, tgrads = _torch_loss(params, s, emulate)
    assert abs(loss - tloss) < 1e-10 * abs(loss)
    for l in range(ar.N_LAYERS):
        for k in range(2):
            ref = tgrads[l][k]
            np.testing.assert_allclose(grads[l][k], ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max(),
                                       err_msg=f"layer {l} {'bias' if k else 'weights'}")


def test_emulated_backward_within_the_bf16_bound():
    """The bf16-emulating gradient differs from the exact one by rounding
    only: each of the about 3 roundings per layer on a gradient's path moves
    it by at most 2^-9 relative, so over 12 layers the relative difference of
    every layer's gradient stays below 36 * 2^-9 = 0.07 (in practice ~0.01);
    a wrong term would be O(1)."""
    params = ar.init_params(seed=22, scale=0.7)
    rng = np.random.default_rng(13)
    params = [(W, rng.normal(scale=0.1, size=b.shape)) for W, b in params]
    s = (2 * rng.integers(0, 2, (8, 6, 6)) - 1).astype(np.int8)
    _, ge = ar.loss_and_grad(params, s, emulate_bf16=True)
    _, gp = ar.loss_and_grad(params, s, emulate_bf16=False)
    for l in range(ar.N_LAYERS):
        for k in range(2):
            rel = np.linalg.norm(ge[l][k] - gp[l][k]) / np.linalg.norm(gp[l][k])
            assert rel < 36 * 2.0 ** -9, (l, k, rel)


def test_sampling_is_ancestral():
    """Sampled spins follow the integer rule on the logits of the earlier
    sites (uniforms in): +1 iff u < 2^32 - t (logit >= 0) or u < t (logit <
    0); the returned log q is the proposal law of those spins."""
    params = ar.init_params(seed=4, scale=2.0)
    rng = np.random.default_rng(2)
    u = rng.integers(0, 1 << 32, (5, 16), dtype=np.uint64)
    u[:, ::3] = rng.integers(0, 1 << 22, (5, 6), dtype=np.uint64)  # minority draws at confident negative logits
    u[:, 1::3] = (1 << 32) - 1 - rng.integers(0, 1 << 22, (5, 5), dtype=np.uint64)  # and at positive ones
    s, lq = ar.sample(params, 5, 4, u)
    _, c = ar.forward(params, s)
    x = c["logit"].reshape(5, 16)
    t = ar.minority_threshold(x)
    up = np.where(x >= 0, u < (1 << 32) - t, u < t)
    assert np.array_equal(s.reshape(5, 16) == 1, up)
    minority = up != (x >= 0)
    assert minority.any() and (~minority).any()
    assert np.allclose(lq, ar.proposal_logq(c["logit"], s), rtol=0, atol=1e-12)


def test_minority_threshold_pins():
    """t(x) = clamp(rint(2^32 sigmoid(-|x|)), 1, 2^31): 2^31 at x = 0 (a fair
    coin), even in x, non-increasing in |x|, within half a unit plus the fp32
    sigmoid's error (a few ulp) of 2^32 sigmoid(-|x|) from fp64, and at least 1
    however large |x| is, so the realised minority probability is t / 2^32,
    never 0 and never below 2^-32."""
    assert int(ar.minority_threshold(0.0)) == 1 << 31
    assert int(ar.minority_threshold(-0.0)) == 1 << 31
    assert int(ar.minority_threshold(np.float32(1e30))) == 1
    assert int(ar.minority_threshold(np.inf)) == 1
    assert int(ar.minority_threshold(np.nan)) == 1
    x = np.concatenate([np.linspace(0, 30, 30001), [15.5, 20.0, 22.18, 25.0]]).astype(np.float32)
    t = ar.minority_threshold(x).astype(np.float64)
    assert np.array_equal(t, ar.minority_threshold(-x).astype(np.float64))
    assert np.all(np.diff(t[:30001]) <= 0)
    exact = 2.0 ** 32 / (1.0 + np.exp(x.astype(np.float64)))
    assert np.all(np.abs(t - np.maximum(exact, 1.0)) <= 0.5 + 4e-7 * exact + 1e-9)
    # at |x| = 20 the sigmoid rule of a 24-bit uniform could not represent
    # e^-20 (2.06e-9 < 2^-24); the integer rule gives 9 / 2^32 = 2.10e-9
    assert int(ar.minority_threshold(np.float32(20.0))) == 9


@pytest.mark.parametrize("scale,bias", [(1.5, 0.0), (3.0, 18.0)])
def test_proposal_law_normalised_over_all_4x4_states(scale, bias):
    """The proposal law sums to 1 over all 2^16 states, also for a network so
    confident (logit bias 18) that the minority values at many sites have
    probabilities of a few times 2^-32."""
    params = ar.init_params(C=8, seed=1, scale=scale)
    params[-1] = (params[-1][0], params[-1][1] + bias)
    states = P.all_states(4)
    _, logit = _forward_all(params, states)
    lq = ar.proposal_logq(logit, states)
    if bias:
        assert (ar.minority_threshold(logit) < 1000).mean() > 0.5
    assert abs(np.logaddexp.reduce(lq)) < 1e-9


def test_proposal_frequencies_match_q_3x3():
    """Empirical frequencies of 20000 ancestral draws on 3x3 lattices (512
    states) against the proposal law: a chi-square statistic (states with
    expected count >= 5 pooled) within its 99.9 % quantile."""
    from scipy import stats
    params = ar.init_params(C=8, seed=6, scale=1.3)
    params = [(W, b + 0.2) for W, b in params]
    n, L = 20000, 3
    rng = np.random.default_rng(9)
    u = rng.integers(0, 1 << 32, (n, L * L), dtype=np.uint64)
    parts = [ar.sample(params, 1000, L, u[k:k + 1000]) for k in range(0, n, 1000)]
    s = np.concatenate([p[0] for p in parts])
    lq = np.concatenate([p[1] for p in parts])
    states = P.all_states(3)
    _, c = ar.forward(params, states)
    q = np.exp(ar.proposal_logq(c["logit"], states))
    assert abs(q.sum() - 1.0) < 1e-9
    code = lambda x: ((x.reshape(x.shape[0], -1) > 0).astype(np.int64) << np.arange(L * L)).sum(axis=1)
    obs = np.bincount(code(s), minlength=1 << (L * L)).astype(np.float64)
    exp = np.zeros_like(obs)
    exp[code(states)] = q * n
    big = exp >= 5
    o = np.append(obs[big], obs[~big].sum())
    e = np.append(exp[big], exp[~big].sum())
    chi2 = ((o - e) ** 2 / e).sum()
    assert chi2 < stats.chi2.ppf(0.999, len(o) - 1), (chi2, len(o))
    # each draw's returned log q is the law's value for its state
    assert np.allclose(lq, np.log(exp[code(s)] / n), rtol=0, atol=1e-9)


@pytest.mark.parametrize("J2,h,T", [(1.0, 3.0, 1.0), (0.5, 0.0, 0.7)])
def test_mh_target_is_the_crbm_marginal(J2, h, T):
    """log pi from integer counts equals the oracle's CRBM marginal (Eq. (4)
    summed over hidden units) up to one constant, for every 4x4 state."""
    inst = oracle.Instance(4, 1.0, J2, h, "const", T)
    states = P.all_states(4)
    wq1, sg1 = oracle.bond_weight(oracle.quantise(1.0), T)
    wq2, sg2 = oracle.bond_weight(oracle.quantise(J2), T)
    aq = oracle.visible_bias(oracle.quantise(h), T)
    counts = np.array([oracle.counts(4, s) for s in states]).T
    lt = ar.log_target(counts, wq1, sg1, wq2, sg2, aq, 4)
    lm = np.array([oracle.log_marginal(inst, 1, 0, s) for s in states])
    d = lt - lm
    assert d.max() - d.min() < 1e-9


def test_mh_with_exact_proposal_accepts_everything():
    """If q is the target itself, log alpha = 0 and every move is accepted."""
    rng = np.random.default_rng(5)
    lp_cur, lp_prop = rng.normal(size=100), rng.normal(size=100)
    acc = ar.mh_accept(lp_cur, lp_cur, lp_prop, lp_prop, rng.random(100))
    assert acc.all()


# ---------------------------------------------------------------- conditional network

def _cond_nonzero(seed, scale=0.3, C=32):
    """A conditioning MLP with random (not zero) output weights."""
    c = ar.init_cond(C=C, seed=seed)
    c["b1"] = np.random.default_rng(seed + 1).standard_normal(c["b1"].shape) * 0.2
    c["W2"] = np.random.default_rng(seed + 2).standard_normal(c["W2"].shape) * scale
    return c


FEATS = np.array([[1.0, 0.0, math.log(0.4)], [0.5, 1.2, math.log(0.2)], [2.0, -0.5, 0.0]])


def test_fresh_conditional_network_is_the_unconditional_one():
    """W2 = 0 at initialisation: every point's offsets vanish."""
    params = ar.init_params(seed=11, scale=0.7)
    c = ar.init_cond(seed=12)
    s = (2 * np.random.default_rng(2).integers(0, 2, (4, 6, 6)) - 1).astype(np.int8)
    off = ar.cond_bias(c, FEATS)[[0, 1, 2, 1]]
    assert np.all(off == 0.0)
    lq0, _ = ar.forward(params, s)
    lq1, _ = ar.forward(params, s, bias_add=off)
    assert np.array_equal(lq0, lq1)


@pytest.mark.parametrize("point", [1])
def test_conditional_normalised_per_point_4x4(point):
    """For every point, q(. | x) sums to 1 over all 2^16 states."""
    params = ar.init_params(C=8, seed=13, scale=1.0)
    c = _cond_nonzero(14, C=8)
    states = P.all_states(4)
    off = np.repeat(ar.cond_bias(c, FEATS)[point][None], states.shape[0], axis=0)
    assert np.abs(off).max() > 0.1  # the offsets are not trivial
    lq, _ = _forward_all(params, states, bias_add=off)
    assert abs(np.logaddexp.reduce(lq)) < 1e-9


def test_constant_offset_is_a_base_bias_shift():
    """The same offsets for every sample equal adding them to the base biases
    (the logit layer uses channel 0 only)."""
    params = ar.init_params(seed=15, scale=0.8)
    rng = np.random.default_rng(3)
    off = rng.standard_normal((ar.N_LAYERS, 32)) * 0.3
    shifted = [(W, b + off[l, :b.size]) for l, (W, b) in enumerate(params)]
    s = (2 * rng.integers(0, 2, (3, 6, 6)) - 1).astype(np.int8)
    lq0, _ = ar.forward(params, s, bias_add=np.repeat(off[None], 3, axis=0))
    lq1, _ = ar.forward(shifted, s)
    assert np.allclose(lq0, lq1, rtol=0, atol=1e-12)


def test_conditional_gradient_matches_finite_differences():
    """d loss / d (W1, b1, W2) from the per-sample bias gradients and the MLP
    backward against central differences of the loss (no bf16 rounding, so
    the loss is smooth)."""
    params = ar.init_params(seed=16, scale=1.0)
    params = [(W, b + 0.05) for W, b in params]  # keep pre-activations off the ReLU kink
    c = _cond_nonzero(17, scale=0.2)
    rng = np.random.default_rng(4)
    s = (2 * rng.integers(0, 2, (5, 4, 4)) - 1).astype(np.int8)
    idx = np.array([0, 2, 1, 2, 0])

    def loss_of(cc):
        off = ar.cond_bias(cc, FEATS)[idx]
        return ar.loss_and_grad(params, s, emulate_bf16=False, bias_add=off)[0]

    _, _, gb = ar.loss_and_grad(params, s, emulate_bf16=False, bias_add=ar.cond_bias(c, FEATS)[idx],
                                per_sample_bias=True)
    g = ar.cond_grad(c, FEATS, idx, gb)
    h = 1e-6
    for name, picks in (("W1", [(0, 3), (2, 17)]), ("b1", [(5,), (30,)]), ("W2", [(1, 0, 4), (7, 11, 0), (9, 5, 31)])):
        for ix in picks:
            cp = {k: v.copy() for k, v in c.items()}
            cm = {k: v.copy() for k, v in c.items()}
            cp[name][ix] += h
            cm[name][ix] -= h
            fd = (loss_of(cp) - loss_of(cm)) / (2 * h)
            assert abs(fd - g[name][ix]) < 1e-6 + 1e-5 * abs(fd), (name, ix, fd, g[name][ix])
    # the logit layer's channels 1..31 carry no gradient
    assert np.all(g["W2"][:, ar.N_LAYERS - 1, 1:] == 0.0)
