"""Pins of the learned-proposal oracle: exact normalisation, causality,
finite-difference gradients, and the MH target equal to the CRBM marginal."""
import math

import numpy as np
import pytest

import oracle
import physics as P
from oracle import ar


@pytest.mark.parametrize("emulate", [False, True])
def test_normalised_over_all_4x4_states(emulate):
    """sum over all 2^16 configurations of q = 1 (an autoregressive model is
    normalised only if every logit depends on earlier sites alone)."""
    params = ar.init_params(seed=1, scale=1.5)
    states = P.all_states(4)
    lq, _ = ar.forward(params, states, emulate_bf16=emulate)
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


def test_sampling_is_ancestral():
    """Sampled spins follow sigmoid(logit) of the earlier sites (uniforms in)."""
    params = ar.init_params(seed=4)
    rng = np.random.default_rng(2)
    u = rng.random((5, 16))
    s, lq = ar.sample(params, 5, 4, u)
    lq2, c = ar.forward(params, s)
    assert np.allclose(lq, lq2)
    p = 1 / (1 + np.exp(-c["logit"].reshape(5, 16)))
    assert np.array_equal(s.reshape(5, 16) == 1, u < p)


@pytest.mark.parametrize("J2,h,T", [(1.0, 3.0, 1.0), (0.5, 0.0, 0.7)])
def test_mh_target_is_the_crbm_marginal(J2, h, T):
    """log pi from integer counts equals the oracle's CRBM marginal (Eq. (4)
    summed over hidden units) up to one constant, for every 4x4 state."""
    inst = oracle.Instance(4, 1.0, J2, h, "const", T)
    states = P.all_states(4)[::5]
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

def _cond_nonzero(seed, scale=0.3):
    """A conditioning MLP with random (not zero) output weights."""
    c = ar.init_cond(seed=seed)
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
    params = ar.init_params(seed=13, scale=1.0)
    c = _cond_nonzero(14)
    states = P.all_states(4)
    off = np.repeat(ar.cond_bias(c, FEATS)[point][None], states.shape[0], axis=0)
    assert np.abs(off).max() > 0.1  # the offsets are not trivial
    lq, _ = ar.forward(params, states, bias_add=off)
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
