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
