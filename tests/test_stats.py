"""tau_int / ESS: the oracle against closed forms, the GPU kernel against the oracle."""
import math

import numpy as np
import pytest

from oracle import stats


def _ar1(phi, n, nc, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((n, nc))
    e = rng.standard_normal((n, nc))
    x[0] = e[0] / math.sqrt(1 - phi * phi)
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    return x


@pytest.mark.parametrize("phi", [0.0, 0.5, 0.9])
def test_ar1_closed_form(phi):
    """For an AR(1) series rho(k) = phi^k and tau_int = (1 + phi)/(1 - phi)."""
    x = _ar1(phi, 4000, 64, 7)
    tau, ess, W, rho = stats.tau_int(x)
    exact = (1 + phi) / (1 - phi)
    assert abs(tau - exact) < 0.06 * exact + 0.05, (tau, exact)
    assert abs(rho[1] - phi) < 0.02
    assert abs(ess - 64 * 4000 / tau) < 1e-6


def test_chains_at_different_levels_count_as_correlated():
    """Chains frozen at different constants (a non-ergodic sampler): rho(k) = 1
    at every lag, the window never closes, tau_int = 1 + 2 max_lag."""
    x = np.ones((300, 8)) * np.arange(8)[None, :]
    tau, ess, W, rho = stats.tau_int(x, max_lag=100)
    assert np.allclose(rho, 1.0)
    assert W == 100 and abs(tau - 201.0) < 1e-9


def test_offsets_enter_through_the_grand_mean():
    """AR(1) chains plus random per-chain offsets d_c: with the grand mean
    removed, rho(k) = (phi^k s2 + v_d) / (s2 + v_d), where s2 = 1 / (1 - phi^2)
    is the AR(1) variance and v_d the offsets' variance about their mean."""
    phi, n, nc = 0.6, 4000, 400
    rng = np.random.default_rng(5)
    d = rng.standard_normal(nc) * 0.5
    x = _ar1(phi, n, nc, 9) + d[None, :]
    s2 = 1 / (1 - phi * phi)
    vd = d.var()
    rho = stats.autocorr(x)
    for k in (1, 2, 5, 20):
        exact = (phi ** k * s2 + vd) / (s2 + vd)
        assert abs(rho[k] - exact) < 0.02, (k, rho[k], exact)


@pytest.mark.gpu
def test_gpu_tau_int_matches_oracle():
    torch = pytest.importorskip("torch")
    import paper_2511_20911_amd as crbm
    rng = np.random.default_rng(3)
    n, nc = 600, 40
    base = _ar1(0.8, n, nc, 11)
    tr = np.zeros((n, nc, 3), np.int32)
    tr[:, :, 0] = np.round(base * 7).astype(np.int32)
    tr[:, :, 1] = rng.integers(-500, 500, (n, nc))
    tr[:, :, 2] = np.round(base * 3).astype(np.int32) + rng.integers(-2, 3, (n, nc))
    w = (-1.5, 1.0, 0.5)
    x = (w[0] * tr[:, :, 0] + w[1] * tr[:, :, 1] + w[2] * tr[:, :, 2]).astype(np.float64)
    for c0, c1, disc in [(0, nc, 0), (5, 33, 100)]:
        ref = stats.tau_int(x[disc:, c0:c1], max_lag=300)
        got = crbm.tau_int(torch.from_numpy(tr).cuda(), w, c0=c0, c1=c1, discard=disc, max_lag=300)
        assert abs(got[0] - ref[0]) < 1e-9 * ref[0]
        assert got[2] == ref[2]
        assert np.allclose(got[3], ref[3][: len(got[3])], rtol=1e-9, atol=1e-12)
