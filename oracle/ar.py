"""Oracle for the learned proposal (test infrastructure only).

A PixelCNN-style masked-convolution autoregressive network over the spins in
raster order, the independent Metropolis-Hastings step that uses it, and the
target distribution both samplers share.  Plain numpy, fp64 arithmetic; the
operands are rounded to bfloat16 at exactly the points where the HIP kernels
round them (matrix-core inputs and stored activations), so kernel and oracle
differ only by fp32 summation order.  Nothing here is shared with the library.

Network (channels C, 12 layers, 3x3 masked kernels, zero padding):
  h0 = sigma (+-1)
  z1 = convA(h0) + b1,           h1 = bf16(relu(z1))
  zl = convB(h_{l-1}) + bl,      hl = bf16(h_{l-1} + relu(zl))     l = 2..11
  logit = convB(h11) + b12
  training loss: -sum_i log sigmoid(sigma_i logit_i)
The proposal draws site i by an integer compare with an exactly known
probability: with t_i = clamp(rint(2^32 sigmoid(-|logit_i|)), 1, 2^31) (the
sigmoid in fp32, as the kernels take the decision) the probability of the
value against the sign of the logit, sigma_i = +1 iff a 32-bit uniform u_i is
below 2^32 - t_i (logit >= 0) or t_i (logit < 0); the proposal's log q sums
log(t_i / 2^32) (minority) or log(1 - t_i / 2^32) over the sites.  It
differs from the sigmoid law by at most half a unit in 2^-32 per site, and it
is the probability with which the proposal was really drawn, which the
Metropolis-Hastings ratio needs.
Mask A taps (dr, dc): (-1,-1) (-1,0) (-1,1) (0,-1) (sites strictly before the
current one in raster order); mask B adds the centre (0,0).  The logit at a
site therefore depends only on earlier sites.

Conditional network: a point x (a few scalar features of the Hamiltonian,
e.g. J2/J1, h/J1 and ln T) shifts every layer's biases by g(x) = W2^T tanh(W1^T x
+ b1), one vector of C values per layer (only channel 0 matters in the logit
layer); a fresh conditional network has W2 = 0 and equals its unconditional
part.

Target of the Gibbs chain (the CRBM marginal with the fixed-point weights):
  log pi(v) = a' M + sum_t c_t n_t(v) + const,  c_t = log cosh(2 w'_t),
n_t = number of type-t bonds with s_a = sig_t s_b, w' = wq / 2^16,
a' = aq / 2^16 (Sec. II.A Eq. (4) with the hidden units summed out).
"""
from __future__ import annotations

import math

import numpy as np

TAPS_A = [(-1, -1), (-1, 0), (-1, 1), (0, -1)]
TAPS_B = TAPS_A + [(0, 0)]
N_LAYERS = 12
COND_FEATURES = 3
COND_HIDDEN = 32


def bf16(x):
    """Round to the nearest bfloat16 (ties to even) via float32, as the kernels do."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def init_params(C=32, seed=0, scale=1.0):
    """Seeded initial parameters (fan-in scaled normal weights, zero biases)."""
    rng = np.random.default_rng(seed)
    P = []
    for l in range(N_LAYERS):
        taps = TAPS_A if l == 0 else TAPS_B
        cin = 1 if l == 0 else C
        cout = 1 if l == N_LAYERS - 1 else C
        std = scale * math.sqrt(2.0 / (len(taps) * cin)) * (0.1 if l == N_LAYERS - 1 else 1.0)
        W = rng.standard_normal((len(taps), cin, cout)) * std
        b = np.zeros(cout)
        P.append((W, b))
    return P


def _conv(x, W, taps):
    """x [B, L, L, Cin], W [T, Cin, Cout] -> [B, L, L, Cout], zero padding."""
    B, L, _, _ = x.shape
    out = np.zeros((B, L, L, W.shape[2]))
    for t, (dr, dc) in enumerate(taps):
        sh = np.zeros_like(x)
        r0, r1 = max(0, -dr), min(L, L - dr)
        c0, c1 = max(0, -dc), min(L, L - dc)
        sh[:, r0:r1, c0:c1, :] = x[:, r0 + dr:r1 + dr, c0 + dc:c1 + dc, :]
        out += sh @ W[t]
    return out


def _conv_t(g, W, taps):
    """Adjoint of _conv with respect to its input."""
    B, L, _, _ = g.shape
    out = np.zeros((B, L, L, W.shape[1]))
    for t, (dr, dc) in enumerate(taps):
        contrib = g @ W[t].T  # [B, L, L, Cin] at the output pixel
        r0, r1 = max(0, -dr), min(L, L - dr)
        c0, c1 = max(0, -dc), min(L, L - dc)
        out[:, r0 + dr:r1 + dr, c0 + dc:c1 + dc, :] += contrib[:, r0:r1, c0:c1, :]
    return out


def _conv_w(x, g, taps):
    """Gradient of sum(g * conv(x, W)) with respect to W: [T, Cin, Cout]."""
    B, L, _, Cin = x.shape
    Cout = g.shape[3]
    dW = np.zeros((len(taps), Cin, Cout))
    for t, (dr, dc) in enumerate(taps):
        sh = np.zeros_like(x)
        r0, r1 = max(0, -dr), min(L, L - dr)
        c0, c1 = max(0, -dc), min(L, L - dc)
        sh[:, r0:r1, c0:c1, :] = x[:, r0 + dr:r1 + dr, c0 + dc:c1 + dc, :]
        dW[t] = sh.reshape(-1, Cin).T @ g.reshape(-1, Cout)
    return dW


def init_cond(C=32, seed=0, H=COND_HIDDEN):
    """Seeded conditioning MLP: W1 [3, H] ~ N(0, 1/3), b1 = 0, W2 = 0 [H, 12, C]."""
    rng = np.random.default_rng(seed)
    return {"W1": rng.standard_normal((COND_FEATURES, H)) / math.sqrt(COND_FEATURES),
            "b1": np.zeros(H), "W2": np.zeros((H, N_LAYERS, C))}


def cond_bias(cond, feats):
    """Bias offsets of points feats [P, 3] -> [P, 12, C]."""
    h = np.tanh(np.asarray(feats, np.float64) @ cond["W1"] + cond["b1"])
    return np.einsum("ph,hlc->plc", h, cond["W2"])


def cond_grad(cond, feats, point_idx, gbias):
    """Gradient of a loss with respect to the MLP, given the loss gradient
    gbias [B, 12, C] with respect to each sample's bias offsets and the
    sample -> point map point_idx [B]."""
    feats = np.asarray(feats, np.float64)
    P = feats.shape[0]
    gp = np.zeros((P,) + gbias.shape[1:])
    np.add.at(gp, np.asarray(point_idx), gbias)  # per point: offsets are shared by its samples
    pre = feats @ cond["W1"] + cond["b1"]
    h = np.tanh(pre)
    dW2 = np.einsum("ph,plc->hlc", h, gp)
    dh = np.einsum("hlc,plc->ph", cond["W2"], gp)
    dpre = dh * (1.0 - h * h)
    return {"W1": feats.T @ dpre, "b1": dpre.sum(axis=0), "W2": dW2}


def forward(params, spins, emulate_bf16=True, bias_add=None):
    """spins [B, L, L] of +-1 -> (sum of log sigmoid(s_i logit_i) [B], the
    training law, and the cache for backward).  bias_add
    [B, 12, C] (optional): per-sample bias offsets of a conditional network."""
    rb = bf16 if emulate_bf16 else (lambda v: np.asarray(v, np.float64))
    s = np.asarray(spins, np.float64)
    h = s[..., None]
    hs, zs = [h], []
    for l in range(N_LAYERS):
        W, b = params[l]
        taps = TAPS_A if l == 0 else TAPS_B
        z = _conv(h, rb(W), taps) + b
        if bias_add is not None:
            z = z + np.asarray(bias_add, np.float64)[:, None, None, l, :z.shape[3]]
        zs.append(z)
        if l == N_LAYERS - 1:
            logit = z[..., 0]
        elif l == 0:
            h = rb(np.maximum(z, 0.0))
        else:
            h = rb(h + np.maximum(z, 0.0))
        if l < N_LAYERS - 1:
            hs.append(h)
    x = s * logit
    logq = -np.logaddexp(0.0, -x).sum(axis=(1, 2))
    return logq, {"hs": hs, "zs": zs, "logit": logit, "spins": s, "rb": rb}


def loss_and_grad(params, spins, emulate_bf16=True, bias_add=None, per_sample_bias=False):
    """Mean negative log-likelihood over the batch and its gradient
    (hand-derived backward, straight through the bf16 roundings).  With
    per_sample_bias, also the gradient with respect to each sample's bias
    offsets [B, 12, C] (zero beyond the logit layer's one channel)."""
    logq, c = forward(params, spins, emulate_bf16, bias_add)
    rb = c["rb"]
    B = spins.shape[0]
    s, logit = c["spins"], c["logit"]
    # d(-log sigmoid(s l))/dl = -s (1 - sigmoid(s l))
    g = -s * (1.0 / (1.0 + np.exp(s * logit))) / B
    grads = [None] * N_LAYERS
    C = params[0][0].shape[2]
    gbias = np.zeros((B, N_LAYERS, C))
    dz = g[..., None]
    for l in range(N_LAYERS - 1, -1, -1):
        W, b = params[l]
        taps = TAPS_A if l == 0 else TAPS_B
        hin = c["hs"][l]
        dzb = rb(dz)
        grads[l] = (_conv_w(hin, dzb, taps), dz.sum(axis=(0, 1, 2)))
        gbias[:, l, :dz.shape[3]] = dz.sum(axis=(1, 2))
        if l == 0:
            break
        dh_in = _conv_t(dzb, rb(W), taps)
        if l < N_LAYERS - 1 and l > 0:
            dh_in = dh_in + dh  # residual path of layer l (l >= 1, not the output layer)
        dh = dh_in
        zprev = c["zs"][l - 1]
        dz = dh * (zprev > 0)
    if per_sample_bias:
        return -logq.mean(), grads, gbias
    return -logq.mean(), grads


def minority_threshold(logit):
    """t = clamp(rint(2^32 sigmoid(-|x|)), 1, 2^31) with the sigmoid in fp32
    (the precision in which the kernels take the decision); uint64 array."""
    x = np.abs(np.asarray(logit, np.float32))
    e = np.exp(-x).astype(np.float32)
    p = (e / (np.float32(1.0) + e)).astype(np.float32)
    t = np.rint(p.astype(np.float64) * 2.0 ** 32)  # p 2^32 is exact: a power-of-two scale
    return np.clip(np.nan_to_num(t, nan=1.0), 1.0, 2.0 ** 31).astype(np.uint64)


def proposal_site_logq(logit, spins):
    """log of the probability with which the proposal draws each site's spin:
    log(t / 2^32) for the minority value, log(1 - t / 2^32) for the sign of the
    logit."""
    x = np.asarray(logit, np.float32)
    t = minority_threshold(x).astype(np.float64) * 2.0 ** -32
    majority = (x >= 0) == (np.asarray(spins) > 0)
    return np.where(majority, np.log1p(-t), np.log(t))


def proposal_logq(logit, spins):
    """log q of configurations [B, L, L] under the proposal's integer rule."""
    return proposal_site_logq(logit, spins).sum(axis=(1, 2))


def up_threshold(logit):
    """sigma = +1 iff u < this: 2^32 - t for logit >= 0, t for logit < 0."""
    x = np.asarray(logit, np.float32)
    t = minority_threshold(x).astype(np.int64)
    return np.where(x >= 0, (1 << 32) - t, t).astype(np.uint64)


def sample(params, n, L, uniforms, emulate_bf16=True, bias_add=None):
    """Ancestral sampling in raster order; uniforms [n, L*L] of 32-bit
    integers: sigma_i = +1 iff u_i < up_threshold(logit_i).  Returns spins
    and their proposal log q."""
    s = np.zeros((n, L, L))
    u = np.asarray(uniforms, np.uint64)
    for i in range(L * L):
        r, c = divmod(i, L)
        _, cache = forward(params, s, emulate_bf16, bias_add)
        x = cache["logit"][:, r, c]
        up = u[:, i] < up_threshold(x)
        s[:, r, c] = np.where(up, 1.0, -1.0)
    _, cache = forward(params, s, emulate_bf16, bias_add)
    return s.astype(np.int8), proposal_logq(cache["logit"], s)


def log_target(counts, wq1, sg1, wq2, sg2, aq, L):
    """log pi (up to a constant) from integer counts (M, B1, B2)."""
    M, B1, B2 = (np.asarray(x, np.int64) for x in counts)
    N = L * L
    n1 = (2 * N - B1) // 2 if sg1 < 0 else (2 * N + B1) // 2
    n2 = (N // 2 - B2) // 2 if sg2 < 0 else (N // 2 + B2) // 2
    c1 = math.log(math.cosh(2.0 * wq1 / 65536.0))
    c2 = math.log(math.cosh(2.0 * wq2 / 65536.0))
    return aq / 65536.0 * M + c1 * n1 + c2 * n2


def mh_accept(logpi_cur, logq_cur, logpi_prop, logq_prop, u):
    """Independent MH: accept iff log u < [log pi' - log pi] + [log q - log q']."""
    log_alpha = (logpi_prop - logpi_cur) + (logq_cur - logq_prop)
    return np.log(u) < log_alpha
