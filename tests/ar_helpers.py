"""Conversion between the oracle's parameter list and the flat parameter
layout of the C ABI (per layer: weights [taps][cin][cout], then bias)."""
import numpy as np


def flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params]).astype(np.float32)


def unflatten(flat, like):
    out, off = [], 0
    for W, b in like:
        nW, nb = W.size, b.size
        out.append((np.asarray(flat[off:off + nW], np.float64).reshape(W.shape),
                    np.asarray(flat[off + nW:off + nW + nb], np.float64)))
        off += nW + nb
    return out


def proposal_uniforms(oracle, n_sites, seed, step, chain, ident):
    """The 32-bit uniforms of one proposal's sites: word 0 of Philox with
    counter (site, step, chain, id << 3 | 6) and key (seed_lo, seed_hi)."""
    key = [seed & 0xffffffff, seed >> 32]
    return np.array([int(oracle.philox([i, step, chain, (ident << 3) | 6], key)[0]) for i in range(n_sites)],
                    np.uint64)


def decisions_follow_rule(ar, spins, logits, u, near=1e-3):
    """Spins of one proposal against the integer rule (+1 iff u < up_threshold)
    evaluated on the oracle's logits.  The oracle's logits differ from the
    kernel's in the last bits, so a site whose uniform lies within `near`
    (as a probability) of the threshold may go either way.  Returns (all
    decisions consistent, share of such near sites)."""
    x = np.asarray(logits, np.float64).reshape(-1)
    tu = ar.up_threshold(x).astype(np.float64)
    up = np.asarray(u, np.float64) < tu
    close = np.abs(np.asarray(u, np.float64) - tu) < near * 2.0 ** 32
    ok = (np.asarray(spins).reshape(-1) == 1) == up
    return bool(np.all(ok | close)), float(close.mean())


# Gradient blocks (each layer's weights, each layer's biases) are compared
# element by element.  Kernel and oracle round the same values to bf16 (the
# stored activations, the weights, the gradient operands of the matrix
# cores); where a pre-rounding fp32 sum of the kernel and the fp64 sum of the
# oracle fall on two sides of a bf16 rounding boundary, the operands differ
# by one bf16 step, 2^-8 = 3.9e-3 relative, and that difference is summed
# into a few gradient elements.  The bound allows 2.5 such steps of the
# block's largest element; measured at 18x18: at most 5e-3 of it, relative
# L2 at most 1.8e-3 per block.
GRAD_ATOL_OF_BLOCK_MAX = 1e-2
GRAD_REL_L2 = 5e-3


def assert_grad_blocks(g, ref_grads, like):
    """Compare a flat gradient with the oracle's per-layer blocks."""
    from oracle import ar
    got = unflatten(g, like)
    for l in range(ar.N_LAYERS):
        for k, kind in enumerate(("weights", "bias")):
            a, b = got[l][k], ref_grads[l][k]
            scale = np.abs(b).max()
            np.testing.assert_allclose(a, b, rtol=0, atol=GRAD_ATOL_OF_BLOCK_MAX * scale,
                                       err_msg=f"layer {l} {kind}")
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            assert rel < GRAD_REL_L2, (l, kind, rel)


def documented_batch(oracle, data, batch, seed, step, augment=True, points=None):
    """The minibatch of training step `step` as crbm_ar_batch documents it,
    written out on the host: configuration b is data[idx_b], idx_b =
    floor(u n / 2^64) with u = out[0] 2^32 + out[1] of Philox (ctr = (b, step,
    0, 7), key = seed); with augment, rolled by (2 (out[2] mod L/2),
    2 ((out[3] >> 1) mod L/2)) along (rows, columns), then transposed if out[3]
    is odd.  Returns (configurations, points, indices)."""
    n, L = data.shape[0], data.shape[1]
    key = [seed & 0xffffffff, seed >> 32]
    out = np.empty((batch, L, L), np.int8)
    pts = np.zeros(batch, np.int32)
    idx = np.zeros(batch, np.int64)
    for b in range(batch):
        w = [int(x) for x in oracle.philox([b, step, 0, 7], key)]
        u = (w[0] << 32) | w[1]
        i = (u * n) >> 64
        x = data[i]
        if augment:
            x = np.roll(x, (2 * (w[2] % (L // 2)), 2 * ((w[3] >> 1) % (L // 2))), axis=(0, 1))
            if w[3] & 1:
                x = x.T
        out[b] = x
        idx[b] = i
        pts[b] = 0 if points is None else points[i]
    return out, pts, idx
