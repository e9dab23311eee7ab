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
