"""Shared test helpers (no arithmetic of the method)."""
import numpy as np

import oracle as O


def real_layout(c, p):
    """complex full-storage coefficients -> the library's real layout"""
    out = np.zeros((p + 1) ** 2)
    for n in range(p + 1):
        out[O.idx(n, 0)] = c[O.idx(n, 0)].real
        for m in range(1, n + 1):
            out[O.idx(n, m)] = c[O.idx(n, m)].real
            out[O.idx(n, -m)] = c[O.idx(n, m)].imag
    return out


def oracle_stream(wl, steps, t0=0, chain=None):
    """(idx, new position (absolute, before wrap), u) of the Philox stream"""
    ch = wl.chain if chain is None else chain
    out = []
    for t in range(t0, t0 + steps):
        i, d, u = O.draw(wl.seed, ch, t, wl.n, wl.max_step)
        out.append((i, d, u))
    return out


def dE_close(a, b, scale, rel=1e-10):
    a, b = np.asarray(a), np.asarray(b)
    tol = rel * np.maximum(np.abs(b), scale)
    return np.abs(a - b) <= tol
