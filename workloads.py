"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests
and the benchmark.

This module holds no arithmetic of the method: it only draws positions and
charges (and the per-chain sizes of the batched workload) from fixed seeds,
so that the CPU oracle and the GPU library see identical inputs.

Workloads (unit periodic cube, k_e = 1, energies in q^2/a, beta = 1):

* ``small``   -- N = 1000 uniform, q = +1 for i < 500 else -1, depth 3, p 8,
                 displacement uniform in [-0.05, 0.05)^3, 2000 proposals.
* ``medium``  -- N = 10^4 uniform, half +1 / half -1, depth 4, p 12,
                 displacement in [-0.02, 0.02)^3, 10^5 proposals.
* ``rocksalt``-- 46^3 = 97336 ions of a rock-salt lattice at (i+1/2)/46 with
                 q = (-1)^(i+j+k), jittered by N(0, (0.01/46)^2) per
                 coordinate, depth 5, p 12, displacement in
                 [-0.3/46, 0.3/46)^3, 10^6 proposals. Stands in for the
                 jittered NaCl crystal of the paper's experiments (Sec. 5.1).
* ``batched`` -- 256 chains, N_c = 2 round(exp(U(ln 1e3, ln 3e4))/2),
                 uniform, half +1 / half -1, depth round(log8(N_c/8)) (at
                 least 2), p 12, displacement 0.5 N_c^(-1/3), 10^4 steps each.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    pos: np.ndarray          # (N, 3) float64, inside [0, box)
    q: np.ndarray            # (N,) float64
    box: float
    depth: int               # octree depth d: 8^d leaf cells, L = d + 1 levels
    p: int                   # expansion degree
    max_step: float          # displacement half-width per component
    steps: int               # proposals of the workload
    beta: float
    seed: int                # key word 0 of the proposal stream
    chain: int = 0           # key word 1 of the proposal stream
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.q.shape[0])


def _rng(cfg: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=100 + cfg))


def _half_charges(n: int) -> np.ndarray:
    q = np.ones(n)
    q[n // 2:] = -1.0
    return q


def small() -> Workload:
    g = _rng(1)
    pos = g.uniform(0.0, 1.0, size=(1000, 3))
    return Workload("small_n1000_d3_p8", pos, _half_charges(1000), 1.0, 3, 8, 0.05, 2000, 1.0, 1)


def medium() -> Workload:
    g = _rng(2)
    pos = g.uniform(0.0, 1.0, size=(10000, 3))
    return Workload("medium_n10000_d4_p12", pos, _half_charges(10000), 1.0, 4, 12, 0.02, 100000, 1.0, 2)


def rocksalt(side: int = 46, depth: int = 5, p: int = 12, steps: int = 1000000) -> Workload:
    g = _rng(3)
    s = 1.0 / side
    idx = np.stack(np.meshgrid(np.arange(side), np.arange(side), np.arange(side), indexing="ij"), -1)
    idx = idx.reshape(-1, 3)
    q = np.where(idx.sum(1) % 2 == 0, 1.0, -1.0)
    pos = (idx + 0.5) * s + g.normal(0.0, 0.01 * s, size=idx.shape)
    pos = np.mod(pos, 1.0)
    pos[pos >= 1.0] = 0.0
    return Workload(f"rocksalt_n{side**3}_d{depth}_p{p}", pos, q, 1.0, depth, p, 0.3 * s, steps, 1.0, 3)


def batched_sizes(nchains: int = 256):
    """(N_c, depth_c, max_step_c) per chain of the batched workload."""
    g = _rng(4)
    u = g.uniform(math.log(1e3), math.log(3e4), size=nchains)
    out = []
    for v in u:
        n = 2 * int(round(math.exp(v) / 2.0))
        d = max(2, int(round(math.log(n / 8.0, 8))))
        out.append((n, d, 0.5 * n ** (-1.0 / 3.0)))
    return out


def batched_chain(c: int, nchains: int = 256, p: int = 12, steps: int = 10000) -> Workload:
    n, d, step = batched_sizes(nchains)[c]
    g = np.random.Generator(np.random.Philox(key=[104, c]))
    pos = g.uniform(0.0, 1.0, size=(n, 3))
    return Workload(f"batched_chain{c}_n{n}_d{d}_p{p}", pos, _half_charges(n), 1.0, d, p, step,
                    steps, 1.0, 4, chain=c)


def uniform(n: int, depth: int, p: int, max_step: float, seed: int, steps: int = 1000,
            key: int = 0) -> Workload:
    """A generic uniform neutral system for tests (half +1, half -1)."""
    g = np.random.Generator(np.random.Philox(key=[200 + key, n]))
    pos = g.uniform(0.0, 1.0, size=(n, 3))
    return Workload(f"uniform_n{n}_d{depth}_p{p}", pos, _half_charges(n), 1.0, depth, p, max_step,
                    steps, 1.0, seed)


def rocksalt_lattice(side: int):
    """Unjittered rock salt: positions (i+1/2)/side, q = (-1)^(i+j+k)."""
    idx = np.stack(np.meshgrid(np.arange(side), np.arange(side), np.arange(side), indexing="ij"), -1)
    idx = idx.reshape(-1, 3)
    q = np.where(idx.sum(1) % 2 == 0, 1.0, -1.0)
    return (idx + 0.5) / side, q
