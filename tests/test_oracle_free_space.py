"""Pins of the oracle under free-space boundary conditions (Sec. 3.4)
against the plain Coulomb sum, which is exact here (no images):

* dE converges in p to q sum_j q_j (1/|r' - r_j| - 1/|r - r_j|) for the M2L
  setup, the direct P2L setup (Alg. L.3) and the multipole variant
  (Alg. M.1-M.3);
* with depth 1 every cell is in the near region (the interaction lists of
  levels 1 and 2 are empty), so dE equals the direct sum to rounding;
* the total energy converges to the O(N^2) pair sum;
* a move out of the box has dE = +inf and is never accepted.
"""
import numpy as np
import pytest

import oracle as O


def _system(n=300, seed=3):
    g = np.random.default_rng(seed)
    pos = g.uniform(0, 1, (n, 3))
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    return pos, q


def _direct_dE(pos, q, k, rn):
    others = np.delete(np.arange(len(q)), k)
    return q[k] * np.sum(q[others] * (1.0 / np.linalg.norm(rn - pos[others], axis=1)
                                      - 1.0 / np.linalg.norm(pos[k] - pos[others], axis=1)))


def _moves(pos, count, step, seed):
    g = np.random.default_rng(seed)
    out = []
    for k in g.integers(0, len(pos), 3 * count):
        r = pos[k] + g.uniform(-step, step, 3)
        if (r >= 0).all() and (r < 1).all():
            out.append((int(k), r))
    return out[:count]


@pytest.fixture(scope="module")
def direct_ref():
    pos, q = _system()
    mv = _moves(pos, 16, 0.05, 4)
    return pos, q, mv, np.array([_direct_dE(pos, q, k, r) for k, r in mv])


@pytest.mark.parametrize("setup", ["fmm", "direct", "multipole"])
@pytest.mark.parametrize("p,bound", [(4, 1.5e-2), (8, 4e-4), (12, 1e-5)])
def test_dE_converges_to_direct_sum(direct_ref, setup, p, bound):
    pos, q, mv, ref = direct_ref
    m = O.Multilevel(pos, q, 1.0, 3, p, setup=setup, free_space=True)
    de = np.array([m.propose(k, r) for k, r in mv])
    assert np.sqrt(np.mean((de - ref) ** 2)) / np.sqrt(np.mean(ref ** 2)) < bound


def test_depth_one_is_all_near_field(direct_ref):
    pos, q, mv, ref = direct_ref
    for setup in ("fmm", "multipole"):
        m = O.Multilevel(pos, q, 1.0, 1, 4, setup=setup, free_space=True)
        de = np.array([m.propose(k, r) for k, r in mv])
        assert np.abs(de - ref).max() < 1e-11 * np.abs(ref).max()


def test_energy_converges_to_pair_sum():
    pos, q = _system(250, 5)
    d = np.linalg.norm(pos[:, None] - pos[None], axis=2)
    iu = np.triu_indices(len(q), 1)
    u_ref = np.sum((q[:, None] * q[None] / np.where(d > 0, d, np.inf))[iu])
    for setup in ("fmm", "multipole"):
        m = O.Multilevel(pos, q, 1.0, 3, 12, setup=setup, free_space=True)
        assert m.energy() == pytest.approx(u_ref, rel=1e-5)


def test_moves_out_of_the_box_are_rejected():
    pos, q = _system(120, 6)
    m = O.Multilevel(pos, q, 1.0, 2, 6, free_space=True)
    assert m.propose(0, np.array([1.05, 0.5, 0.5])) == np.inf
    assert m.propose(1, np.array([0.5, -1e-9, 0.5])) == np.inf
    tr = m.run(seed=5, chain=0, t0=0, nsteps=200, beta=1.0, max_step=0.3)
    out = ((tr["newpos"] < 0) | (tr["newpos"] >= 1)).any(axis=1)
    assert out.sum() > 10
    assert not tr["acc"][out].any() and np.isinf(tr["dE"][out]).all()
    assert tr["acc"][~out].any()
    assert ((m.positions() >= 0) & (m.positions() < 1)).all()
