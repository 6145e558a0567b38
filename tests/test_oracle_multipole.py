"""Pins of the oracle's multipole-based variant (Sec. 3.3, Alg. M.1-M.3)
against things other than itself:

* Alg. M.3 (each level's multipoles formed directly from the charges)
  equals the FMM upward pass (P2M on the leaves, then M2M) to rounding,
  because M2M translation is exact at every order <= p;
* after accepted moves, the multipoles maintained by Alg. M.2 equal Alg. M.3
  applied to the new positions;
* dE converges in p to the Ewald oracle (pinned to Madelung and brute force)
  and meets the 1e-5 relative RMS gate at p = 12;
* the multipole and local variants agree to their truncation error;
* the total energy converges to the Ewald energy;
* a null move costs nothing, and the run follows the Metropolis rule.
"""
import numpy as np
import pytest

import oracle as O


def _system(n=200, seed=5):
    g = np.random.default_rng(seed)
    pos = g.uniform(0, 1, (n, 3))
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    return pos, q


def _moves(pos, count, step, seed):
    g = np.random.default_rng(seed)
    ks = g.integers(0, len(pos), count)
    return [(int(k), pos[k] + g.uniform(-step, step, 3)) for k in ks]


def _max_rel(a, b):
    scale = np.abs(b).max()
    return np.abs(a - b).max() / scale if scale > 0 else np.abs(a).max()


@pytest.mark.parametrize("depth", [2, 3])
def test_direct_multipoles_equal_upward_pass(depth):
    pos, q = _system(150, 3)
    a = O.Multilevel(pos, q, 1.0, depth, 8, setup="multipole")
    b = O.Multilevel(pos, q, 1.0, depth, 8, setup="multipole_upward")
    for level in range(2, depth + 2):
        for cell in range(8 ** (level - 1)):
            assert _max_rel(a.multipole(level, cell), b.multipole(level, cell)) < 1e-13


def test_maintained_multipoles_equal_fresh_ones_after_accepts():
    pos, q = _system(120, 4)
    m = O.Multilevel(pos, q, 1.0, 2, 8, setup="multipole")
    for k, r in _moves(pos, 12, 0.2, 6):
        m.accept(k, r)
    fresh = O.Multilevel(m.positions(), q, 1.0, 2, 8, setup="multipole")
    for level in (2, 3):
        for cell in range(8 ** (level - 1)):
            assert _max_rel(m.multipole(level, cell), fresh.multipole(level, cell)) < 1e-12
    assert np.allclose(m.K(), fresh.K(), rtol=0, atol=1e-12 * np.abs(fresh.K()).max())


@pytest.fixture(scope="module")
def ewald_ref():
    pos, q = _system()
    e = O.Ewald(pos, q, 1.0)
    mv = _moves(pos, 16, 0.05, 9)
    return pos, q, mv, np.array([e.propose(k, r) for k, r in mv]), e.energy()


@pytest.mark.parametrize("p,bound", [(4, 5e-3), (8, 3e-4), (12, 1e-5)])
def test_dE_converges_to_ewald(ewald_ref, p, bound):
    pos, q, mv, ref, _ = ewald_ref
    m = O.Multilevel(pos, q, 1.0, 2, p, setup="multipole")
    de = np.array([m.propose(k, r) for k, r in mv])
    rel = np.sqrt(np.mean((de - ref) ** 2)) / np.sqrt(np.mean(ref ** 2))
    assert rel < bound


def test_multipole_and_local_variants_agree_to_truncation(ewald_ref):
    pos, q, mv, ref, u_ewald = ewald_ref
    a = O.Multilevel(pos, q, 1.0, 2, 12, setup="multipole")
    b = O.Multilevel(pos, q, 1.0, 2, 12)
    da = np.array([a.propose(k, r) for k, r in mv])
    db = np.array([b.propose(k, r) for k, r in mv])
    rms = np.sqrt(np.mean(ref ** 2))
    assert np.abs(da - db).max() < 1e-4 * rms
    # both energies approach the Ewald energy
    assert a.energy() == pytest.approx(u_ewald, rel=1e-5)
    assert b.energy() == pytest.approx(u_ewald, rel=1e-5)


def test_null_move_and_metropolis_rule():
    pos, q = _system(100, 7)
    m = O.Multilevel(pos, q, 1.0, 2, 6, setup="multipole")
    for k in (0, 37, 99):
        assert abs(m.propose(k, pos[k])) < 1e-12
    tr = m.run(seed=3, chain=0, t0=0, nsteps=40, beta=2.0, max_step=0.05)
    assert np.array_equal(tr["acc"], tr["u"] < np.exp(-2.0 * tr["dE"]))
    assert 0 < tr["acc"].sum() < 40
