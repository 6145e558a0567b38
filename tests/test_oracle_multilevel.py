"""Pins of the plain multilevel oracle (O2) against things other than
itself: convergence in p to the Ewald oracle (which is pinned to Madelung
and brute force), the rock-salt Madelung energy, agreement of the two
initialisations, antisymmetry of a move and its reverse, energy
bookkeeping, wrap invariance, and the lazy (sampled) mode."""
import numpy as np
import pytest

import oracle as O
import workloads

MADELUNG = 1.7475645946331822


def _system(n=200, seed=5):
    g = np.random.default_rng(seed)
    pos = g.uniform(0, 1, (n, 3))
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    return pos, q


def _moves(pos, n, count, step, seed):
    g = np.random.default_rng(seed)
    ks = g.integers(0, len(pos), count)
    return [(int(k), pos[k] + g.uniform(-step, step, 3)) for k in ks]


@pytest.fixture(scope="module")
def ewald_ref():
    pos, q = _system()
    e = O.Ewald(pos, q, 1.0)
    mv = _moves(pos, len(q), 30, 0.05, 9)
    return pos, q, mv, np.array([e.propose(k, r) for k, r in mv])


@pytest.mark.parametrize("p,bound", [(4, 5e-3), (8, 5e-4), (12, 5e-5), (16, 5e-6), (20, 1.5e-6)])
def test_dE_converges_to_ewald(ewald_ref, p, bound):
    # the whole periodic method (IL expansions with images, near field,
    # self-image correction, far lattice with its 1/2, tin-foil term)
    pos, q, mv, ref = ewald_ref
    m = O.Multilevel(pos, q, 1.0, 2, p)
    de = np.array([m.propose(k, r) for k, r in mv])
    rel = np.sqrt(np.mean((de - ref) ** 2)) / np.sqrt(np.mean(ref ** 2))
    assert rel < bound


def test_rocksalt_madelung_energy_to_truncation():
    pos, q = workloads.rocksalt_lattice(4)
    ref = -(len(q) / 2.0) * MADELUNG * 4
    m = O.Multilevel(pos, q, 1.0, 2, 12)
    assert m.energy() == pytest.approx(ref, rel=1e-6)


def test_fmm_and_direct_initialisations_agree_to_truncation():
    pos, q = _system(150, 2)
    mv = _moves(pos, len(q), 10, 0.05, 3)
    a = O.Multilevel(pos, q, 1.0, 2, 12, setup="fmm")
    b = O.Multilevel(pos, q, 1.0, 2, 12, setup="direct")
    da = np.array([a.propose(k, r) for k, r in mv])
    db = np.array([b.propose(k, r) for k, r in mv])
    assert np.abs(da - db).max() < 1e-4 * np.sqrt(np.mean(db ** 2))
    # the level-3 expansions of one cell agree where they are evaluated
    for cell in (5, 40):
        n = 4
        c = np.array([cell % n, (cell // n) % n, cell // (n * n)])
        centre = (c + 0.5) / n
        for x in centre + np.random.default_rng(cell).uniform(-0.12, 0.12, (4, 3)):
            va = O.l2p(12, a.local(3, cell), x, centre)
            vb = O.l2p(12, b.local(3, cell), x, centre)
            assert va == pytest.approx(vb, abs=1e-4 * (1 + abs(vb)))


def test_antisymmetry_and_energy_bookkeeping():
    pos, q = _system(200, 8)
    m = O.Multilevel(pos, q, 1.0, 2, 12)
    u0 = m.energy()
    total = 0.0
    g = np.random.default_rng(1)
    for _ in range(25):
        k = int(g.integers(0, len(q)))
        old = m.positions()[k].copy()
        rn = old + g.uniform(-0.1, 0.1, 3)
        de = m.propose(k, rn)
        m.accept(k, rn)
        total += de
        back = m.propose(k, old)
        assert back == pytest.approx(-de, abs=1e-4 * (1 + abs(de)))
    # maintained energy, fresh initialisation and U0 + sum dE agree to truncation
    u_kept = m.energy()
    fresh = O.Multilevel(m.positions(), q, 1.0, 2, 12)
    ew = O.Ewald(m.positions(), q, 1.0)
    assert u_kept == pytest.approx(u0 + total, abs=2e-3)
    assert fresh.energy() == pytest.approx(u0 + total, abs=2e-3)
    assert ew.energy() == pytest.approx(fresh.energy(), abs=2e-3)


def test_wrap_invariance_and_null_move():
    pos, q = _system(120, 4)
    m = O.Multilevel(pos, q, 1.0, 2, 10)
    assert abs(m.propose(7, pos[7])) < 1e-11
    shifted = pos[7] + np.array([1.0, 0.0, -1.0])
    assert abs(m.propose(7, shifted)) < 1e-9


def test_lazy_mode_matches_eager_mode_after_accepts():
    pos, q = _system(150, 6)
    eager = O.Multilevel(pos, q, 1.0, 2, 8, setup="fmm")
    lazy = O.Multilevel(pos, q, 1.0, 2, 8, setup="lazy")
    g = np.random.default_rng(2)
    for _ in range(12):
        k = int(g.integers(0, len(q)))
        rn = eager.positions()[k] + g.uniform(-0.08, 0.08, 3)
        a, b = eager.propose(k, rn), lazy.propose(k, rn)
        assert a == pytest.approx(b, rel=1e-12, abs=1e-12)
        eager.accept(k, rn)
        lazy.accept(k, rn)
    for cell in (0, 17, 40, 63):
        assert np.allclose(eager.local(3, cell), lazy.local(3, cell), rtol=0, atol=1e-10)


def test_run_decisions_follow_metropolis_rule():
    wl = workloads.uniform(200, 2, 6, 0.05, seed=3)
    m = O.Multilevel(wl.pos, wl.q, 1.0, 2, 6)
    tr = m.run(wl.seed, 0, 0, 60, 1.0, wl.max_step)
    assert np.array_equal(tr["acc"], tr["u"] < np.exp(-tr["dE"]))
    for t in range(60):
        i, d, u = O.draw(wl.seed, 0, t, wl.n, wl.max_step)
        assert i == tr["idx"][t] and u == tr["u"][t]
    assert 0 < tr["acc"].sum() < 60


def _deep_moves(pos, count, step, seed):
    g = np.random.default_rng(seed)
    ks = g.integers(0, len(pos), count)
    return [(int(k), pos[k] + g.uniform(-step, step, 3)) for k in ks]


@pytest.mark.parametrize("depth,n,bound12,bound8", [(3, 2000, 1e-5, 3e-4), (4, 4000, 2e-5, 1e-3)])
def test_deep_periodic_dE_converges_to_ewald(depth, n, bound12, bound8):
    # Depth >= 3 under periodicity: levels with 4 and more cells per side,
    # where interaction lists are no longer aliased and the images of the
    # extended domain enter through distinct cells. The error against Ewald
    # must be small at p = 12 and fall by more than an order of magnitude
    # from p = 8 (a wrong offset, sign or missing level would not converge).
    pos, q = _system(n, 40 + depth)
    mv = _deep_moves(pos, 30, 0.3 / n ** (1 / 3), 7)
    e = O.Ewald(pos, q, 1.0)
    ref = np.array([e.propose(k, r) for k, r in mv])
    err = {}
    for p in (8, 12):
        m = O.Multilevel(pos, q, 1.0, depth, p, setup="lazy")
        de = np.array([m.propose(k, r) for k, r in mv])
        err[p] = np.sqrt(np.mean((de - ref) ** 2)) / np.sqrt(np.mean(ref ** 2))
    assert err[12] < bound12 and err[8] < bound8
    assert err[8] > 10 * err[12]


def test_deep_periodic_accepts_follow_ewald():
    # depth 3, p = 12: 20 accepted moves (Alg. L.2 on levels 2..4 with
    # images), then proposals from the moved state against Ewald following
    # the same accepts
    pos, q = _system(2000, 43)
    m = O.Multilevel(pos, q, 1.0, 3, 12, setup="lazy")
    e = O.Ewald(pos, q, 1.0)
    step = 0.3 / 2000 ** (1 / 3)
    for k, r in _deep_moves(pos, 20, step, 11):
        m.accept(k, r)
        e.accept(k, r)
    cur = m.positions()
    assert np.allclose(cur, e_positions_after(pos, _deep_moves(pos, 20, step, 11)), rtol=0, atol=0)
    mv = _deep_moves(cur, 30, step, 12)
    de = np.array([m.propose(k, r) for k, r in mv])
    ref = np.array([e.propose(k, r) for k, r in mv])
    assert np.sqrt(np.mean((de - ref) ** 2)) / np.sqrt(np.mean(ref ** 2)) < 1e-5


def e_positions_after(pos, moves):
    """positions after the moves, wrapped into the unit box (no arithmetic
    of the method: the wrap of the oracle itself)"""
    out = pos.copy()
    for k, r in moves:
        out[k] = [O.wrap(float(v), 1.0) for v in r]
    return out
