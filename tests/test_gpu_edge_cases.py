"""Edge cases of the GPU path through the C ABI:

* the smallest system (two opposite charges, depth 1) against the oracle;
* the largest degree the library supports (p = 24) and the largest depth
  (7: 8^7 leaves, 8 levels) against the oracle (lazy initialisation at
  depth 7);
* a move onto another charge: the single-call proposal reports
  FMM_MC_ESINGULAR, and in a replayed list the step is rejected while the
  steps around it match the oracle;
* a leaf bin filled to its capacity: the accept that would overflow it
  reports FMM_MC_EOVERFLOW.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import dE_close

pytestmark = pytest.mark.gpu

ESINGULAR, EOVERFLOW = -4, -7


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _proposals_match(gpu, orc, wl, count, seed, rel=1e-10):
    pos = orc.positions()
    g = np.random.default_rng(seed)
    de, ref = [], []
    for _ in range(count):
        i = int(g.integers(0, wl.n))
        rn = pos[i] + g.uniform(-wl.max_step, wl.max_step, 3)
        de.append(gpu.propose(i, rn))
        ref.append(orc.propose(i, rn))
    ref = np.array(ref)
    assert dE_close(de, ref, np.sqrt(np.mean(ref ** 2)), rel).all(), np.abs(np.array(de) - ref).max()


def test_two_charges():
    from paper_2006_16622_amd import Chain, run_chains
    pos = np.array([[0.3, 0.4, 0.5], [0.7, 0.45, 0.55]])
    q = np.array([1.0, -1.0])
    gpu = Chain(pos, q, 1.0, 1, 4)
    orc = O.Multilevel(pos, q, 1.0, 1, 4)
    assert gpu.energy() == pytest.approx(orc.energy(), rel=1e-10)
    st, tr = run_chains([gpu], 100, 7, 1.0, 0.1, mode=2, traces=True)
    ref = orc.run(7, 0, 0, 100, 1.0, 0.1)
    assert st[0]["status"] == 0
    assert np.array_equal(tr["acc"][0], ref["acc"]) and np.array_equal(tr["newpos"][0], ref["newpos"])
    assert dE_close(tr["dE"][0], ref["dE"], np.sqrt(np.mean(ref["dE"] ** 2))).all()


def test_largest_degree():
    from paper_2006_16622_amd import Chain
    wl = W.uniform(200, 1, 24, 0.05, seed=92, key=52)
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    # Tolerance at p = 24: the far-lattice operator uses lattice sums up to
    # degree 2p = 48, which both sides evaluate by Ewald splits with an
    # absolute error of about 1e-15 (pinned against brute force in the
    # oracle's lattice tests); the operator multiplies S_(j+n) by factors up
    # to C(48, 24) ~ 3e13, so two correct evaluations differ by a few 1e-10
    # of RMS dE (6e-10 measured) instead of the 1e-10 that holds up to p = 20.
    assert gpu.energy() == pytest.approx(orc.energy(), rel=1e-9)
    _proposals_match(gpu, orc, wl, 12, 93, rel=5e-9)


def test_largest_depth():
    from paper_2006_16622_amd import Chain, run_chains
    wl = W.uniform(3000, 7, 3, 0.003, seed=91, key=51)
    say("[edge] depth 7: setups")
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p, setup="lazy")
    _proposals_match(gpu, orc, wl, 20, 94)
    st, tr = run_chains([gpu], 60, wl.seed, wl.beta, wl.max_step, mode=2, traces=True)
    ref = orc.run(wl.seed, 0, 0, 60, wl.beta, wl.max_step)
    assert st[0]["status"] == 0 and ref["acc"].sum() > 5
    assert np.array_equal(tr["acc"][0], ref["acc"]) and np.array_equal(tr["newpos"][0], ref["newpos"])
    assert dE_close(tr["dE"][0], ref["dE"], np.sqrt(np.mean(ref["dE"] ** 2))).all()


def test_move_onto_another_charge():
    from paper_2006_16622_amd import Chain, FmmMcError
    wl = W.uniform(500, 2, 6, 0.05, seed=95, key=53)
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    pos = gpu.positions()
    with pytest.raises(FmmMcError) as e:
        gpu.propose(3, pos[10])
    assert e.value.code == ESINGULAR
    # a replayed list: ordinary moves around one onto charge 10's position
    g = np.random.default_rng(96)
    idx = g.integers(0, wl.n, 9)
    idx[idx == 10] = 11  # charge 10 stays where it is
    idx[4] = 3
    new = pos[idx] + g.uniform(-0.05, 0.05, (9, 3))
    new[4] = pos[10]
    u = g.uniform(0, 1, 9)
    dE, acc, _ = gpu.replay(idx, new, u, 1.0)
    assert not acc[4]
    for k in range(9):
        if k == 4:
            continue
        d = orc.propose(int(idx[k]), new[k])
        assert dE[k] == pytest.approx(d, rel=1e-10, abs=1e-10)
        assert acc[k] == (u[k] < np.exp(-d))
        if acc[k]:
            orc.accept(int(idx[k]), new[k])
    assert np.array_equal(gpu.positions(), orc.positions())


def test_leaf_overflow_is_reported():
    from paper_2006_16622_amd import Chain, FmmMcError
    wl = W.uniform(128, 2, 4, 0.05, seed=97, key=54)
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    cap = 32  # the bin capacity for 2 charges per leaf: next power of two >= 3 * 2 + 16
    pos = gpu.positions()
    leaf = np.floor(pos * 4).astype(int)
    in_leaf = (leaf == 0).all(axis=1)
    movers = [k for k in range(wl.n) if not in_leaf[k]]
    g = np.random.default_rng(98)
    count = int(in_leaf.sum())
    code = 0
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    before = None
    for k in movers:
        target = g.uniform(0.01, 0.24, 3)
        before = (gpu.positions(), gpu.running_energy(), gpu.locals(2), gpu.locals(3), gpu.energy())
        try:
            gpu.accept(k, target)
        except FmmMcError as e:
            code = e.code
            break
        orc.accept(k, target)
        count += 1
    assert code == EOVERFLOW and count == cap
    # the refused move changed nothing: positions, running energy, every
    # expansion and the energy are those before it, and the chain goes on
    # exactly as the oracle that never saw the move
    assert np.array_equal(gpu.positions(), before[0])
    assert gpu.running_energy() == before[1]
    assert np.array_equal(gpu.locals(2), before[2]) and np.array_equal(gpu.locals(3), before[3])
    assert gpu.energy() == before[4]
    assert np.array_equal(gpu.positions(), orc.positions())
    # a charge inside the full leaf moves within it (no change of bin)
    cur = gpu.positions()
    k = int(np.nonzero(((cur >= 0.03) & (cur < 0.22)).all(axis=1))[0][0])
    rn = cur[k] + np.array([0.01, -0.02, 0.015])
    assert gpu.propose(k, rn) == pytest.approx(orc.propose(k, rn), rel=1e-10, abs=1e-10)
    gpu.accept(k, rn)
    orc.accept(k, rn)
    assert np.array_equal(gpu.positions(), orc.positions())
