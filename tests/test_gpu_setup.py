"""The setup pass in its batched and graph-replayed forms.

* fmm_mc_setup_batch runs every setup kernel once over many chains (the
  M2L of all levels of all chains in one launch): its expansions, bins and
  energies must equal, bit for bit, those of one fmm_mc_setup per chain.
* fmm_mc_resetup rebuilds the expansions from the device-resident
  positions through a captured HIP graph: each replay, with Monte Carlo
  steps and host synchronisations between replays, must equal bit for bit
  an eager fmm_mc_setup of the same positions.
* The expansions of the batched setup equal the oracle's within 1e-10 (the
  single-chain setup is checked the same way by the parity tests)."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import real_layout

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _same_state(a, b, depth):
    for level in range(2, depth + 2):
        assert np.array_equal(a.locals(level), b.locals(level)), level
    assert np.array_equal(a.positions(), b.positions())
    assert a.running_energy() == b.running_energy()


def _batch_systems():
    sizes = W.batched_sizes()
    depth = np.array([s[1] for s in sizes])
    picks = [int(np.nonzero(depth == d)[0][k]) for d in (2, 3, 4) for k in range(2)]
    return [W.batched_chain(c) for c in picks]


def test_batched_setup_equals_single_setups():
    from paper_2006_16622_amd import Chain, setup_batch
    wls = _batch_systems()
    say(f"[setup] batch of {len(wls)} chains, depths {[w.depth for w in wls]}")
    batch = setup_batch([(w.pos, w.q, w.box, w.depth) for w in wls], wls[0].p)
    for w, b in zip(wls, batch):
        single = Chain(w.pos, w.q, w.box, w.depth, w.p)
        _same_state(b, single, w.depth)
        assert b.energy() == single.energy()


def test_batched_setup_matches_oracle():
    from paper_2006_16622_amd import setup_batch
    wls = [W.uniform(600, 2, 6, 0.05, seed=41, key=9), W.uniform(1200, 3, 6, 0.05, seed=42, key=10),
           W.uniform(300, 1, 6, 0.05, seed=43, key=11)]
    batch = setup_batch([(w.pos, w.q, w.box, w.depth) for w in wls], 6)
    for w, b in zip(wls, batch):
        orc = O.Multilevel(w.pos, w.q, w.box, w.depth, w.p)
        for level in range(2, w.depth + 2):
            got = b.locals(level)
            cells = range(min(64, 8 ** (level - 1)))
            ref = np.array([real_layout(orc.local(level, c), w.p) for c in cells])
            assert np.abs(got[list(cells)] - ref).max() <= 1e-10 * np.abs(ref).max()
        assert b.energy() == pytest.approx(orc.energy(), rel=1e-10)


def test_resetup_graph_replays_equal_eager_setup():
    from paper_2006_16622_amd import Chain, run_chains
    wl = W.uniform(3000, 3, 12, 0.04, seed=44, key=12)
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    for k in range(3):
        st = run_chains([gpu], 150, wl.seed, wl.beta, wl.max_step, t0=150 * k, mode=k % 2)
        assert st[0]["status"] == 0 and st[0]["accepted"] > 0
        say(f"[setup] resetup replay {k}")
        gpu.resetup()
        fresh = Chain(gpu.positions(), wl.q, wl.box, wl.depth, wl.p)
        for level in range(2, wl.depth + 2):
            assert np.array_equal(gpu.locals(level), fresh.locals(level)), (k, level)
        # the running energy is replaced by the fresh total energy
        assert gpu.running_energy() == fresh.running_energy()
        assert gpu.energy() == fresh.energy()
        # a proposal on the re-set-up chain equals one on the fresh chain
        i, d, _ = O.draw(wl.seed, 0, 9999 + k, wl.n, wl.max_step)
        r = gpu.positions()[i] + d
        assert gpu.propose(i, r) == fresh.propose(i, r)
        fresh.close()


def _oracle_with_resetups(wl, steps, every, chain=0):
    """the oracle's chain with a fresh setup from its positions after every
    `every` accepted moves (the re-setup the run loop performs)"""
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    out = {k: [] for k in ("idx", "newpos", "dE", "u", "acc")}
    since = 0
    for t in range(steps):
        tr = orc.run(wl.seed, chain, t, 1, wl.beta, wl.max_step)
        for k in out:
            out[k].append(tr[k][0])
        if tr["acc"][0]:
            since += 1
            if since == every and t + 1 < steps:
                orc = O.Multilevel(orc.positions(), wl.q, wl.box, wl.depth, wl.p)
                since = 0
    return {k: np.array(v) for k, v in out.items()}, orc


@pytest.mark.parametrize("mode", [0, 1])
def test_run_with_periodic_resetup_matches_oracle(mode):
    from paper_2006_16622_amd import Chain, run_chains
    wl = W.uniform(600, 2, 6, 0.05, seed=45, key=14)
    steps, every = 240, 20
    ref, orc = _oracle_with_resetups(wl, steps, every)
    assert ref["acc"].sum() > 3 * every
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    st, tr = run_chains([gpu], steps, wl.seed, wl.beta, wl.max_step, mode=mode, traces=True,
                        resetup_every=every)
    assert st[0]["status"] == 0 and st[0]["proposed"] == steps
    assert np.array_equal(tr["idx"][0], ref["idx"])
    assert np.array_equal(tr["newpos"][0], ref["newpos"])
    assert np.array_equal(tr["acc"][0], ref["acc"])
    rms = np.sqrt(np.mean(ref["dE"] ** 2))
    assert np.abs(tr["dE"][0] - ref["dE"]).max() <= 1e-10 * rms
    assert np.array_equal(gpu.positions(), orc.positions())


def test_batched_run_with_periodic_resetup_matches_oracle():
    from paper_2006_16622_amd import Chain, run_chains
    wls = [W.uniform(500 + 100 * k, 2, 6, 0.05, seed=46, key=15 + k) for k in range(3)]
    steps, every = 200, 15
    chains = [Chain(w.pos, w.q, w.box, w.depth, w.p) for w in wls]
    st, tr = run_chains(chains, steps, wls[0].seed, 1.0, [w.max_step for w in wls], mode=1, traces=True,
                        resetup_every=every)
    for k, w in enumerate(wls):
        ref, _ = _oracle_with_resetups(w, steps, every, chain=k)
        assert st[k]["status"] == 0 and st[k]["proposed"] == steps
        assert np.array_equal(tr["acc"][k], ref["acc"])
        assert np.array_equal(tr["newpos"][k], ref["newpos"])
        rms = np.sqrt(np.mean(ref["dE"] ** 2))
        assert np.abs(tr["dE"][k] - ref["dE"]).max() <= 1e-10 * rms


def test_autotune_keeps_state_and_results():
    from paper_2006_16622_amd import Chain, run_chains
    wl = W.uniform(3000, 3, 12, 0.04, seed=47, key=18)
    a = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    levels = range(2, wl.depth + 2)
    before = {l: a.locals(l) for l in levels}
    pos = a.positions()
    t = a.autotune(steps=300, beta=wl.beta, max_step=wl.max_step)
    say(f"[setup] autotune: {t}")
    assert t["m2l_rows"] in (96, 192) and t["helpers"] >= 1 and len(t["step_us"]) >= 2
    # the trials ran on a clone: the chain is unchanged
    for l in levels:
        assert np.array_equal(a.locals(l), before[l])
    assert np.array_equal(a.positions(), pos)
    # a new chain of this shape uses the tuned M2L tile: identical expansions
    b = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    for l in levels:
        assert np.array_equal(b.locals(l), before[l])
    # a run with the tuned helper count follows the oracle's trajectory
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    tr = orc.run(wl.seed, 0, 0, 150, wl.beta, wl.max_step)
    st, gt = run_chains([b], 150, wl.seed, wl.beta, wl.max_step, mode=2, traces=True)
    assert st[0]["status"] == 0
    assert np.array_equal(gt["acc"][0], tr["acc"]) and np.array_equal(gt["newpos"][0], tr["newpos"])
    rms = np.sqrt(np.mean(tr["dE"] ** 2))
    assert np.abs(gt["dE"][0] - tr["dE"]).max() <= 1e-10 * rms
