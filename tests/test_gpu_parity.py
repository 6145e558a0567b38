"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs. Bit-exact: leaf cells, accept decisions, proposal
stream. dE within 1e-10 relative (to max(|dE|, RMS dE)); expansions within
1e-10 of each level's largest coefficient."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import dE_close, real_layout

pytestmark = pytest.mark.gpu

CASES = {
    "n600_d2_p6": lambda: W.uniform(600, 2, 6, 0.05, seed=11, key=1),
    "n1000_d3_p8": W.small,
    "n64_d1_p4": lambda: W.uniform(64, 1, 4, 0.1, seed=12, key=2),
    "n300_d2_p16": lambda: W.uniform(300, 2, 16, 0.05, seed=13, key=3),
    # the third 16-lane degree bound (p 13..15): the whole-GPU chain and k_run_chains
    "n800_d2_p14": lambda: W.uniform(800, 2, 14, 0.05, seed=15, key=5),
    "n2000_d3_p3_ragged": lambda: W.uniform(2002, 3, 3, 0.03, seed=14, key=4),
}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    from paper_2006_16622_amd import Chain
    wl = CASES[request.param]()
    say(f"[parity] case {request.param}: oracle setup")
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    say(f"[parity] case {request.param}: gpu setup")
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    return request.param, wl, orc, gpu


def test_setup_expansions_match(case):
    name, wl, orc, gpu = case
    p = wl.p
    for level in range(2, wl.depth + 2):
        got = gpu.locals(level)
        ncell = 8 ** (level - 1)
        cells = range(ncell) if ncell <= 64 else np.random.default_rng(level).choice(ncell, 64, replace=False)
        ref = np.array([real_layout(orc.local(level, int(c)), p) for c in cells])
        scale = np.abs(ref).max()
        assert np.abs(got[list(cells)] - ref).max() <= 1e-10 * scale, (name, level)


def test_setup_energy_matches(case):
    name, wl, orc, gpu = case
    assert gpu.energy() == pytest.approx(orc.energy(), rel=1e-10, abs=1e-9)
    assert gpu.running_energy() == pytest.approx(orc.energy(), rel=1e-10, abs=1e-9)


def test_propose_matches(case):
    name, wl, orc, gpu = case
    pos = orc.positions()
    g = np.random.default_rng(7)
    des, ref = [], []
    for t in range(60):
        i, d, u = O.draw(wl.seed, 0, t, wl.n, wl.max_step)
        rn = pos[i] + d
        if t % 7 == 0:
            rn = pos[i] + g.uniform(-0.4, 0.4, 3)  # also far moves
        des.append(gpu.propose(i, rn))
        ref.append(orc.propose(i, rn))
    ref = np.array(ref)
    rms = np.sqrt(np.mean(ref ** 2))
    assert dE_close(des, ref, rms).all(), np.abs(np.array(des) - ref).max()


def _check_traces(wl, tr_o, dE, acc, leaf=None, idx=None, newpos=None):
    rms = np.sqrt(np.mean(tr_o["dE"] ** 2))
    # no near-tie may make a decision ambiguous at the dE tolerance
    margin = np.abs(tr_o["u"] - np.exp(-wl.beta * tr_o["dE"]))
    assert margin.min() > 1e-9
    assert dE_close(dE, tr_o["dE"], rms).all(), np.abs(dE - tr_o["dE"]).max()
    assert np.array_equal(acc, tr_o["acc"])
    if idx is not None:
        assert np.array_equal(idx, tr_o["idx"])
    if newpos is not None:
        assert np.array_equal(newpos, tr_o["newpos"])  # bit-exact wrap
    if leaf is not None:
        n = 2 ** wl.depth
        c = np.minimum(np.floor(tr_o["newpos"] * (n / wl.box)).astype(int), n - 1)
        assert np.array_equal(leaf, c[:, 0] + n * (c[:, 1] + n * c[:, 2]))


def test_replay_and_state_after_accepts(case):
    from paper_2006_16622_amd import Chain
    name, wl, _, _ = case
    steps = 120
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    u0 = orc.energy()
    tr = orc.run(wl.seed, 0, 0, steps, wl.beta, wl.max_step)
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    say(f"[parity] case {name}: replay {steps}")
    dE, acc, leaf = gpu.replay(tr["idx"], tr["newpos"], tr["u"], wl.beta)
    _check_traces(wl, tr, dE, acc, leaf)
    assert tr["acc"].sum() > 5
    assert np.array_equal(gpu.positions(), orc.positions())
    for level in range(2, wl.depth + 2):
        got = gpu.locals(level)
        cells = range(min(64, 8 ** (level - 1)))
        ref = np.array([real_layout(orc.local(level, c), wl.p) for c in cells])
        assert np.abs(got[list(cells)] - ref).max() <= 1e-10 * np.abs(ref).max()
    # running energy = setup energy + accepted dE (the bookkeeping of Sec. 4.1)
    assert gpu.running_energy() == pytest.approx(u0 + tr["dE"][tr["acc"]].sum(), rel=1e-10)
    # the maintained state's energy equals a fresh evaluation on both sides
    assert gpu.energy() == pytest.approx(orc.energy(), rel=1e-10)


@pytest.mark.parametrize("mode", [0, 1])
def test_run_matches_oracle_trajectory(case, mode):
    from paper_2006_16622_amd import Chain, run_chains
    name, wl, _, _ = case
    steps = 150
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    tr = orc.run(wl.seed, 0, 0, steps, wl.beta, wl.max_step)
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    say(f"[parity] case {name}: run mode {mode}")
    st, gt = run_chains([gpu], steps, wl.seed, wl.beta, wl.max_step, mode=mode, traces=True)
    assert st[0]["status"] == 0
    assert st[0]["proposed"] == steps and st[0]["accepted"] == tr["acc"].sum()
    _check_traces(wl, tr, gt["dE"][0], gt["acc"][0], idx=gt["idx"][0], newpos=gt["newpos"][0])
    assert np.array_equal(gpu.positions(), orc.positions())


def test_accept_entry_point(case):
    from paper_2006_16622_amd import Chain
    name, wl, _, _ = case
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    g = np.random.default_rng(3)
    for _ in range(6):
        k = int(g.integers(wl.n))
        rn = orc.positions()[k] + g.uniform(-0.2, 0.2, 3)
        de_o = orc.propose(k, rn)
        de_g = gpu.accept(k, rn)  # proposes first when dE is not given
        orc.accept(k, rn)
        assert de_g == pytest.approx(de_o, rel=1e-10, abs=1e-10)
    k = int(g.integers(wl.n))
    rn = orc.positions()[k] + 0.05
    gpu.accept(k, rn, dE=123.0)
    orc.accept(k, rn)
    for level in range(2, wl.depth + 2):
        got = gpu.locals(level)[:8]
        ref = np.array([real_layout(orc.local(level, c), wl.p) for c in range(8)])
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
