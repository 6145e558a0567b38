"""Parity at the benchmark's full size: the jittered rock-salt system of 46^3
= 97336 charges, depth 5, degree 12, run by the same whole-GPU kernel and
launch shape that bench.py times. The oracle computes each cell's local
expansion on first use (lazy mode), so sampled proposals and a prefix of the
chain can be checked one by one: indices, wrapped positions and decisions
bit-exact, dE within 1e-10 relative."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import dE_close

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def rocksalt():
    return W.rocksalt()


def _compare(wl, tr_o, dE, acc, idx, newpos):
    rms = np.sqrt(np.mean(tr_o["dE"] ** 2))
    margin = np.abs(tr_o["u"] - np.exp(-wl.beta * tr_o["dE"]))
    assert margin.min() > 1e-9  # no decision is a near-tie at the dE tolerance
    assert np.array_equal(idx, tr_o["idx"])
    assert np.array_equal(newpos, tr_o["newpos"])
    assert dE_close(dE, tr_o["dE"], rms).all(), np.abs(dE - tr_o["dE"]).max()
    assert np.array_equal(acc, tr_o["acc"])


def test_rocksalt_run_prefix_bit_exact(rocksalt):
    from paper_2006_16622_amd import Chain, run_chains
    wl = rocksalt
    steps = 240
    say("[fullsize] gpu setup + run")
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    st, tr = run_chains([gpu], steps, wl.seed, wl.beta, wl.max_step, mode=0, traces=True)
    assert st[0]["status"] == 0
    say("[fullsize] oracle (lazy) run")
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p, setup="lazy")
    tr_o = orc.run(wl.seed, 0, 0, steps, wl.beta, wl.max_step)
    _compare(wl, tr_o, tr["dE"][0], tr["acc"][0], tr["idx"][0], tr["newpos"][0])
    assert tr_o["acc"].sum() > 50
    assert np.array_equal(gpu.positions(), orc.positions())
    assert gpu.running_energy() == pytest.approx(st[0]["energy"], rel=1e-12)


def test_rocksalt_after_warmup_matches(rocksalt):
    # the bench's timed region starts after 2000 warmup steps: the oracle
    # applies the GPU's accepted moves of the warmup, then the next 40 steps
    # are compared one by one
    from paper_2006_16622_amd import Chain, run_chains
    wl = rocksalt
    warm, steps = 2000, 40
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    st, tr = run_chains([gpu], warm, wl.seed, wl.beta, wl.max_step, mode=0, traces=True)
    assert st[0]["status"] == 0
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p, setup="lazy")
    acc = tr["acc"][0]
    for t in np.nonzero(acc)[0]:
        orc.accept(int(tr["idx"][0][t]), tr["newpos"][0][t])
    assert np.array_equal(gpu.positions(), orc.positions())
    say(f"[fullsize] {acc.sum()} warmup accepts applied; comparing {steps} steps")
    st2, tr2 = run_chains([gpu], steps, wl.seed, wl.beta, wl.max_step, t0=warm, mode=0, traces=True)
    tr_o = orc.run(wl.seed, 0, warm, steps, wl.beta, wl.max_step)
    _compare(wl, tr_o, tr2["dE"][0], tr2["acc"][0], tr2["idx"][0], tr2["newpos"][0])
