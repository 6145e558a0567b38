"""Parity at high expansion degree (p = 18 and 20, the 32-lane variant
with degree bound 24) on deep trees: sampled proposals against the oracle,
which initialises each cell's local expansion on first use (lazy mode)."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import dE_close

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


CASES = {
    "n300_d2_p20": (lambda: W.uniform(300, 2, 20, 0.05, seed=31, key=7), 30),
    "n10000_d4_p18": (lambda: W.uniform(10000, 4, 18, 0.02, seed=32, key=8), 12),
    "rocksalt_d5_p18": (lambda: W.rocksalt(p=18), 8),
}


@pytest.mark.parametrize("name", list(CASES))
def test_high_degree_proposals_match_oracle(name):
    from paper_2006_16622_amd import Chain
    make, count = CASES[name]
    wl = make()
    say(f"[high-p] {name}: gpu setup")
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p, setup="lazy")
    pos = orc.positions()
    de, ref = [], []
    for t in range(count):
        i, d, _ = O.draw(wl.seed, 0, t, wl.n, wl.max_step)
        de.append(gpu.propose(i, pos[i] + d))
        ref.append(orc.propose(i, pos[i] + d))
    de, ref = np.array(de), np.array(ref)
    rms = np.sqrt(np.mean(ref ** 2))
    say(f"[high-p] {name}: max |dE_gpu - dE_oracle| / RMS = {np.abs(de - ref).max() / rms:.3e}")
    assert dE_close(de, ref, rms).all()
