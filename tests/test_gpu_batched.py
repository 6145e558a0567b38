"""GPU parity of the batched launch: several independent chains of uneven
size and depth in one kernel, each against its own oracle run."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import dE_close

pytestmark = pytest.mark.gpu


def test_batched_chains_match_oracle():
    from paper_2006_16622_amd import Chain, run_chains
    specs = [(200, 1, 6, 0.08), (600, 2, 6, 0.05), (1500, 2, 6, 0.04), (400, 2, 6, 0.06)]
    wls = [W.uniform(n, d, p, s, seed=21, key=10 + i) for i, (n, d, p, s) in enumerate(specs)]
    steps = 80
    chains = [Chain(w.pos, w.q, w.box, w.depth, w.p) for w in wls]
    print("[batched] run", file=sys.stderr, flush=True)
    st, tr = run_chains(chains, steps, 21, 1.0, [w.max_step for w in wls], traces=True)
    for c, w in enumerate(wls):
        orc = O.Multilevel(w.pos, w.q, w.box, w.depth, w.p)
        to = orc.run(21, c, 0, steps, 1.0, w.max_step)
        assert st[c]["status"] == 0
        assert np.array_equal(tr["idx"][c], to["idx"])
        assert np.array_equal(tr["newpos"][c], to["newpos"])
        assert np.array_equal(tr["acc"][c], to["acc"])
        rms = np.sqrt(np.mean(to["dE"] ** 2))
        assert dE_close(tr["dE"][c], to["dE"], rms).all()
        assert np.array_equal(chains[c].positions(), orc.positions())
