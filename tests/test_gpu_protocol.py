"""The whole-GPU chain's update protocol under runs of consecutive accepts.

A target row of one accepted move can belong to another helper workgroup on
the next move, so a row update lost or applied twice would leave a local
expansion off by a whole P2L term (Alg. L.2) while the decisions around it
could still agree. The test runs a chain whose moves are accepted about half
of the time (more than a quarter of the steps follow an accepted step), then
replays its accepted moves on an oracle whose expansions start at zero: the
change of every local expansion of the GPU chain over the run must equal the
oracle's sum of the P2L updates, within 1e-10 of each level's largest
coefficient (1e-5 in mixed precision, whose update harmonics are FP32;
a lost or doubled term is of the order of 1e-2). The FP64 run is repeated
with 16 and 23 helper workgroups instead of one per accept block, so that
a helper holds several blocks, of more than one level.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import real_layout

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("flags,helpers", [(0, 0), (1, 0), (0, 16), (0, 23)])
def test_consecutive_accepts_update_every_row_once(flags, helpers):
    from paper_2006_16622_amd import Chain, run_chains
    wl = W.uniform(4000, 4, 8, 0.01, seed=101, key=61)
    steps = 3000
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=flags)
    gpu.set_helpers(helpers)  # 0: one helper per accept block; else blocks of several levels per helper
    before = {l: gpu.locals(l) for l in range(2, wl.depth + 2)}
    say(f"[protocol] flags {flags}, helpers {helpers}: whole-GPU run of {steps} steps")
    st, tr = run_chains([gpu], steps, wl.seed, wl.beta, wl.max_step, mode=2, traces=True)
    assert st[0]["status"] == 0
    acc = tr["acc"][0]
    assert (acc[1:] & acc[:-1]).mean() > 0.25
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p, setup="none")
    for k in np.nonzero(acc)[0]:
        orc.accept(int(tr["idx"][0][k]), tr["newpos"][0][k])
    assert np.array_equal(orc.positions(), gpu.positions())
    for level in range(2, wl.depth + 2):
        got = gpu.locals(level) - before[level]
        ref = np.array([real_layout(orc.local(level, c), wl.p) for c in range(8 ** (level - 1))])
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(f"[protocol] level {level}: max |change - P2L sum| / level max = {err:.2e}")
        assert err <= (1e-5 if flags else 1e-10)


def test_set_helpers_rejects_a_negative_count():
    from paper_2006_16622_amd import Chain, FmmMcError
    wl = W.uniform(300, 2, 4, 0.05, seed=102, key=62)
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    with pytest.raises(FmmMcError) as e:
        gpu.set_helpers(-1)
    assert e.value.code == -1  # FMM_MC_EINVAL
    gpu.set_helpers(0)
