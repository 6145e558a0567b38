"""The direct P2L initialisation (Alg. L.3, FMM_MC_DIRECT_SETUP) against the
oracle's Alg. L.3 on the same seeded inputs, through the C ABI:

* local expansions within 1e-10 of each level's largest coefficient and
  the setup energy within 1e-10;
* a whole-GPU run after the direct setup: decisions bit-exact, dE within
  1e-10;
* the batched setup and the re-setup graph bit-identical to single eager
  setups;
* the direct and the M2L setups agree to truncation (1e-4 of RMS dE);
* at full size (rock salt, N = 97336, depth 5, p = 12), sampled cells of
  levels 4..6 against the oracle's P2L summed over the cell's interaction
  list, one charge at a time.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import dE_close, real_layout

pytestmark = pytest.mark.gpu

DIRECT = 0x4

CASES = {
    "n600_d2_p6": lambda: W.uniform(600, 2, 6, 0.05, seed=71, key=31),
    "n1000_d3_p8": W.small,
    "n300_d2_p16": lambda: W.uniform(300, 2, 16, 0.05, seed=72, key=32),
    "n2002_d3_p12": lambda: W.uniform(2002, 3, 12, 0.03, seed=73, key=33),
}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    from paper_2006_16622_amd import Chain
    wl = CASES[request.param]()
    say(f"[direct] case {request.param}: oracle and gpu setup")
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p, setup="direct")
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=DIRECT)
    return request.param, wl, orc, gpu


def test_direct_setup_locals_and_energy(case):
    name, wl, orc, gpu = case
    for level in range(2, wl.depth + 2):
        got = gpu.locals(level)
        ncell = 8 ** (level - 1)
        cells = range(ncell) if ncell <= 64 else np.random.default_rng(level).choice(ncell, 64, replace=False)
        ref = np.array([real_layout(orc.local(level, int(c)), wl.p) for c in cells])
        assert np.abs(got[list(cells)] - ref).max() <= 1e-10 * np.abs(ref).max(), (name, level)
    assert gpu.energy() == pytest.approx(orc.energy(), rel=1e-10, abs=1e-9)


def test_run_after_direct_setup_matches_oracle():
    from paper_2006_16622_amd import Chain, run_chains
    wl = W.uniform(1000, 3, 8, 0.05, seed=74, key=34)
    steps = 200
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p, setup="direct")
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=DIRECT)
    st, tr = run_chains([gpu], steps, wl.seed, wl.beta, wl.max_step, mode=2, traces=True)
    ref = orc.run(wl.seed, 0, 0, steps, wl.beta, wl.max_step)
    assert st[0]["status"] == 0
    assert np.abs(ref["u"] - np.exp(-wl.beta * ref["dE"])).min() > 1e-9
    assert np.array_equal(tr["acc"][0], ref["acc"]) and np.array_equal(tr["newpos"][0], ref["newpos"])
    rms = np.sqrt(np.mean(ref["dE"] ** 2))
    assert dE_close(tr["dE"][0], ref["dE"], rms).all()
    assert np.array_equal(gpu.positions(), orc.positions())


def test_direct_batched_setup_and_resetup_are_bit_identical():
    from paper_2006_16622_amd import Chain, run_chains, setup_batch
    wls = [W.uniform(500 + 300 * k, 2 + k % 2, 8, 0.05, seed=75, key=35 + k) for k in range(3)]
    batch = setup_batch([(w.pos, w.q, w.box, w.depth) for w in wls], 8, flags=DIRECT)
    for w, b in zip(wls, batch):
        single = Chain(w.pos, w.q, w.box, w.depth, w.p, flags=DIRECT)
        for level in range(2, w.depth + 2):
            assert np.array_equal(b.locals(level), single.locals(level))
        assert b.energy() == single.energy()
    w, gpu = wls[1], batch[1]
    st = run_chains([gpu], 100, w.seed, w.beta, w.max_step, mode=2)
    assert st[0]["status"] == 0 and st[0]["accepted"] > 0
    gpu.resetup()
    fresh = Chain(gpu.positions(), w.q, w.box, w.depth, w.p, flags=DIRECT)
    for level in range(2, w.depth + 2):
        assert np.array_equal(gpu.locals(level), fresh.locals(level))
    assert gpu.running_energy() == fresh.running_energy()


def test_direct_and_m2l_setups_agree_to_truncation():
    from paper_2006_16622_amd import Chain
    wl = W.uniform(3000, 3, 12, 0.04, seed=76, key=38)
    a = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=DIRECT)
    b = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    pos = a.positions()
    da, db = [], []
    for t in range(40):
        i, d, _ = O.draw(wl.seed, 0, t, wl.n, wl.max_step)
        da.append(a.propose(i, pos[i] + d))
        db.append(b.propose(i, pos[i] + d))
    da, db = np.array(da), np.array(db)
    rms = np.sqrt(np.mean(db ** 2))
    say(f"[direct] direct vs M2L setup: max |dE diff| / RMS = {np.abs(da - db).max() / rms:.2e}")
    assert np.abs(da - db).max() < 1e-4 * rms


def test_full_size_sampled_cells():
    from paper_2006_16622_amd import Chain
    wl = W.rocksalt()
    say("[direct] rock salt full size: gpu direct setup")
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=DIRECT)
    pos, q, a, p = gpu.positions(), wl.q, wl.box, wl.p
    g = np.random.default_rng(77)
    for level, count in ((wl.depth + 1, 4), (wl.depth, 3), (wl.depth - 1, 2)):
        n = 2 ** (level - 1)
        h = a / n
        cell_of = np.minimum(np.floor(pos * (n / a)).astype(np.int64), n - 1)
        lin = cell_of[:, 0] + n * (cell_of[:, 1] + n * cell_of[:, 2])
        got_all = gpu.locals(level)
        scale = np.abs(got_all).max()
        for cell in g.choice(n ** 3, count, replace=False):
            c = np.array([cell % n, (cell // n) % n, cell // (n * n)])
            centre = (c + 0.5) * h
            ref = np.zeros(O.ncoef(p), dtype=np.complex128)
            for off in O.il_offsets(c & 1):
                b = c + off
                s = b % n
                shift = (b // n) * a
                for j in np.nonzero(lin == s[0] + n * (s[1] + n * s[2]))[0]:
                    ref += O.p2l(p, q[j], pos[j] + shift, centre)
            err = np.abs(got_all[cell] - real_layout(ref, p)).max()
            say(f"[direct] level {level} cell {cell}: max error / level max = {err / scale:.2e}")
            assert err <= 1e-10 * scale
