"""GPU parity at the configurations the benchmark measures, against the
oracle, element by element:

* the batched launch (one workgroup per chain, the kernel of the 256-chain
  line) at p = 12 in FP64 on chains of the batched workload of depth 2, 3
  and 4 and its largest chain, 400 steps each, for the local method and for
  the multipole-based variant;
* the whole-GPU chain on the medium workload (N = 10^4, depth 4, p = 12)
  and on the small workload (N = 10^3, depth 3, p = 8, all 2000 of its
  proposals).

Bit-exact: indices, wrapped new positions, decisions, final positions. dE
within 1e-10 relative (to max(|dE|, RMS dE)). After the run, the energy of
the maintained expansions within 1e-10, and sampled local expansions (or
multipoles) within 1e-10 of each level's largest coefficient."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import dE_close, real_layout

pytestmark = pytest.mark.gpu

MP = 0x2


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _batched_picks():
    sizes = W.batched_sizes()
    depth = np.array([s[1] for s in sizes])
    picks = [int(np.nonzero(depth == d)[0][0]) for d in (2, 3, 4)]
    picks.append(int(np.argmax([s[0] for s in sizes])))
    return picks


def _check_trace(wl, tr_o, idx, newpos, acc, dE):
    rms = np.sqrt(np.mean(tr_o["dE"] ** 2))
    margin = np.abs(tr_o["u"] - np.exp(-wl.beta * tr_o["dE"]))
    assert margin.min() > 1e-9  # no decision is a near-tie at the dE tolerance
    assert np.array_equal(idx, tr_o["idx"])
    assert np.array_equal(newpos, tr_o["newpos"])
    assert np.array_equal(acc, tr_o["acc"])
    assert dE_close(dE, tr_o["dE"], rms).all(), np.abs(dE - tr_o["dE"]).max()


def _expansions_close(gpu, orc, wl, multipole):
    for level in range(2, wl.depth + 2):
        got = gpu.multipoles(level) if multipole else gpu.locals(level)
        ncell = 8 ** (level - 1)
        cells = range(ncell) if ncell <= 64 else np.random.default_rng(level).choice(ncell, 64, replace=False)
        get = orc.multipole if multipole else orc.local
        ref = np.array([real_layout(get(level, int(c)), wl.p) for c in cells])
        assert np.abs(got[list(cells)] - ref).max() <= 1e-10 * np.abs(ref).max(), level


@pytest.mark.parametrize("variant", ["local", "multipole"])
def test_batched_p12_chains_match_oracle(variant):
    from paper_2006_16622_amd import Chain, run_chains
    flags = MP if variant == "multipole" else 0
    picks = _batched_picks()
    wls = [W.batched_chain(c) for c in picks]
    steps = 400
    say(f"[measured] batched p=12 {variant}: chains {picks} (n {[w.n for w in wls]}, "
        f"depth {[w.depth for w in wls]}), gpu run")
    chains = [Chain(w.pos, w.q, w.box, w.depth, w.p, flags=flags) for w in wls]
    # slot k of the launch is chain k of the run: the oracle runs chain k
    st, tr = run_chains(chains, steps, wls[0].seed, 1.0, [w.max_step for w in wls], mode=1, traces=True)
    for k, w in enumerate(wls):
        say(f"[measured] oracle chain {picks[k]} (n={w.n}, depth {w.depth})")
        assert st[k]["status"] == 0
        orc = O.Multilevel(w.pos, w.q, w.box, w.depth, w.p, setup="multipole" if flags else "fmm")
        tr_o = orc.run(w.seed, k, 0, steps, 1.0, w.max_step)
        _check_trace(w, tr_o, tr["idx"][k], tr["newpos"][k], tr["acc"][k], tr["dE"][k])
        assert tr_o["acc"].sum() > 50
        assert np.array_equal(chains[k].positions(), orc.positions())
        if not flags:
            # the energy of the maintained expansions (the multipole
            # variant's is not symmetric between the charges: compared as
            # the running sum instead)
            assert chains[k].energy() == pytest.approx(orc.energy(), rel=1e-10)
        _expansions_close(chains[k], orc, w, multipole=bool(flags))
        orc.close()
        chains[k].close()


@pytest.mark.parametrize("name", ["medium", "small"])
def test_whole_gpu_workload_matches_oracle(name):
    from paper_2006_16622_amd import Chain, run_chains
    wl = W.medium() if name == "medium" else W.small()
    steps = 400 if name == "medium" else wl.steps
    say(f"[measured] {wl.name}: gpu setup and {steps} whole-GPU steps")
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    st, tr = run_chains([gpu], steps, wl.seed, wl.beta, wl.max_step, mode=2, traces=True)
    assert st[0]["status"] == 0
    say(f"[measured] {wl.name}: oracle")
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    tr_o = orc.run(wl.seed, 0, 0, steps, wl.beta, wl.max_step)
    _check_trace(wl, tr_o, tr["idx"][0], tr["newpos"][0], tr["acc"][0], tr["dE"][0])
    assert np.array_equal(gpu.positions(), orc.positions())
    assert gpu.energy() == pytest.approx(orc.energy(), rel=1e-10)
    _expansions_close(gpu, orc, wl, multipole=False)
