"""fmm_mc_run_noalloc (the entry point for callers that cannot allocate)
against fmm_mc_run, through the C ABI: two calls in a row on batched chains
(one workgroup each), the second with fewer chains and steps, and one call
on a whole-GPU chain; every result equal bit for bit (the two share their
kernels). Plus its limit: more chains than FMM_MC_NOALLOC_MAX_CHAINS is
refused before anything is touched, and so is a run with re-setups."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

ENOMEM, EINVAL = -5, -1


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _chains(wls):
    from paper_2006_16622_amd import Chain
    return [Chain(w.pos, w.q, w.box, w.depth, w.p) for w in wls]


def _same(st_a, tr_a, st_b, tr_b, ca, cb):
    for a, b in zip(st_a, st_b):
        for k in ("proposed", "accepted", "singular", "dE_sum", "energy", "status"):
            assert a[k] == b[k], k
    for k in ("idx", "newpos", "acc", "dE"):
        assert np.array_equal(tr_a[k], tr_b[k]), k
    for x, y in zip(ca, cb):
        assert np.array_equal(x.positions(), y.positions())
        assert x.running_energy() == y.running_energy()


def test_noalloc_matches_run_on_two_calls():
    from paper_2006_16622_amd import run_chains
    specs = [(600, 2, 12, 0.05), (1500, 2, 12, 0.04), (3000, 3, 12, 0.03), (800, 2, 8, 0.05),
             (2000, 3, 12, 0.03), (400, 2, 12, 0.06)]
    wls = [W.uniform(n, d, 12, s, seed=31, key=70 + i) for i, (n, d, p, s) in enumerate(specs)]
    ref = _chains(wls)
    new = _chains(wls)
    steps = [w.max_step for w in wls]
    say("[noalloc] call 1: 6 chains x 150 steps")
    st_r, tr_r = run_chains(ref, 150, 5, 1.0, steps, mode=1, traces=True)
    st_n, tr_n = run_chains(new, 150, 5, 1.0, steps, mode=1, traces=True, noalloc=True)
    _same(st_r, tr_r, st_n, tr_n, ref, new)
    assert sum(s["accepted"] for s in st_n) > 100
    say("[noalloc] call 2: 3 chains x 60 steps")
    st_r, tr_r = run_chains(ref[:3], 60, 6, 1.0, steps[:3], t0=150, mode=1, traces=True)
    st_n, tr_n = run_chains(new[:3], 60, 6, 1.0, steps[:3], t0=150, mode=1, traces=True, noalloc=True)
    _same(st_r, tr_r, st_n, tr_n, ref[:3], new[:3])
    say("[noalloc] call 3: one chain on the whole GPU")
    st_r, tr_r = run_chains(ref[2:3], 80, 7, 1.0, steps[2], t0=210, mode=2, traces=True)
    st_n, tr_n = run_chains(new[2:3], 80, 7, 1.0, steps[2], t0=210, mode=2, traces=True, noalloc=True)
    _same(st_r, tr_r, st_n, tr_n, ref[2:3], new[2:3])
    for c in ref + new:
        c.close()


def test_noalloc_refuses_beyond_its_limits():
    from paper_2006_16622_amd import binding, run_chains, FmmMcError
    lib = binding.load_library()
    opts = binding.RunOpts()
    opts.beta = 1.0
    opts.max_step = 0.01
    maxc = 1024  # FMM_MC_NOALLOC_MAX_CHAINS
    hs = (ctypes.c_void_p * (maxc + 1))()
    stats = (binding.Stats * (maxc + 1))()
    assert lib.fmm_mc_run_noalloc(hs, maxc + 1, 10, 1, ctypes.byref(opts), stats) == ENOMEM
    wl = W.uniform(300, 2, 6, 0.05, seed=32, key=80)
    (c,) = _chains([wl])
    with pytest.raises(FmmMcError) as e:
        run_chains([c], 10, 1, 1.0, wl.max_step, resetup_every=5, noalloc=True)
    assert e.value.code == EINVAL
    c.close()
