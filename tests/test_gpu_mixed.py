"""The mixed-precision mode (FMM_MC_MIXED) against the FP64 oracle and the
Ewald oracle.

In this mode the setup M2L runs on FP32 matrix-core tiles, and the solid
harmonics of L2P (propose) and P2L (accept) and the near-field inverse
distances are evaluated in FP32. The local coefficients, every sum, the dE
subtraction and the periodic lattice term stay FP64. So the results are
not bit-exact against the oracle. Each test states its error bound and
prints the measured error:
* the setup's local expansions are within 2e-5 of each level's largest
  coefficient;
* proposals are within 1e-4 of RMS dE;
* a run's decisions equal the oracle's wherever |u - exp(-beta dE)| exceeds
  that error;
* against Ewald at p = 12, the relative RMS error meets the same 1e-5 gate
  as the FP64 path.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import real_layout

pytestmark = pytest.mark.gpu

MIXED = 0x1


def say(*a):
    print(*a, file=sys.stderr, flush=True)


CASES = {
    "n1000_d3_p8": W.small,
    "n2000_d3_p12": lambda: W.uniform(2000, 3, 12, 0.04, seed=51, key=13),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    from paper_2006_16622_amd import Chain
    wl = CASES[request.param]()
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=MIXED)
    return request.param, wl, orc, gpu


def test_mixed_setup_expansions(case):
    name, wl, orc, gpu = case
    worst = 0.0
    for level in range(2, wl.depth + 2):
        got = gpu.locals(level)
        cells = range(min(64, 8 ** (level - 1)))
        ref = np.array([real_layout(orc.local(level, c), wl.p) for c in cells])
        err = np.abs(got[list(cells)] - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
    say(f"[mixed] {name}: setup expansions, max error / level max = {worst:.2e}")
    assert worst < 2e-5


def test_mixed_proposals(case):
    name, wl, orc, gpu = case
    pos = orc.positions()
    de, ref = [], []
    for t in range(80):
        i, d, _ = O.draw(wl.seed, 0, t, wl.n, wl.max_step)
        de.append(gpu.propose(i, pos[i] + d))
        ref.append(orc.propose(i, pos[i] + d))
    de, ref = np.array(de), np.array(ref)
    rms = np.sqrt(np.mean(ref ** 2))
    err = np.abs(de - ref).max() / rms
    say(f"[mixed] {name}: proposals, max |dE - dE_oracle| / RMS = {err:.2e}")
    assert err < 1e-4


@pytest.mark.parametrize("mode", [0, 1])
def test_mixed_run_follows_oracle(case, mode):
    from paper_2006_16622_amd import Chain, run_chains
    name, wl, _, _ = case
    steps = 150
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    tr = orc.run(wl.seed, 0, 0, steps, wl.beta, wl.max_step)
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=MIXED)
    st, gt = run_chains([gpu], steps, wl.seed, wl.beta, wl.max_step, mode=mode, traces=True)
    assert st[0]["status"] == 0
    rms = np.sqrt(np.mean(tr["dE"] ** 2))
    margin = np.abs(tr["u"] - np.exp(-wl.beta * tr["dE"]))
    # up to the first decision that could flip at the mixed-precision error,
    # the trajectories are the same
    k = int(np.argmax(margin < 1e-3)) if (margin < 1e-3).any() else steps
    assert np.array_equal(gt["idx"][0][:k], tr["idx"][:k])
    assert np.array_equal(gt["acc"][0][:k], tr["acc"][:k])
    err = np.abs(gt["dE"][0][:k] - tr["dE"][:k]).max() / rms
    say(f"[mixed] {name} mode {mode}: {k} steps compared, max dE error / RMS = {err:.2e}")
    assert err < 1e-4 and k > 50


def test_mixed_chain_prefix_meets_ewald_gate():
    from paper_2006_16622_amd import Chain, run_chains
    wl = W.medium()
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=MIXED)
    steps = 2000
    st, tr = run_chains([gpu], steps, wl.seed, wl.beta, wl.max_step, mode=0, traces=True)
    assert st[0]["status"] == 0
    ew = O.Ewald(wl.pos, wl.q, wl.box)
    ref = np.empty(steps)
    for t in range(steps):
        ref[t] = ew.propose(int(tr["idx"][0][t]), tr["newpos"][0][t])
        if tr["acc"][0][t]:
            ew.accept(int(tr["idx"][0][t]), tr["newpos"][0][t])
    err = np.sqrt(np.mean((tr["dE"][0] - ref) ** 2)) / np.sqrt(np.mean(ref ** 2))
    say(f"[mixed] {wl.name}: chain prefix of {steps} against Ewald, relative RMS error {err:.3e}")
    assert err < 1e-5
