"""GPU parity of the volume move (fmm_mc_rescale, fmm_mc_rescale_undo)
against the oracle: after some Metropolis steps, the box is scaled by s.

* dE equals the difference of the oracle's energies of the scaled and the
  current configuration (both freshly initialised) within 1e-10 of |U|, and
  the closed form dE = U (1/s - 1) of a homogeneous energy;
* the scaled positions are those the oracle forms (x s, wrapped) bit for
  bit, and the chain then runs as the oracle in the new box (indices,
  positions, decisions bit-exact, dE within 1e-10);
* undo restores every position bit for bit, the energy is the fresh energy
  of the state before, and the chain runs on as the oracle in the old box;
  an undo after another call is refused;
* on a small rock-salt crystal dE agrees with the Ewald oracle's energy
  difference to truncation."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import dE_close

pytestmark = pytest.mark.gpu

ESTATE = -8


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _run_matches(gpu, orc, wl, steps, seed, max_step, t0=0):
    from paper_2006_16622_amd import run_chains
    st, tr = run_chains([gpu], steps, seed, wl.beta, max_step, t0=t0, traces=True)
    to = orc.run(seed, 0, t0, steps, wl.beta, max_step)
    assert st[0]["status"] == 0
    assert np.array_equal(tr["idx"][0], to["idx"])
    assert np.array_equal(tr["newpos"][0], to["newpos"])
    assert np.array_equal(tr["acc"][0], to["acc"])
    # free space: moves out of the box have dE = +inf on both sides
    fin = np.isfinite(to["dE"])
    assert np.array_equal(np.isfinite(tr["dE"][0]), fin)
    rms = np.sqrt(np.mean(to["dE"][fin] ** 2))
    assert dE_close(tr["dE"][0][fin], to["dE"][fin], rms).all()
    assert np.array_equal(gpu.positions(), orc.positions())


@pytest.mark.parametrize("s,free", [(1.07, False), (0.91, False), (1.2, True)])
def test_rescale_matches_oracle_and_closed_form(s, free):
    from paper_2006_16622_amd import FMM_MC_FREE_SPACE, Chain, FmmMcError
    wl = W.uniform(1000, 3, 8, 0.03, seed=81, key=90)
    flags = FMM_MC_FREE_SPACE if free else 0
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=flags)
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p, free_space=free)
    say(f"[volume] s={s} free={free}: 150 steps in the unit box")
    _run_matches(gpu, orc, wl, 150, wl.seed, wl.max_step)
    pos = gpu.positions()
    u_old = O.Multilevel(pos, wl.q, 1.0, wl.depth, wl.p, free_space=free).energy()
    dE = gpu.rescale(s)
    scaled = O.Multilevel(pos * s, wl.q, s, wl.depth, wl.p, free_space=free)
    u_new = scaled.energy()
    assert abs(dE - (u_new - u_old)) <= 1e-10 * abs(u_old)
    assert abs(dE - u_old * (1.0 / s - 1.0)) <= 1e-10 * abs(u_old)
    assert np.array_equal(gpu.positions(), scaled.positions())
    assert gpu.running_energy() == pytest.approx(u_new, rel=1e-10)
    say("[volume] 150 steps in the scaled box")
    _run_matches(gpu, scaled, wl, 150, wl.seed + 1, wl.max_step * s)
    with pytest.raises(FmmMcError) as e:
        gpu.rescale_undo()
    assert e.value.code == ESTATE


def test_rescale_undo_restores_the_state():
    from paper_2006_16622_amd import Chain
    wl = W.uniform(1000, 3, 8, 0.03, seed=82, key=91)
    gpu = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    orc = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    _run_matches(gpu, orc, wl, 100, wl.seed, wl.max_step)
    pos = gpu.positions()
    gpu.rescale(1.11)
    gpu.rescale_undo()
    assert np.array_equal(gpu.positions(), pos)
    fresh = O.Multilevel(pos, wl.q, 1.0, wl.depth, wl.p)
    assert gpu.running_energy() == pytest.approx(fresh.energy(), rel=1e-10)
    assert gpu.energy() == pytest.approx(fresh.energy(), rel=1e-10)
    say("[volume] after undo: 150 steps in the unit box")
    _run_matches(gpu, fresh, wl, 150, wl.seed, wl.max_step, t0=100)


def test_rescale_rock_salt_against_ewald():
    from paper_2006_16622_amd import Chain
    pos, q = W.rocksalt_lattice(10)
    pos = np.mod(pos + np.random.default_rng(83).normal(0.0, 0.001, pos.shape), 1.0)
    gpu = Chain(pos, q, 1.0, 3, 12)
    s = 1.03
    dE = gpu.rescale(s)
    e0 = O.Ewald(pos, q, 1.0).energy()
    e1 = O.Ewald(np.mod(pos * s, s), q, s).energy()
    say(f"[volume] rock salt n=1000: dE {dE:.6f}, Ewald {e1 - e0:.6f}")
    assert abs(dE - (e1 - e0)) <= 1e-5 * abs(e0)
