"""Pins of the oracle's energies in a box of side other than 1, as a volume
move (a scaling of every position and of the box) uses them. The Coulomb
energy is homogeneous of degree -1 in length: U(s r, s a) = U(r, a) / s,
for the exact periodic sum and for the multilevel method alike (all its
geometry scales with the box). This fixes the energy change of a volume
move in closed form, dE = U (1/s - 1), and it holds for both oracles; the
multilevel energy in the scaled box also agrees with Ewald to truncation."""
import numpy as np
import pytest

import oracle as O


def _system(n, seed):
    g = np.random.default_rng(seed)
    pos = g.uniform(0, 1, (n, 3))
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    return pos, q


@pytest.mark.parametrize("s", [0.83, 1.07, 2.5])
def test_multilevel_energy_scales_as_one_over_length(s):
    pos, q = _system(300, 71)
    u = O.Multilevel(pos, q, 1.0, 2, 8).energy()
    us = O.Multilevel(pos * s, q, s, 2, 8).energy()
    assert us == pytest.approx(u / s, rel=1e-11)


@pytest.mark.parametrize("s", [0.83, 2.5])
def test_multilevel_free_space_energy_scales(s):
    pos, q = _system(200, 72)
    u = O.Multilevel(pos, q, 1.0, 2, 8, free_space=True).energy()
    us = O.Multilevel(pos * s, q, s, 2, 8, free_space=True).energy()
    assert us == pytest.approx(u / s, rel=1e-11)


def test_ewald_energy_scales_and_matches_multilevel_in_scaled_box():
    pos, q = _system(300, 73)
    s = 1.3
    e = O.Ewald(pos, q, 1.0).energy()
    es = O.Ewald(pos * s, q, s).energy()
    assert es == pytest.approx(e / s, rel=1e-11)
    # the multilevel method in the scaled box converges to the same energy
    # as p grows (relative errors 8.4e-6 and 1.3e-6 here, as in the unit box)
    err = {p: abs(O.Multilevel(pos * s, q, s, 2, p).energy() - es) / abs(es) for p in (12, 16)}
    assert err[12] < 2e-5 and err[16] < 3e-6 and err[16] < err[12] / 4
