"""Pins of the Ewald oracle (O1): rock-salt Madelung energy, independence of
the splitting parameter, brute-force cube-ordered sums on tiny systems with
the tin-foil surface term, and move consistency."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
MADELUNG = 1.7475645946331822  # rock-salt Madelung constant


def test_madelung_constant_value_matches_statement():
    assert MADELUNG == pytest.approx(GOLD["madelung_nacl"]["value"], abs=5e-7)


@pytest.mark.parametrize("side", [2, 4, 10])
def test_rocksalt_madelung_energy(side):
    pos, q = workloads.rocksalt_lattice(side)
    e = O.Ewald(pos, q, 1.0)
    s = 1.0 / side
    ref = -(len(q) / 2.0) * MADELUNG / s
    assert e.energy() == pytest.approx(ref, rel=1e-12)


def _random_system(n, seed):
    g = np.random.default_rng(seed)
    pos = g.uniform(0, 1, (n, 3))
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    return pos, q


def test_alpha_independence():
    pos, q = _random_system(40, 3)
    e1 = O.Ewald(pos, q, 1.0)
    a, rc, km = O.ewald_parameters(1.0, 32.0, 0.45)
    e2 = O.Ewald(pos, q, 1.0, alpha=a, rc=rc, kmax=km)
    assert e1.alpha != e2.alpha
    assert e1.energy() == pytest.approx(e2.energy(), rel=1e-12)
    rn = pos[5] + np.array([0.03, -0.02, 0.01])
    assert e1.propose(5, rn) == pytest.approx(e2.propose(5, rn), rel=1e-11, abs=1e-11)


def _brute_cube_energy(pos, q, K=40):
    """Cube-ordered lattice sum 1/2 sum_ij sum_{|nu|_inf<=K}' q_i q_j/|r_i-r_j+nu|,
    partial sums per shell, extrapolated in K."""
    r = np.arange(-K, K + 1)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    nu = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(float)
    inf = np.abs(nu).max(1).astype(int)
    shell = np.zeros(K + 1)
    n = len(q)
    for i in range(n):
        for j in range(n):
            d = pos[i] - pos[j] + nu
            rr = np.sqrt((d * d).sum(1))
            w = np.where(rr > 0, 1.0 / np.where(rr > 0, rr, 1.0), 0.0)
            shell += 0.5 * q[i] * q[j] * np.bincount(inf, weights=w, minlength=K + 1)
    partial = np.cumsum(shell)
    Ks = np.arange(K + 1).astype(float)
    sel = Ks >= 10
    A = np.stack([np.ones(sel.sum())] + [Ks[sel] ** -j for j in (2, 3, 4, 5, 6)], 1)
    return np.linalg.lstsq(A, partial[sel], rcond=None)[0][0]


@pytest.mark.parametrize("n,seed", [(2, 1), (8, 2), (12, 7)])
def test_brute_force_cube_sum_with_tinfoil_surface_term(n, seed):
    # tin-foil Ewald == cube-ordered direct lattice sum - (2 pi / 3V) |D|^2
    pos, q = _random_system(n, seed)
    D = (q[:, None] * pos).sum(0)
    ucube = _brute_cube_energy(pos, q)
    e = O.Ewald(pos, q, 1.0)
    assert e.energy() == pytest.approx(ucube - 2 * np.pi / 3.0 * (D @ D), abs=1e-8)
    assert abs(D @ D) > 1e-3  # the surface term is exercised


def test_propose_equals_energy_difference_and_antisymmetry():
    pos, q = _random_system(30, 11)
    e = O.Ewald(pos, q, 1.0)
    u0 = e.energy()
    rn = np.mod(pos[3] + np.array([0.2, -0.35, 0.6]), 1.0)
    de = e.propose(3, rn)
    e.accept(3, rn)
    u1 = e.energy()
    assert de == pytest.approx(u1 - u0, abs=1e-11)
    back = e.propose(3, pos[3])
    assert back == pytest.approx(-de, abs=1e-11)
    # exact fresh recomputation of the moved state
    pos2 = pos.copy()
    pos2[3] = rn
    assert O.Ewald(pos2, q, 1.0).energy() == pytest.approx(u1, abs=1e-11)
