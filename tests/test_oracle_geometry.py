"""Pins of the oracle's octree geometry against the definitions of Sec. 3.1
and Sec. 3.4 checked by brute force."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
OCTS = list(itertools.product((0, 1), repeat=3))


def _il_brute(alpha):
    """IL(alpha) = children(N_b(parent(alpha))) minus alpha and N_b(alpha),
    as sets of integer cell coordinates (Sec. 3.1), with no offset algebra."""
    parent = tuple(a // 2 for a in alpha)
    out = set()
    for e in itertools.product((-1, 0, 1), repeat=3):
        pn = tuple(p + ei for p, ei in zip(parent, e))
        for c in itertools.product((0, 1), repeat=3):
            out.add(tuple(2 * x + ci for x, ci in zip(pn, c)))
    near = {tuple(a + ei for a, ei in zip(alpha, e)) for e in itertools.product((-1, 0, 1), repeat=3)}
    return out - near


@pytest.mark.parametrize("oct_", OCTS)
def test_il_size_and_definition(oct_):
    offs = O.il_offsets(oct_)
    assert len(offs) == GOLD["interaction_list_size"]["value"] == 6 ** 3 - 3 ** 3
    alpha = tuple(10 + o for o in oct_)
    brute = {tuple(int(a + o) for a, o in zip(alpha, off)) for off in offs}
    assert brute == _il_brute(alpha)


def test_il_distinct_offsets_and_symmetry():
    allo = set()
    for oc in OCTS:
        for off in O.il_offsets(oc):
            allo.add(tuple(off))
            # beta in IL(alpha)  <=>  alpha in IL(beta)
            oc2 = tuple((o + d) % 2 for o, d in zip(oc, off))
            assert tuple(-off) in {tuple(x) for x in O.il_offsets(oc2)}
    assert len(allo) == 316


@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_near_and_interaction_lists_tile_extended_domain(L):
    # Sec. 3.4: with periodic images, the near cells of a leaf plus the
    # interaction lists of the leaf and all its ancestors on levels 2..L
    # cover every leaf-sized cell of the 27-box extended domain exactly once
    nL = 2 ** (L - 1)
    rng = np.random.default_rng(L)
    for _ in range(3):
        leaf = tuple(int(v) for v in rng.integers(0, nL, 3))
        covered = {}
        for e in itertools.product((-1, 0, 1), repeat=3):
            c = tuple(a + ei for a, ei in zip(leaf, e))
            covered[c] = covered.get(c, 0) + 1
        for l in range(2, L + 1):
            scale = 2 ** (L - l)
            anc = tuple(a // scale for a in leaf)
            for off in O.il_offsets(tuple(a & 1 for a in anc)):
                b = tuple(a + o for a, o in zip(anc, off))
                for sub in itertools.product(range(scale), repeat=3):
                    c = tuple(bi * scale + si for bi, si in zip(b, sub))
                    covered[c] = covered.get(c, 0) + 1
        assert all(v == 1 for v in covered.values())
        assert len(covered) == 27 * 8 ** (L - 1)
        assert all(-nL <= min(c) and max(c) < 2 * nL for c in covered)


def test_cells_per_level():
    for l in range(1, 7):
        n = 2 ** (l - 1)
        assert n ** 3 == 8 ** (l - 1)


def test_wrap_edge_cases():
    assert O.wrap(0.25, 1.0) == 0.25
    assert O.wrap(1.0, 1.0) == 0.0
    assert O.wrap(-1e-300, 1.0) == 0.0  # 1 - tiny rounds to 1 -> 0
    assert O.wrap(-0.25, 1.0) == 0.75
    assert O.wrap(1.25, 1.0) == 0.25
    assert O.wrap(3.5, 2.0) == 1.5
    x = np.nextafter(1.0, 0.0)
    assert O.wrap(x, 1.0) == x


def test_cell_coord_edges():
    assert O.cell_coord(0.0, 1.0, 8) == 0
    assert O.cell_coord(0.125, 1.0, 8) == 1  # a point on a face belongs to the upper cell
    assert O.cell_coord(np.nextafter(0.125, 0), 1.0, 8) == 0
    assert O.cell_coord(np.nextafter(1.0, 0), 1.0, 8) == 7


def test_self_image_constant_closed_form():
    terms = GOLD["self_image_terms"]
    v = sum(c / np.sqrt(d) for c, d in zip(terms["value"], terms["divisors"]))
    brute = sum(1.0 / np.linalg.norm(nu) for nu in itertools.product((-1, 0, 1), repeat=3) if any(nu))
    assert O.self_image_constant() == pytest.approx(v, rel=1e-15)
    assert brute == pytest.approx(v, rel=1e-14)
    assert v == pytest.approx(19.104083527755577, rel=1e-15)
