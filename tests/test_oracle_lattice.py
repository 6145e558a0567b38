"""Pin of the oracle's periodic lattice sums (Sec. 3.4; the operator R whose
definition the paper defers to another text) by an independent method:
brute-force cube-shell summation, extrapolated in the shell index."""
import numpy as np
import pytest
from scipy.special import factorial, lpmv

import oracle as O


def _shell_partial_sums(K, l, m):
    r = np.arange(-K, K + 1)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    X, Y, Z = X.ravel(), Y.ravel(), Z.ravel()
    inf = np.maximum(np.maximum(abs(X), abs(Y)), abs(Z))
    sel = inf >= 2
    X, Y, Z, inf = X[sel], Y[sel], Z[sel], inf[sel]
    R = np.sqrt(X * X + Y * Y + Z * Z)
    am = abs(m)
    Yv = (np.sqrt(factorial(l - am) / factorial(l + am)) * lpmv(am, l, Z / R) * (-1) ** am
          * np.exp(1j * m * np.arctan2(Y, X)))
    t = Yv / R ** (l + 1)
    per_shell = np.bincount(inf, weights=t.real, minlength=K + 1)
    return np.cumsum(per_shell)[2:]  # partial sums for K' = 2..K


def _extrapolate(partial, K):
    Ks = np.arange(2, K + 1).astype(float)
    sel = Ks >= 12
    A = np.stack([np.ones(sel.sum())] + [Ks[sel] ** -j for j in (2, 3, 4, 5, 6)], 1)
    return np.linalg.lstsq(A, partial[sel], rcond=None)[0][0]


@pytest.mark.parametrize("l,m", [(4, 0), (4, 4), (6, 0), (6, 4), (8, 0), (8, 8)])
def test_far_lattice_sums_match_cube_shell_brute_force(l, m):
    S = O.lattice_sums(8)
    ref = _extrapolate(_shell_partial_sums(56, l, m), 56)
    assert S[O.idx(l, m)].real == pytest.approx(ref, abs=1e-10)
    assert abs(S[O.idx(l, m)].imag) < 1e-14


def test_lattice_sum_symmetries():
    S = O.lattice_sums(16)
    for l in range(17):
        for m in range(-l, l + 1):
            v = S[O.idx(l, m)]
            if l <= 2 or l % 2 == 1 or m % 4 != 0:
                # l<=2: neutral cell / inversion / cube-order cubic symmetry;
                # odd l: inversion; m not = 0 mod 4: four-fold axis
                assert abs(v) < 1e-14, (l, m, v)
    assert abs(S[O.idx(4, 0)]) > 0.1


def test_lattice_sums_scale_with_box():
    S1 = O.lattice_sums(10, 1.0)
    S2 = O.lattice_sums(10, 2.5)
    for l in range(11):
        for m in range(-l, l + 1):
            assert S2[O.idx(l, m)] == pytest.approx(S1[O.idx(l, m)] / 2.5 ** (l + 1), abs=1e-16)


def test_full_lattice_sum_z4():
    # the full sum over nu != 0 of P_4(cos)/|nu|^5 (cube order) from the far
    # part plus the 26 nearest images, against brute force including them
    S = O.lattice_sums(4)
    near = 0.0
    import itertools
    for nu in itertools.product((-1, 0, 1), repeat=3):
        if any(nu):
            v = np.array(nu, float)
            r = np.linalg.norm(v)
            c = v[2] / r
            near += (35 * c ** 4 - 30 * c ** 2 + 3) / 8 / r ** 5
    full = S[O.idx(4, 0)].real + near
    ref = _extrapolate(_shell_partial_sums(56, 4, 0), 56) + near
    assert full == pytest.approx(ref, abs=1e-10)
    assert full == pytest.approx(3.1082266827, abs=1e-9)


@pytest.mark.parametrize("l,m", [(16, 0), (16, 4), (24, 0), (24, 8), (32, 4), (40, 0), (48, 0), (48, 12)])
def test_high_degree_lattice_sums_to_absolute_precision(l, m):
    # for l >= 16 the far sum converges absolutely and fast (the tail beyond
    # cube shell K is O(K^(2-l))), so plain shell sums to K = 24 are exact to
    # rounding; the Ewald-split evaluation keeps an absolute error of about
    # 1e-15 at every degree, which is the floor of the highest sums (S_48 is
    # about 4e-15)
    S = O.lattice_sums(48)
    ref = _shell_partial_sums(24, l, m)[-1]
    assert abs(S[O.idx(l, m)].real - ref) < 1e-14
