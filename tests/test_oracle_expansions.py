"""Pins of the oracle's harmonics and expansion operators against the
mathematics (not against the oracle itself): scipy's Legendre functions,
the Legendre addition theorem, brute-force 1/r sums, and the exactness of
M2M / L2L / M2L-of-a-monopole."""
import numpy as np
import pytest
from scipy.special import eval_legendre, factorial, lpmv

import oracle as O

RNG = np.random.default_rng(12345)


def _sph(v):
    r = np.linalg.norm(v)
    return r, np.arccos(v[2] / r), np.arctan2(v[1], v[0])


@pytest.mark.parametrize("theta,phi", [(0.3, 0.2), (1.1, -2.5), (2.9, 3.0), (np.pi / 2, 0.7)])
def test_ylm_matches_scipy_without_condon_shortley(theta, phi):
    # Sec. 3.2: Y_n^m = sqrt((n-|m|)!/(n+|m|)!) P_n^|m|(cos) e^{im phi}; scipy's lpmv
    # carries the Condon-Shortley phase (-1)^m, removed here
    nmax = 20
    Y = O.ylm(nmax, theta, phi)
    for n in range(nmax + 1):
        for m in range(-n, n + 1):
            am = abs(m)
            ref = (np.sqrt(factorial(n - am) / factorial(n + am)) * lpmv(am, n, np.cos(theta))
                   * (-1) ** am * np.exp(1j * m * phi))
            assert abs(Y[O.idx(n, m)] - ref) < 1e-13 * max(1.0, abs(ref))


def test_ylm_pole_and_conjugate_symmetry():
    Y = O.ylm(12, 0.0, 0.0)
    for n in range(13):
        assert Y[O.idx(n, 0)] == pytest.approx(1.0, abs=1e-15)
        for m in range(1, n + 1):
            assert abs(Y[O.idx(n, m)]) < 1e-15
    Y = O.ylm(12, 0.9, 1.7)
    for n in range(13):
        for m in range(1, n + 1):
            assert Y[O.idx(n, -m)] == np.conj(Y[O.idx(n, m)])


def test_legendre_addition_theorem():
    # sum_m Y_n^{-m}(a) Y_n^m(b) = P_n(cos gamma): the identity behind every
    # expansion of Sec. 3.2 (no 4 pi/(2n+1) factor in this normalisation)
    for _ in range(5):
        a = RNG.normal(size=3)
        b = RNG.normal(size=3)
        _, ta, pa = _sph(a)
        _, tb, pb = _sph(b)
        Ya, Yb = O.ylm(15, ta, pa), O.ylm(15, tb, pb)
        cg = a @ b / np.linalg.norm(a) / np.linalg.norm(b)
        for n in range(16):
            s = sum(Ya[O.idx(n, -m)] * Yb[O.idx(n, m)] for m in range(-n, n + 1))
            assert abs(s - eval_legendre(n, cg)) < 1e-13


def _cluster(n, centre, radius):
    pts = centre + RNG.uniform(-radius, radius, size=(n, 3))
    return pts, RNG.normal(size=n)


def test_p2m_m2p_converges_to_direct_sum():
    src, q = _cluster(8, np.zeros(3), 0.5)
    x = np.array([2.0, -1.5, 1.0])
    direct = sum(qi / np.linalg.norm(x - s) for s, qi in zip(src, q))
    errs = []
    for p in (2, 4, 8, 16):
        M = sum(O.p2m(p, qi, s, np.zeros(3)) for s, qi in zip(src, q))
        errs.append(abs(O.m2p(p, M, x, np.zeros(3)) - direct))
    assert errs[-1] < 1e-10 * abs(direct) + 1e-12
    assert all(e1 < e0 for e0, e1 in zip(errs, errs[1:]))


def test_p2l_l2p_converges_to_direct_sum():
    src, q = _cluster(8, np.array([2.0, 1.0, -1.5]), 0.4)
    x = np.array([0.1, -0.2, 0.15])
    direct = sum(qi / np.linalg.norm(x - s) for s, qi in zip(src, q))
    errs = []
    for p in (2, 4, 8, 16):
        L = sum(O.p2l(p, qi, s, np.zeros(3)) for s, qi in zip(src, q))
        errs.append(abs(O.l2p(p, L, x, np.zeros(3)) - direct))
    assert errs[-1] < 1e-10 * abs(direct)
    assert all(e1 < e0 for e0, e1 in zip(errs, errs[1:]))


@pytest.mark.parametrize("p", [4, 8, 12])
def test_m2m_is_exact(p):
    # shifting a multipole expansion is exact for the first p degrees:
    # M2M(P2M about the child centre) == P2M about the parent centre
    src, q = _cluster(6, np.array([0.1, -0.05, 0.08]), 0.1)
    child, parent = np.array([0.125, -0.125, 0.125]), np.zeros(3)
    Mc = sum(O.p2m(p, qi, s, child) for s, qi in zip(src, q))
    Mp = sum(O.p2m(p, qi, s, parent) for s, qi in zip(src, q))
    Mt = O.m2m(p, Mc, child - parent)
    assert np.abs(Mt - Mp).max() < 1e-13 * np.abs(Mp).max()


def test_l2l_is_exact_for_degree_p():
    p = 10
    src, q = _cluster(5, np.array([3.0, 0.0, -2.0]), 0.3)
    c0 = np.zeros(3)
    L0 = sum(O.p2l(p, qi, s, c0) for s, qi in zip(src, q))
    c1 = np.array([0.1, 0.05, -0.07])
    L1 = O.l2l(p, L0, c0 - c1)
    for _ in range(5):
        x = c1 + RNG.uniform(-0.05, 0.05, 3)
        assert O.l2p(p, L1, x, c1) == pytest.approx(O.l2p(p, L0, x, c0), rel=1e-13)


def test_m2l_of_centred_monopole_is_p2l():
    p = 12
    s = np.array([2.0, -3.0, 1.5])
    M = O.p2m(p, 0.7, s, s)  # pure monopole about its own centre
    L = O.m2l(p, M, s - np.zeros(3))
    Lref = O.p2l(p, 0.7, s, np.zeros(3))
    assert np.abs(L - Lref).max() < 1e-15 * np.abs(Lref).max() * 10


def test_m2l_converges_to_direct_sum():
    cs = np.array([3.0, 1.0, -2.0])
    src, q = _cluster(8, cs, 0.4)
    x = np.array([0.1, 0.2, -0.1])
    direct = sum(qi / np.linalg.norm(x - s) for s, qi in zip(src, q))
    errs = []
    for p in (2, 4, 8, 14):
        M = sum(O.p2m(p, qi, s, cs) for s, qi in zip(src, q))
        L = O.m2l(p, M, cs)
        errs.append(abs(O.l2p(p, L, x, np.zeros(3)) - direct))
    assert errs[-1] < 1e-9 * abs(direct)
    assert all(e1 < e0 for e0, e1 in zip(errs, errs[1:]))


def test_m2l_interaction_energy_is_symmetric():
    # the interaction energy of two clusters computed through M2L from A to B
    # equals the one from B to A (a transposed or mis-signed operator fails)
    p = 10
    ca, cb = np.zeros(3), np.array([2.0, 0.5, -1.0])
    A, qa = _cluster(5, ca, 0.3)
    B, qb = _cluster(5, cb, 0.3)
    Ma = sum(O.p2m(p, qi, s, ca) for s, qi in zip(A, qa))
    Mb = sum(O.p2m(p, qi, s, cb) for s, qi in zip(B, qb))
    Lb = O.m2l(p, Ma, ca - cb)
    La = O.m2l(p, Mb, cb - ca)
    e_ab = sum(qi * O.l2p(p, Lb, s, cb) for s, qi in zip(B, qb))
    e_ba = sum(qi * O.l2p(p, La, s, ca) for s, qi in zip(A, qa))
    direct = sum(qi * qj / np.linalg.norm(si - sj) for si, qi in zip(A, qa) for sj, qj in zip(B, qb))
    assert e_ab == pytest.approx(e_ba, rel=1e-12)
    assert e_ab == pytest.approx(direct, rel=1e-5)
