"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, validates arguments before touching the device, and its
host-built operators agree with the oracle's translation theorems."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from helpers import real_layout

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmm_mc.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2006_16622_amd import build, binding
    if build.is_stale():
        build.build()
    return binding.load_library()


def test_library_exports_every_declared_symbol(lib):
    names = set(re.findall(r"\b(fmm_mc_\w+)\s*\(", open(HEADER).read()))
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    from paper_2006_16622_amd import binding
    assert names == set(binding.SYMBOLS)


def test_workspace_bytes_validation(lib):
    out = ctypes.c_size_t()
    assert lib.fmm_mc_workspace_bytes(1000, 3, 8, 0, ctypes.byref(out)) == 0
    assert out.value > 1000 * 8
    for args in [(1, 3, 8), (1000, 0, 8), (1000, 8, 8), (1000, 3, -1), (1000, 3, 25)]:
        assert lib.fmm_mc_workspace_bytes(*args, 0, ctypes.byref(out)) == -1
    b3 = ctypes.c_size_t()
    lib.fmm_mc_workspace_bytes(10000, 4, 12, 0, ctypes.byref(b3))
    assert b3.value > out.value


def test_setup_rejects_bad_input_before_device_use(lib):
    from paper_2006_16622_amd import binding
    n = 4
    pos = np.random.default_rng(0).uniform(0, 1, (n, 3))
    q = np.array([1.0, -1.0, 1.0, -1.0])
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)  # aligned, never dereferenced on these paths
    d = binding._d

    def call(pos, q, box=1.0, levels=2, p=4, ws=1 << 30, ptr=fake):
        return lib.fmm_mc_setup(ctypes.byref(h), ptr, ws, None, len(q), d(pos), d(q), box, levels, p, 0)

    assert call(pos, np.array([1.0, 1.0, 1.0, -1.0])) == -3  # non-neutral
    bad = pos.copy()
    bad[1, 2] = np.nan
    assert call(bad, q) == -1
    assert call(pos, q, box=0.0) == -1
    assert call(pos, q, levels=0) == -1
    assert call(pos, q, p=30) == -1
    assert call(pos, q, ws=16) == -5  # workspace too small
    assert call(pos, q, ptr=ctypes.c_void_p((1 << 20) + 8)) == -1  # misaligned
    assert lib.fmm_mc_propose(None, 0, d(np.zeros(3)), d(np.zeros(1))) == -8
    assert lib.fmm_mc_strerror(-3) == b"charges do not sum to zero"


def _rand_sym(p, rng):
    c = np.zeros((p + 1) ** 2, complex)
    for n in range(p + 1):
        c[O.idx(n, 0)] = rng.normal()
        for m in range(1, n + 1):
            v = rng.normal() + 1j * rng.normal()
            c[O.idx(n, m)] = v
            c[O.idx(n, -m)] = np.conj(v)
    return c


@pytest.mark.parametrize("p", [3, 8, 12])
def test_library_operators_match_oracle_translation_theorems(lib, p):
    from paper_2006_16622_amd import host_operator
    rng = np.random.default_rng(p)
    for o in [(2, 0, 0), (3, -2, 1), (-2, -2, -2), (1, 3, -3)]:
        T = host_operator(0, p, o)
        M = _rand_sym(p, rng)
        ref = real_layout(O.m2l(p, M, np.array(o, float)), p)
        got = T.T @ real_layout(M, p)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    for oc in range(8):
        T = host_operator(1, p, (oc, 0, 0))
        M = _rand_sym(p, rng)
        d = np.array([0.5 * (oc & 1) - 0.25, 0.5 * ((oc >> 1) & 1) - 0.25, 0.5 * ((oc >> 2) & 1) - 0.25])
        ref = real_layout(O.m2m(p, M, d), p)
        scale = np.array([0.5 ** n for n in range(p + 1) for m in range(-n, n + 1)])
        got = T.T @ (real_layout(M, p) / scale)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    R = host_operator(2, p)
    K = _rand_sym(p, rng)
    ref = real_layout(O.lattice_apply(p, O.lattice_sums(2 * p), K), p)
    got = R @ real_layout(K, p)
    assert np.abs(got - ref).max() <= 1e-7 * np.abs(ref).max()
