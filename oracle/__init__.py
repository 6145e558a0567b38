"""CPU FP64 oracle of the multilevel local-expansion Monte Carlo method.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It shares no
code with the GPU library (``paper_2006_16622_amd``); the two meet only
through the seeded input generators in ``workloads.py``.

Two oracles (plain C, gcc -O2, no fast-math, no FP contraction):

* ``Multilevel`` -- the paper's method step by step in FP64
  (Sec. 3.2 Alg. L.1, L.2, L.3, Alg. 1; Sec. 3.4 periodic modifications).
* ``Ewald`` -- tin-foil Ewald summation with structure-factor updates, the
  O(sqrt N)-per-move comparator the paper names (Sec. 2, Sec. 5.3).

Plus the Philox4x64-10 proposal stream and the free functions of the
expansions (harmonics, P2M/P2L/L2P/M2P, M2M/M2L/L2L, lattice sums).

Complex coefficients use full storage, index n*n+n+m for m = -n..n.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "fmm_oracle.c"), os.path.join(_HERE, "ewald_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_ip = ctypes.POINTER(ctypes.c_int)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C99/C11, -O2, no fast-math, no FP
    contraction, so that wrap/locate/decision round exactly as IEEE)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-o", tmp] + _SRC + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or any(
            os.path.getmtime(s) > os.path.getmtime(_LIB_PATH) for s in _SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    sig = {
        "orc_ylm": (None, [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp]),
        "orc_p2m": (None, [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]),
        "orc_p2e": (None, [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]),
        "orc_p2l": (None, [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]),
        "orc_l2p": (ctypes.c_double, [ctypes.c_int, _dp, _dp, _dp]),
        "orc_m2p": (ctypes.c_double, [ctypes.c_int, _dp, _dp, _dp]),
        "orc_m2m": (None, [ctypes.c_int, _dp, _dp, _dp]),
        "orc_m2l": (None, [ctypes.c_int, _dp, _dp, _dp]),
        "orc_l2l": (None, [ctypes.c_int, _dp, _dp, _dp]),
        "orc_il_offsets": (ctypes.c_int, [_ip, _ip]),
        "orc_wrap": (ctypes.c_double, [ctypes.c_double, ctypes.c_double]),
        "orc_cell_coord": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_int]),
        "orc_lattice_sums": (None, [ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp]),
        "orc_lattice_apply": (None, [ctypes.c_int, _dp, _dp, _dp]),
        "orc_self_image_constant": (ctypes.c_double, []),
        "orc_philox4x64_10": (None, [_u64p, _u64p, _u64p]),
        "orc_draw": (None, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                            ctypes.c_double, _i64p, _dp, _dp]),
        "orc_create": (vp, [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_int, ctypes.c_int]),
        "orc_destroy": (None, [vp]),
        "orc_setup_fmm": (None, [vp, ctypes.c_int]),
        "orc_setup_direct": (None, [vp]),
        "orc_setup_none": (None, [vp]),
        "orc_setup_multipole": (None, [vp, ctypes.c_int]),
        "orc_set_free_space": (None, [vp]),
        "orc_get_multipole": (None, [vp, ctypes.c_int, ctypes.c_int, _dp]),
        "orc_propose": (ctypes.c_double, [vp, ctypes.c_int, _dp]),
        "orc_accept": (None, [vp, ctypes.c_int, _dp]),
        "orc_energy": (ctypes.c_double, [vp]),
        "orc_get_local": (None, [vp, ctypes.c_int, ctypes.c_int, _dp]),
        "orc_get_K": (None, [vp, _dp]),
        "orc_get_positions": (None, [vp, _dp]),
        "orc_leaf_of": (ctypes.c_int, [vp, ctypes.c_int]),
        "orc_run": (ctypes.c_int64, [vp, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                     _i64p, _dp, _dp, _dp, _u8p]),
        "ewd_create": (vp, [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_int]),
        "ewd_destroy": (None, [vp]),
        "ewd_energy": (ctypes.c_double, [vp]),
        "ewd_propose": (ctypes.c_double, [vp, ctypes.c_int, _dp]),
        "ewd_accept": (None, [vp, ctypes.c_int, _dp]),
        "ewd_num_k": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _vec3(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3))


def ncoef(p: int) -> int:
    return (p + 1) * (p + 1)


def idx(n: int, m: int) -> int:
    return n * n + n + m


# ---------------------------------------------------------------- expansions
def ylm(nmax: int, theta: float, phi: float) -> np.ndarray:
    """Y_n^m(theta, phi), n <= nmax, Greengard-Rokhlin normalisation without
    Condon-Shortley phase (Sec. 3.2, Eq. local_expansion)."""
    out = np.zeros(ncoef(nmax), dtype=np.complex128)
    _load().orc_ylm(nmax, float(theta), float(phi), out.ctypes.data_as(_dp))
    return out


def _op3(name, p, q, s, c):
    out = np.zeros(ncoef(p), dtype=np.complex128)
    getattr(_load(), name)(p, float(q), _d(_vec3(s)), _d(_vec3(c)), out.ctypes.data_as(_dp))
    return out


def p2m(p, q, s, c):
    """M_n^m = q rho^n Y_n^{-m}(s - c), Eq. (multipole_expansion_coefficients)."""
    return _op3("orc_p2m", p, q, s, c)


def p2e(p, q, s, c):
    """E_n^m = q rho^n Y_n^m(s - c) (Sec. 3.4)."""
    return _op3("orc_p2e", p, q, s, c)


def p2l(p, q, s, c):
    """L_n^m = q rho^{-(n+1)} Y_n^{-m}(s - c) (Alg. L.2 / L.3)."""
    return _op3("orc_p2l", p, q, s, c)


def l2p(p, L, x, c):
    L = np.ascontiguousarray(L, dtype=np.complex128)
    return _load().orc_l2p(p, L.ctypes.data_as(_dp), _d(_vec3(x)), _d(_vec3(c)))


def m2p(p, M, x, c):
    M = np.ascontiguousarray(M, dtype=np.complex128)
    return _load().orc_m2p(p, M.ctypes.data_as(_dp), _d(_vec3(x)), _d(_vec3(c)))


def _trans(name, p, O, d):
    O = np.ascontiguousarray(O, dtype=np.complex128)
    out = np.zeros(ncoef(p), dtype=np.complex128)
    getattr(_load(), name)(p, O.ctypes.data_as(_dp), _d(_vec3(d)), out.ctypes.data_as(_dp))
    return out


def m2m(p, O, d):
    """Multipole about Q re-expanded about Q - d (d = old centre - new centre)."""
    return _trans("orc_m2m", p, O, d)


def m2l(p, O, d):
    """Multipole about a source centre to a local expansion about a target
    centre; d = source centre - target centre."""
    return _trans("orc_m2l", p, O, d)


def l2l(p, O, d):
    return _trans("orc_l2l", p, O, d)


def il_offsets(octant) -> np.ndarray:
    """Offsets of the interaction list of a cell of the given octant
    (Sec. 3.1 definition)."""
    oc = (ctypes.c_int * 3)(*[int(v) for v in octant])
    out = (ctypes.c_int * (189 * 3 + 3 * 216))()
    n = _load().orc_il_offsets(oc, out)
    return np.array(out[: 3 * n], dtype=np.int64).reshape(n, 3)


def wrap(x: float, a: float) -> float:
    return _load().orc_wrap(float(x), float(a))


def cell_coord(x: float, a: float, n: int) -> int:
    return _load().orc_cell_coord(float(x), float(a), int(n))


def lattice_sums(lmax: int, a: float = 1.0, cut: int = 12) -> np.ndarray:
    """S_l^mu = sum over images with max|nu_k| >= 2 of Y_l^mu(nu^)/|a nu|^{l+1}."""
    out = np.zeros(ncoef(lmax), dtype=np.complex128)
    _load().orc_lattice_sums(lmax, float(a), cut, out.ctypes.data_as(_dp))
    return out


def lattice_apply(p, S, K):
    S = np.ascontiguousarray(S, dtype=np.complex128)
    K = np.ascontiguousarray(K, dtype=np.complex128)
    out = np.zeros(ncoef(p), dtype=np.complex128)
    _load().orc_lattice_apply(p, S.ctypes.data_as(_dp), K.ctypes.data_as(_dp), out.ctypes.data_as(_dp))
    return out


def self_image_constant() -> float:
    return _load().orc_self_image_constant()


# ---------------------------------------------------------------- RNG
def philox4x64_10(counter, key):
    c = (ctypes.c_uint64 * 4)(*[int(v) & (2**64 - 1) for v in counter])
    k = (ctypes.c_uint64 * 2)(*[int(v) & (2**64 - 1) for v in key])
    o = (ctypes.c_uint64 * 4)()
    _load().orc_philox4x64_10(c, k, o)
    return [int(v) for v in o]


def draw(seed: int, chain: int, step: int, n: int, max_step: float):
    """(idx, delta[3], u) of MH step `step` of chain `chain`."""
    idx = ctypes.c_int64()
    delta = np.zeros(3)
    u = ctypes.c_double()
    _load().orc_draw(seed, chain, step, n, float(max_step), ctypes.byref(idx), _d(delta),
                     ctypes.byref(u))
    return int(idx.value), delta, float(u.value)


# ---------------------------------------------------------------- states
class Multilevel:
    """The plain multilevel local-expansion method (Sec. 3.2, 3.4), FP64.

    ``setup`` is ``"fmm"`` (P2M, M2M, M2L; the initialisation the GPU path
    uses), ``"lazy"`` (the same, with each cell's M2L deferred to its first
    use: for sampled checks at full size), ``"direct"`` (Alg. L.3) or
    ``"none"`` (zero expansions, lattice moments only: timing of the
    per-step cost, never a reference value).

    ``setup="multipole"`` selects the multipole-based variant of Sec. 3.3
    (Alg. M.1-M.3, multipoles formed directly per level);
    ``"multipole_upward"`` is the same variant with the multipoles formed by
    the FMM upward pass (P2M, M2M).

    ``free_space=True`` selects free-space boundary conditions (Sec. 3.4):
    no images, no lattice or tin-foil terms, a move out of the box has
    dE = +inf.
    """

    def __init__(self, pos, q, box: float, depth: int, p: int, setup: str = "fmm", free_space: bool = False):
        lib = _load()
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        self.N = len(q)
        self.box = float(box)
        self.depth = int(depth)
        self.p = int(p)
        self.C = ncoef(p)
        if free_space and not ((pos >= 0).all() and (pos < box).all()):
            raise ValueError("free space: every position must lie in [0, box)")
        self._h = lib.orc_create(self.N, _d(pos), _d(q), self.box, self.depth, self.p)
        if free_space:
            lib.orc_set_free_space(self._h)
        if setup == "fmm":
            lib.orc_setup_fmm(self._h, 0)
        elif setup == "lazy":
            lib.orc_setup_fmm(self._h, 1)
        elif setup == "direct":
            lib.orc_setup_direct(self._h)
        elif setup == "none":  # zero expansions: for timing the per-step cost only
            lib.orc_setup_none(self._h)
        elif setup == "multipole":
            lib.orc_setup_multipole(self._h, 0)
        elif setup == "multipole_upward":
            lib.orc_setup_multipole(self._h, 1)
        else:
            raise ValueError(setup)

    def close(self):
        if self._h:
            _load().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def propose(self, k: int, newpos) -> float:
        return _load().orc_propose(self._h, int(k), _d(_vec3(newpos)))

    def accept(self, k: int, newpos) -> None:
        _load().orc_accept(self._h, int(k), _d(_vec3(newpos)))

    def energy(self) -> float:
        return _load().orc_energy(self._h)

    def local(self, level: int, cell: int) -> np.ndarray:
        out = np.zeros(self.C, dtype=np.complex128)
        _load().orc_get_local(self._h, int(level), int(cell), out.ctypes.data_as(_dp))
        return out

    def multipole(self, level: int, cell: int) -> np.ndarray:
        """multipole coefficients of one cell (the live state of the
        multipole-based variant; the setup state of the "fmm" setup)"""
        out = np.zeros(self.C, dtype=np.complex128)
        _load().orc_get_multipole(self._h, int(level), int(cell), out.ctypes.data_as(_dp))
        return out

    def K(self) -> np.ndarray:
        out = np.zeros(self.C, dtype=np.complex128)
        _load().orc_get_K(self._h, out.ctypes.data_as(_dp))
        return out

    def positions(self) -> np.ndarray:
        out = np.zeros((self.N, 3))
        _load().orc_get_positions(self._h, _d(out))
        return out

    def leaf_of(self, k: int) -> int:
        return _load().orc_leaf_of(self._h, int(k))

    def run(self, seed: int, chain: int, t0: int, nsteps: int, beta: float, max_step: float):
        """MH steps [t0, t0+nsteps) on the Philox stream; returns traces."""
        tr_idx = np.zeros(nsteps, dtype=np.int64)
        tr_pos = np.zeros((nsteps, 3))
        tr_de = np.zeros(nsteps)
        tr_u = np.zeros(nsteps)
        tr_acc = np.zeros(nsteps, dtype=np.uint8)
        _load().orc_run(self._h, seed, chain, t0, nsteps, float(beta), float(max_step),
                        tr_idx.ctypes.data_as(_i64p), _d(tr_pos), _d(tr_de), _d(tr_u),
                        tr_acc.ctypes.data_as(_u8p))
        return dict(idx=tr_idx, newpos=tr_pos, dE=tr_de, u=tr_u, acc=tr_acc.astype(bool))


def ewald_parameters(box: float, tol_exp: float = 32.0, rc_frac: float = 0.5):
    """alpha, rc, kmax for a target relative error of about exp(-tol_exp):
    erfc(alpha rc) ~ exp(-(alpha rc)^2), exp(-k^2/4alpha^2) at the cutoff."""
    rc = rc_frac * box
    alpha = np.sqrt(tol_exp) / rc
    kcut = 2.0 * alpha * np.sqrt(tol_exp)
    kmax = int(np.ceil(kcut * box / (2 * np.pi)))
    return float(alpha), float(rc), kmax


class Ewald:
    """Tin-foil Ewald summation with structure-factor updates (O1)."""

    def __init__(self, pos, q, box: float, alpha=None, rc=None, kmax=None, tol_exp=32.0):
        lib = _load()
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        a0, r0, k0 = ewald_parameters(box, tol_exp)
        self.alpha = a0 if alpha is None else float(alpha)
        self.rc = r0 if rc is None else float(rc)
        self.kmax = k0 if kmax is None else int(kmax)
        self.N = len(q)
        self._h = lib.ewd_create(self.N, _d(pos), _d(q), float(box), self.alpha, self.rc, self.kmax)

    def close(self):
        if self._h:
            _load().ewd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def energy(self) -> float:
        return _load().ewd_energy(self._h)

    def propose(self, k: int, newpos) -> float:
        return _load().ewd_propose(self._h, int(k), _d(_vec3(newpos)))

    def accept(self, k: int, newpos) -> None:
        _load().ewd_accept(self._h, int(k), _d(_vec3(newpos)))
