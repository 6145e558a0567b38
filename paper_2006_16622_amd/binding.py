"""ctypes binding of libfmm_mc.so (argument marshalling only).

Every entry point of ``include/fmm_mc.h`` is reachable under the same name;
``Chain`` owns one chain's device workspace (a torch uint8 tensor) and
handle. No computation happens here.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FMM_MC_LIB", os.path.join(HERE, "libfmm_mc.so"))

FMM_MC_MIXED = 0x1
FMM_MC_MULTIPOLE = 0x2
FMM_MC_DIRECT_SETUP = 0x4
FMM_MC_FREE_SPACE = 0x8
_ERRORS = {0: "ok", -1: "EINVAL", -2: "ERANGE", -3: "ENONNEUTRAL", -4: "ESINGULAR", -5: "ENOMEM",
           -6: "EDEVICE", -7: "EOVERFLOW", -8: "ESTATE"}


class FmmMcError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_ERRORS.get(code, code)} ({code})")
        self.code = code


class RunOpts(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("max_step", ctypes.c_double),
                ("chain_max_step", ctypes.POINTER(ctypes.c_double)), ("t0", ctypes.c_int64),
                ("mode", ctypes.c_int32), ("resetup_every", ctypes.c_int32),
                ("trace_idx", ctypes.c_void_p), ("trace_newpos", ctypes.c_void_p),
                ("trace_dE", ctypes.c_void_p), ("trace_acc", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("m2l_rows", ctypes.c_int32), ("helpers", ctypes.c_int32),
                ("n_helper_candidates", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("m2l_ms", ctypes.c_double * 2), ("helper_candidates", ctypes.c_int32 * 8),
                ("step_us", ctypes.c_double * 8)]


class Stats(ctypes.Structure):
    _fields_ = [("proposed", ctypes.c_int64), ("accepted", ctypes.c_int64),
                ("singular", ctypes.c_int64), ("dE_sum", ctypes.c_double),
                ("energy", ctypes.c_double), ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("t_propose_us", ctypes.c_double), ("t_accept_us", ctypes.c_double),
                ("t_wait_us", ctypes.c_double)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i32p = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p

SYMBOLS = {
    "fmm_mc_workspace_bytes": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_uint32,
                                              ctypes.POINTER(ctypes.c_size_t)]),
    "fmm_mc_setup": (ctypes.c_int, [ctypes.POINTER(_vp), _vp, ctypes.c_size_t, _vp, ctypes.c_int64, _dp, _dp,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_uint32]),
    "fmm_mc_setup_batch": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp),
                                          ctypes.POINTER(ctypes.c_size_t), _vp, _i64p, ctypes.POINTER(_dp),
                                          ctypes.POINTER(_dp), _dp, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                          ctypes.c_uint32]),
    "fmm_mc_propose": (ctypes.c_int, [_vp, ctypes.c_int64, _dp, _dp]),
    "fmm_mc_accept": (ctypes.c_int, [_vp, ctypes.c_int64, _dp, _dp, _dp]),
    "fmm_mc_run": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                  ctypes.POINTER(RunOpts), ctypes.POINTER(Stats)]),
    "fmm_mc_run_noalloc": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                          ctypes.POINTER(RunOpts), ctypes.POINTER(Stats)]),
    "fmm_mc_replay": (ctypes.c_int, [_vp, ctypes.c_int64, _i64p, _dp, _dp, ctypes.c_double, _dp, _u8p, _i32p]),
    "fmm_mc_energy": (ctypes.c_int, [_vp, _dp]),
    "fmm_mc_running_energy": (ctypes.c_int, [_vp, _dp]),
    "fmm_mc_get_positions": (ctypes.c_int, [_vp, _dp]),
    "fmm_mc_dump_locals": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "fmm_mc_dump_multipoles": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "fmm_mc_resetup": (ctypes.c_int, [_vp]),
    "fmm_mc_rescale": (ctypes.c_int, [_vp, ctypes.c_double, _dp]),
    "fmm_mc_rescale_undo": (ctypes.c_int, [_vp]),
    "fmm_mc_autotune": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                       ctypes.POINTER(Tuning)]),
    "fmm_mc_set_helpers": (ctypes.c_int, [_vp, ctypes.c_int]),
    "fmm_mc_destroy": (ctypes.c_int, [_vp]),
    "fmm_mc_release_tables": (ctypes.c_int, []),
    "fmm_mc_last_timing": (ctypes.c_int, [_vp, _dp, ctypes.c_int]),
    "fmm_mc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "fmm_mc_host_operator": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _dp]),
}


# Chains still open; closed, and the shared tables freed, by an exit hook
# that runs before the interpreter tears down its modules (a handle's HIP
# objects are released while the runtime is still whole).
_live = weakref.WeakSet()


def _close_all():
    for c in list(_live):
        try:
            c.close()
        except Exception:
            pass
    if _lib is not None:
        _lib.fmm_mc_release_tables()


def load_library():
    """Load libfmm_mc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FmmMcError(-6, f"HIP library missing at {LIB_PATH}; run paper_2006_16622_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SYMBOLS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    atexit.register(_close_all)
    return lib


def _check(code: int, what: str):
    if code != 0:
        raise FmmMcError(code, what)


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def workspace_bytes(n: int, levels: int, p: int, flags: int = 0) -> int:
    out = ctypes.c_size_t()
    _check(load_library().fmm_mc_workspace_bytes(n, levels, p, flags, ctypes.byref(out)), "workspace_bytes")
    return int(out.value)


def host_operator(kind: int, p: int, o=(0, 0, 0)) -> np.ndarray:
    C = (p + 1) ** 2
    out = np.zeros(C * C)
    oo = (ctypes.c_int * 3)(*[int(v) for v in o])
    _check(load_library().fmm_mc_host_operator(kind, p, oo, _d(out)), "host_operator")
    return out.reshape(C, C)


class Chain:
    """One Markov chain: positions/charges set up on the GPU (``fmm_mc_setup``)."""

    def __init__(self, pos, q, box: float, levels: int, p: int, flags: int = 0, device: str = "cuda:0",
                 stream=None, _defer: bool = False):
        import torch
        lib = load_library()
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        self._pos, self._q = pos, q
        self.n = len(q)
        self.levels, self.p, self.box, self.flags = int(levels), int(p), float(box), int(flags)
        self.device = torch.device(device)
        self.nbytes = workspace_bytes(self.n, self.levels, self.p, flags)
        self.ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = _vp()
        _live.add(self)
        if _defer:
            return
        with torch.cuda.device(self.device):
            rc = lib.fmm_mc_setup(ctypes.byref(self._h), _vp(self.ws_ptr), self.nbytes,
                                  _vp(self.stream.cuda_stream), self.n, _d(pos), _d(q), self.box, self.levels,
                                  self.p, flags)
        _check(rc, "fmm_mc_setup")

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load_library().fmm_mc_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def propose(self, idx: int, new_pos) -> float:
        r = np.ascontiguousarray(new_pos, dtype=np.float64).reshape(3)
        out = ctypes.c_double()
        _check(load_library().fmm_mc_propose(self._h, int(idx), _d(r), ctypes.byref(out)), "fmm_mc_propose")
        return out.value

    def accept(self, idx: int, new_pos, dE=None) -> float:
        r = np.ascontiguousarray(new_pos, dtype=np.float64).reshape(3)
        out = ctypes.c_double()
        dein = ctypes.byref(ctypes.c_double(dE)) if dE is not None else None
        _check(load_library().fmm_mc_accept(self._h, int(idx), _d(r), dein, ctypes.byref(out)), "fmm_mc_accept")
        return out.value

    def energy(self) -> float:
        out = ctypes.c_double()
        _check(load_library().fmm_mc_energy(self._h, ctypes.byref(out)), "fmm_mc_energy")
        return out.value

    def running_energy(self) -> float:
        out = ctypes.c_double()
        _check(load_library().fmm_mc_running_energy(self._h, ctypes.byref(out)), "fmm_mc_running_energy")
        return out.value

    def positions(self) -> np.ndarray:
        out = np.zeros((self.n, 3))
        _check(load_library().fmm_mc_get_positions(self._h, _d(out)), "fmm_mc_get_positions")
        return out

    def locals(self, level: int) -> np.ndarray:
        C = (self.p + 1) ** 2
        out = np.zeros((8 ** (level - 1), C))
        _check(load_library().fmm_mc_dump_locals(self._h, int(level), _d(out)), "fmm_mc_dump_locals")
        return out

    def multipoles(self, level: int) -> np.ndarray:
        C = (self.p + 1) ** 2
        out = np.zeros((8 ** (level - 1), C))
        _check(load_library().fmm_mc_dump_multipoles(self._h, int(level), _d(out)), "fmm_mc_dump_multipoles")
        return out

    def autotune(self, steps: int = 1000, beta: float = 1.0, max_step: float = 0.0) -> dict:
        """fmm_mc_autotune: pick the M2L tile and the helper count for this shape"""
        t = Tuning()
        _check(load_library().fmm_mc_autotune(self._h, int(steps), float(beta), float(max_step),
                                              ctypes.byref(t)), "fmm_mc_autotune")
        k = t.n_helper_candidates
        return dict(m2l_rows=t.m2l_rows, helpers=t.helpers, m2l_ms=list(t.m2l_ms),
                    helper_candidates=list(t.helper_candidates[:k]), step_us=list(t.step_us[:k]))

    def set_helpers(self, helpers: int):
        """fmm_mc_set_helpers: helper workgroups of the whole-GPU run (0: one per accept block)"""
        _check(load_library().fmm_mc_set_helpers(self._h, int(helpers)), "fmm_mc_set_helpers")

    def resetup(self):
        _check(load_library().fmm_mc_resetup(self._h), "fmm_mc_resetup")

    def rescale(self, new_box: float) -> float:
        """fmm_mc_rescale: volume move to box side new_box; returns dE"""
        out = ctypes.c_double()
        _check(load_library().fmm_mc_rescale(self._h, float(new_box), ctypes.byref(out)), "fmm_mc_rescale")
        self._box_prev, self.box = self.box, float(new_box)
        return out.value

    def rescale_undo(self):
        """fmm_mc_rescale_undo: back to the state before the last rescale"""
        _check(load_library().fmm_mc_rescale_undo(self._h), "fmm_mc_rescale_undo")
        self.box = self._box_prev

    def replay(self, idx, new_pos, u, beta: float):
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        new_pos = np.ascontiguousarray(new_pos, dtype=np.float64).reshape(-1, 3)
        u = np.ascontiguousarray(u, dtype=np.float64)
        m = len(idx)
        dE = np.zeros(m)
        acc = np.zeros(m, dtype=np.uint8)
        leaf = np.zeros(m, dtype=np.int32)
        _check(load_library().fmm_mc_replay(self._h, m, idx.ctypes.data_as(_i64p), _d(new_pos), _d(u),
                                            float(beta), _d(dE), acc.ctypes.data_as(_u8p),
                                            leaf.ctypes.data_as(_i32p)), "fmm_mc_replay")
        return dE, acc.astype(bool), leaf

    def last_timing(self):
        out = np.zeros(4)
        _check(load_library().fmm_mc_last_timing(self._h, _d(out), 4), "fmm_mc_last_timing")
        return out


def setup_batch(systems, p: int, flags: int = 0, device: str = "cuda:0", stream=None):
    """fmm_mc_setup_batch over a list of (pos, q, box, levels): one setup
    pass for all chains. Returns the Chain objects in order."""
    import torch
    lib = load_library()
    chains = [Chain(pos, q, box, levels, p, flags, device, stream, _defer=True)
              for (pos, q, box, levels) in systems]
    nc = len(chains)
    hs = (_vp * nc)()
    ws = (_vp * nc)(*[c.ws_ptr for c in chains])
    wb = (ctypes.c_size_t * nc)(*[c.nbytes for c in chains])
    ns = np.array([c.n for c in chains], dtype=np.int64)
    pp = (_dp * nc)(*[_d(c._pos) for c in chains])
    qq = (_dp * nc)(*[_d(c._q) for c in chains])
    boxes = np.array([c.box for c in chains], dtype=np.float64)
    lv = (ctypes.c_int * nc)(*[c.levels for c in chains])
    with torch.cuda.device(chains[0].device):
        rc = lib.fmm_mc_setup_batch(hs, nc, ws, wb, _vp(chains[0].stream.cuda_stream), ns.ctypes.data_as(_i64p),
                                    pp, qq, _d(boxes), lv, int(p), int(flags))
    _check(rc, "fmm_mc_setup_batch")
    for c, h in zip(chains, hs):
        c._h = _vp(h)
    return chains


def run_chains(chains, steps: int, seed: int, beta: float, max_step, t0: int = 0, mode: int = 0,
               traces: bool = False, resetup_every: int = 0, trace_ptrs=None, noalloc: bool = False):
    """fmm_mc_run over a list of Chain objects (same device and stream).
    With traces, device buffers (torch) are allocated and returned as numpy.
    trace_ptrs: device addresses (ints) of caller-owned trace buffers,
    keys idx, newpos, dE, acc, laid out [chain * steps + t] as in
    fmm_mc_run_opts; nothing is allocated or returned for them.
    noalloc: call fmm_mc_run_noalloc instead of fmm_mc_run."""
    import torch
    lib = load_library()
    nc = len(chains)
    hs = (_vp * nc)(*[c.handle for c in chains])
    ms = np.ascontiguousarray(np.broadcast_to(np.asarray(max_step, dtype=np.float64), (nc,)))
    opts = RunOpts()
    opts.beta = float(beta)
    opts.max_step = float(ms[0])
    opts.chain_max_step = _d(ms)
    opts.t0 = int(t0)
    opts.mode = int(mode)
    opts.resetup_every = int(resetup_every)
    tr = None
    if trace_ptrs is not None:
        opts.trace_idx = trace_ptrs.get("idx")
        opts.trace_newpos = trace_ptrs.get("newpos")
        opts.trace_dE = trace_ptrs.get("dE")
        opts.trace_acc = trace_ptrs.get("acc")
    if traces:
        dev = chains[0].device
        tr = dict(idx=torch.zeros(nc * steps, dtype=torch.int64, device=dev),
                  newpos=torch.zeros(nc * steps * 3, dtype=torch.float64, device=dev),
                  dE=torch.zeros(nc * steps, dtype=torch.float64, device=dev),
                  acc=torch.zeros(nc * steps, dtype=torch.uint8, device=dev))
        opts.trace_idx = tr["idx"].data_ptr()
        opts.trace_newpos = tr["newpos"].data_ptr()
        opts.trace_dE = tr["dE"].data_ptr()
        opts.trace_acc = tr["acc"].data_ptr()
    stats = (Stats * nc)()
    entry = lib.fmm_mc_run_noalloc if noalloc else lib.fmm_mc_run
    rc = entry(hs, nc, int(steps), int(seed), ctypes.byref(opts), stats)
    _check(rc, "fmm_mc_run_noalloc" if noalloc else "fmm_mc_run")
    out = [dict(proposed=s.proposed, accepted=s.accepted, singular=s.singular, dE_sum=s.dE_sum,
                energy=s.energy, status=s.status, t_propose_us=s.t_propose_us,
                t_accept_us=s.t_accept_us, t_wait_us=s.t_wait_us) for s in stats]
    if traces:
        torch.cuda.synchronize(chains[0].device)
        tr = {k: v.cpu().numpy() for k, v in tr.items()}
        tr["newpos"] = tr["newpos"].reshape(nc, steps, 3)
        for k in ("idx", "dE", "acc"):
            tr[k] = tr[k].reshape(nc, steps)
        tr["acc"] = tr["acc"].astype(bool)
        return out, tr
    return out
