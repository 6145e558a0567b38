"""Benchmark: Metropolis-Hastings steps per second of the multilevel
local-expansion method on one MI355X.

Workload (default): the jittered rock-salt system of 46^3 = 97336 charges in
the periodic unit cube, octree depth 5, degree p = 12, beta = 1, displacement
uniform in [-0.3/46, 0.3/46)^3, one chain, FP64. A step is one whole MH step
(proposal energy, decision, and on acceptance the O(189 p^2 L) update of the
interaction-list expansions plus bookkeeping), all inside one persistent
kernel. The setup (P2M, M2M, M2L, lattice) is timed separately.

Also measured in the same run and reported beside the headline value:
* the same chain in mixed precision with an FP64 re-setup every 10^4
  accepts;
* the batched form: 256 independent chains of uneven size and depth, set up
  in one pass and run in one launch, in FP64 and in mixed precision, as
  aggregate steps/s;
* the multipole-based variant (Alg. M.1-M.3) on the same chain;
* the scaling sweep N = 10^3 .. 10^6 of the propose and accept times of
  the whole-GPU chain, local method and multipole variant, each fitted to
  the paper's performance model, with the speedup of the local method;
* in the cpu_baseline leg: the FP64 oracle's per-step rate, the Ewald
  oracle's, and the dE error of both precisions against Ewald on proposals
  from the initial rock-salt state.

Prints one JSON line. Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# HBM bytes of the timed single-chain launch of the default command (200000
# steps after 2000 warmup steps), from rocprofv3 FETCH_SIZE and WRITE_SIZE
# scaled by the counts of a plain 1 GiB device copy (FETCH_SIZE reads half the
# copied bytes, WRITE_SIZE all of them). Valid only for the kernel sources
# they were taken on; otherwise the traffic is reported as null.
MEASURED_TRAFFIC = {
    "src_sha256": "cd0e08b0bb0669f0fa02ad5defdcc51a3dda5c44e9419650d16d6fa3b3afde00",
    "steps": 200000, "warmup": 2000,
    "fetch_kib": 78057741.25, "fetch_scale": 2.0,
    "write_kib": 91775901.03125, "write_scale": 1.0,
}


def kernel_sources_sha256():
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2006_16622_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(steps, warmup):
    m = MEASURED_TRAFFIC
    if kernel_sources_sha256() != m["src_sha256"] or steps != m["steps"] or warmup != m["warmup"]:
        return None
    return 1024.0 * (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def il_offsets():
    """interaction-list offsets per octant (Sec. 3.1), for byte counting"""
    out = {}
    for oc in range(8):
        c = [(oc >> k) & 1 for k in range(3)]
        lst = []
        for oz in range(-2 - c[2], 4 - c[2]):
            for oy in range(-2 - c[1], 4 - c[1]):
                for ox in range(-2 - c[0], 4 - c[0]):
                    if max(abs(ox), abs(oy), abs(oz)) >= 2:
                        lst.append((ox, oy, oz))
        out[oc] = np.array(lst)
    return out


def accept_targets(r, rn, box, L, ilo):
    """distinct stored cells updated by one accepted move (all levels 2..L)"""
    tot = 0
    for l in range(2, L + 1):
        n = 2 ** (l - 1)
        sets = []
        for x in (r, rn):
            c = np.minimum(np.floor(np.asarray(x) * (n / box)).astype(int), n - 1)
            oc = int(c[0] & 1) | (int(c[1] & 1) << 1) | (int(c[2] & 1) << 2)
            b = np.mod(c[None, :] + ilo[oc], n)
            sets.append(b[:, 0] + n * (b[:, 1] + n * b[:, 2]))
        tot += len(np.union1d(sets[0], sets[1]))
    return tot


def algorithmic_bytes(wl, pos_before, tr_idx, tr_pos, tr_acc, sample=1500):
    """HBM bytes the method must touch: per proposal the 2d expansion blocks,
    the near-field records of 2 x 27 leaf cells and the lattice vectors; per
    accepted move a read and a write of every distinct interaction-list
    target on every level plus the lattice vectors. Old positions come from
    a forward replay of the trace from the positions before the timed run."""
    C = (wl.p + 1) ** 2
    L = wl.depth + 1
    mean_leaf = wl.n / 8 ** wl.depth
    prop = 2 * wl.depth * C * 8 + 2 * 27 * (mean_leaf * 36 + 4) + 2 * C * 8
    pos = pos_before.copy()
    ilo = il_offsets()
    acc_idx = np.nonzero(tr_acc)[0]
    pick = set(acc_idx[:: max(1, len(acc_idx) // sample)].tolist())
    targets = []
    for t in acc_idx:
        i = int(tr_idx[t])
        if t in pick:
            targets.append(accept_targets(pos[i], tr_pos[t], wl.box, L, ilo))
        pos[i] = tr_pos[t]
    mean_t = float(np.mean(targets)) if targets else 0.0
    acc_bytes = mean_t * C * 8 * 2 + 2 * C * 8 * 3
    return prop, acc_bytes, float(np.mean(tr_acc)), mean_t


def batched_algorithmic_bytes(wls, st, sample=40):
    """algorithmic bytes of a batched run: per chain its proposals and its
    accepts (mean distinct interaction-list targets per accept estimated on
    `sample` moves of the chain's own step size from its initial state)"""
    total = 0.0
    ilo = il_offsets()
    for w, s in zip(wls, st):
        C = (w.p + 1) ** 2
        L = w.depth + 1
        mean_leaf = w.n / 8 ** w.depth
        prop = 2 * w.depth * C * 8 + 2 * 27 * (mean_leaf * 36 + 4) + 2 * C * 8
        g = np.random.default_rng(w.chain)
        idx = g.integers(0, w.n, sample)
        tg = [accept_targets(w.pos[i], np.mod(w.pos[i] + g.uniform(-w.max_step, w.max_step, 3), w.box),
                             w.box, L, ilo) for i in idx]
        acc = float(np.mean(tg)) * C * 8 * 2 + 2 * C * 8 * 3
        total += s["proposed"] * prop + s["accepted"] * acc
    return total


def cpu_baseline(wl, nu, nprop=8000, nacc=1000):
    """The FP64 oracle timed on one host core: proposals and accepts of the
    same workload timed separately on a state whose expansions are not
    initialised (their values do not change the per-step cost; the
    initialisation of 97336 charges is out of reach of one core here), and
    combined as t_prop + nu t_acc with the acceptance rate of the GPU run."""
    import oracle as O
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    t0 = time.perf_counter()
    m = O.Multilevel(wl.pos, wl.q, wl.box, wl.depth, wl.p, setup="none")
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    for t in range(nprop):
        i, d, u = O.draw(wl.seed, 0, t, wl.n, wl.max_step)
        m.propose(i, wl.pos[i] + d)
    tp = (time.perf_counter() - t0) / nprop
    t0 = time.perf_counter()
    for t in range(nacc):
        i, d, u = O.draw(wl.seed, 0, t, wl.n, wl.max_step)
        m.accept(i, wl.pos[i] + d)
    ta = (time.perf_counter() - t0) / nacc
    step = tp + nu * ta
    out = {"value": 1.0 / step, "unit": "MH steps/s", "cores": 1, "kind": "oracle",
           "sample": f"{nprop} proposals and {nacc} accepts of the rocksalt workload on one core "
                     f"(expansions not initialised; lattice moments formed in {t_setup:.1f} s), "
                     f"t_prop={tp*1e3:.3f} ms, t_acc={ta*1e3:.3f} ms, combined at nu={nu:.3f}"}
    m.close()
    # the Ewald oracle (tin-foil, structure-factor updates): its per-step
    # rate, and the dE of the GPU in both precisions against it
    from paper_2006_16622_amd import FMM_MC_MIXED, Chain
    t0 = time.perf_counter()
    ew = O.Ewald(wl.pos, wl.q, wl.box)
    t_ew_setup = time.perf_counter() - t0
    moves = []
    for t in range(200):
        i, d, u = O.draw(wl.seed, 0, t, wl.n, wl.max_step)
        moves.append((i, wl.pos[i] + d))
    t0 = time.perf_counter()
    ref = np.array([ew.propose(i, r) for i, r in moves])
    tpe = (time.perf_counter() - t0) / len(moves)
    t0 = time.perf_counter()
    for i, r in moves[:100]:
        ew.accept(i, r)
    tae = (time.perf_counter() - t0) / 100
    errs = {}
    for name, flags in (("f64", 0), ("mixed", FMM_MC_MIXED), ("direct_setup", 4), ("multipole", 2)):
        ch = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=flags)
        de = np.array([ch.propose(i, r) for i, r in moves])
        ch.close()
        errs[name] = float(np.sqrt(np.mean((de - ref) ** 2)) / np.sqrt(np.mean(ref ** 2)))
    out["ewald"] = {"value": 1.0 / (tpe + nu * tae), "unit": "MH steps/s", "cores": 1, "kind": "oracle",
                    "setup_s": t_ew_setup, "t_prop_ms": tpe * 1e3, "t_acc_ms": tae * 1e3}
    out["dE_rel_rms_err_vs_ewald"] = errs
    out["dE_err_sample"] = ("200 proposals of the Philox stream from the initial rock-salt state, p = 12; "
                            "direct_setup: local expansions by Alg. L.3; multipole: Alg. M.1-M.3")
    return out


def run_batched(seed=4, steps=10000, nchains=256, flags=0, resetup_every=0):
    import workloads as W
    from paper_2006_16622_amd import run_chains, setup_batch
    import torch
    wls = [W.batched_chain(c, nchains, steps=steps) for c in range(nchains)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chains = setup_batch([(w.pos, w.q, w.box, w.depth) for w in wls], wls[0].p, flags=flags)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    m2l_ms = chains[0].last_timing()[1]
    # warmup a few steps (kernel load), then the timed launch
    run_chains(chains, 20, seed, 1.0, [w.max_step for w in wls], t0=0, mode=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = run_chains(chains, steps, seed, 1.0, [w.max_step for w in wls], t0=20, mode=1,
                    resetup_every=resetup_every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern = chains[0].last_timing()[0] * 1e-3
    acc = sum(s["accepted"] for s in st)
    abytes = batched_algorithmic_bytes(wls, st)
    for c in chains:
        c.close()
    return {"value": nchains * steps / dt, "unit": "MH steps/s", "chains": nchains, "steps_per_chain": steps,
            "precision": "mixed" if flags else "f64", "resetup_every": resetup_every,
            "kernel_s": kern, "wall_s": dt, "nu": acc / (nchains * steps), "setup_s": t_setup,
            "setup_m2l_ms": m2l_ms,
            "roofline": {"bound": "hbm", "achieved": abytes / kern / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": abytes / kern / 1e9 / HBM_PEAK_GBS, "kernel": "k_run_batched",
                         "algorithmic_bytes": abytes},
            "n_range": [min(w.n for w in wls), max(w.n for w in wls)],
            "depths": {str(d): sum(1 for w in wls if w.depth == d) for d in sorted({w.depth for w in wls})},
            "status": [s["status"] for s in st if s["status"] != 0][:4]}


SWEEP_N = (1000, 2000, 5000, 10000, 20000, 50000, 100000, 200000, 500000, 1000000)


def _stage_times(st, steps, flags):
    """per-proposal and per-accept times (us) from the kernel's own clock.
    In the local method the helpers' wait belongs to the accept; in the
    multipole-based variant it is the far field of the proposal."""
    acc = max(1, st["accepted"])
    if flags & 2:
        return (st["t_propose_us"] + st["t_wait_us"]) / steps, st["t_accept_us"] / acc
    return st["t_propose_us"] / steps, (st["t_accept_us"] + st["t_wait_us"]) / acc


def _fit(rows):
    A = np.array([[1.0, r["L"], r["n"] / 8 ** (r["L"] - 1), r["n"]] for r in rows])
    fit = {}
    for stage in ("prop", "acc"):
        y = np.array([r[f"t_{stage}_us"] for r in rows])
        coef = np.linalg.lstsq(A, y, rcond=None)[0]
        fit[stage] = {"tau_us": coef[0], "gamma_us": coef[1], "kappa_us": coef[2], "sigma_us": coef[3]}
    return fit


def _model_t(f, n, L):
    return f["tau_us"] + f["gamma_us"] * L + f["kappa_us"] * n / 8 ** (L - 1) + f["sigma_us"] * n


def run_sweep(steps=2000, warmup=300, nu_paper=0.438):
    """Propose and accept time of the whole-GPU chain of the local method and
    of the multipole-based variant for N = 10^3 .. 10^6 uniform charges
    (about 3 per leaf cell, steps of 0.1 mean spacing); the least-squares
    fit of each stage to the paper's performance model
    T(N) = tau + gamma L + kappa N / N_cell + sigma N, and the speedup of
    the local method over the multipole variant, measured per step and
    predicted from the fits at the paper's acceptance rate, with its limit
    S_inf = (g_prop^mp + nu g_acc^mp) / (g_prop^loc + nu g_acc^loc)
    (Sec. 5.4)."""
    import workloads as W
    from paper_2006_16622_amd import Chain, run_chains
    import torch
    rows = {0: [], 2: []}
    for i, n in enumerate(SWEEP_N):
        depth = max(2, int(round(math.log(n / 3.0, 8))))
        wl = W.uniform(n, depth, 12, 0.1 * n ** (-1.0 / 3.0), seed=50 + i, key=30 + i)
        for flags in (0, 2):
            ch = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=flags)
            run_chains([ch], warmup, wl.seed, 1.0, wl.max_step, t0=0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = run_chains([ch], steps, wl.seed, 1.0, wl.max_step, t0=warmup)[0]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            tp, ta = _stage_times(st, steps, flags)
            rows[flags].append({"n": n, "depth": depth, "L": depth + 1, "n_per_leaf": n / 8 ** depth,
                                "t_prop_us": tp, "t_acc_us": ta, "nu": st["accepted"] / steps,
                                "steps_per_s": steps / dt, "status": st["status"]})
            ch.close()
            log(f"[bench] sweep {'multipole' if flags else 'local'} n={n} d={depth}: prop {tp:.2f} us, "
                f"acc {ta:.2f} us, {steps / dt:.0f} steps/s")
    fit_loc, fit_mp = _fit(rows[0]), _fit(rows[2])
    speed = []
    for rl, rm in zip(rows[0], rows[2]):
        n, L = rl["n"], rl["L"]
        num = _model_t(fit_mp["prop"], n, L) + nu_paper * _model_t(fit_mp["acc"], n, L)
        den = _model_t(fit_loc["prop"], n, L) + nu_paper * _model_t(fit_loc["acc"], n, L)
        speed.append({"n": n, "measured": rl["steps_per_s"] / rm["steps_per_s"], "model": num / den})
    g = lambda f, st: f[st]["gamma_us"]  # noqa: E731
    s_inf = (g(fit_mp, "prop") + nu_paper * g(fit_mp, "acc")) / (g(fit_loc, "prop") + nu_paper * g(fit_loc, "acc"))
    return {"model": "T(N) = tau + gamma L + kappa N/N_cell + sigma N (least squares, microseconds)",
            "p": 12, "precision": "f64", "mode": "whole GPU", "steps": steps,
            "rows": rows[0], "fit": fit_loc, "multipole": {"rows": rows[2], "fit": fit_mp},
            "speedup_local_over_multipole": {"nu": nu_paper, "per_n": speed, "s_inf": s_inf}}


def run_single_variant(wl, steps, warmup, flags, resetup_every=0, tune=False):
    """one chain of the workload with the given flags, on the whole GPU"""
    from paper_2006_16622_amd import Chain, run_chains
    import torch
    ch = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=flags)
    t = ch.autotune(steps=2000, beta=wl.beta, max_step=wl.max_step) if tune else None
    run_chains([ch], warmup, wl.seed, wl.beta, wl.max_step, t0=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = run_chains([ch], steps, wl.seed, wl.beta, wl.max_step, t0=warmup, resetup_every=resetup_every)[0]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ch.close()
    tp, ta = _stage_times(st, steps, flags)
    out = {"value": steps / dt, "unit": "MH steps/s", "steps": steps, "accepted": st["accepted"],
           "status": st["status"], "t_prop_us": tp, "t_acc_us": ta}
    if t is not None:
        out["helpers"] = t["helpers"]
    return out


def run_single_mixed(wl, steps, warmup, resetup_every=10000):
    from paper_2006_16622_amd import FMM_MC_MIXED, Chain, run_chains
    import torch
    ch = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=FMM_MC_MIXED)
    run_chains([ch], warmup, wl.seed, wl.beta, wl.max_step, t0=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = run_chains([ch], steps, wl.seed, wl.beta, wl.max_step, t0=warmup, resetup_every=resetup_every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ch.close()
    return {"value": steps / dt, "unit": "MH steps/s", "precision": "mixed", "resetup_every": resetup_every,
            "accepted": st[0]["accepted"], "status": st[0]["status"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=10000)
    ap.add_argument("--no-sweep", action="store_true", help="skip the N = 1e3 .. 1e6 scaling sweep")
    ap.add_argument("--mode", type=int, default=0, help="0 auto, 1 one workgroup, 2 whole GPU")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8,
                          "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this method's single chain does not shard, and the "
              "batched chains are independent (see the scaling paragraph of the design notes); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    from paper_2006_16622_amd import Chain, run_chains
    from paper_2006_16622_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    wl = W.rocksalt()
    log(f"[bench] workload {wl.name}: setup")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    m2l_ms = ch.last_timing()[1]
    log(f"[bench] setup {t_setup*1e3:.1f} ms (M2L {m2l_ms:.2f} ms); autotune")
    tune = ch.autotune(steps=2000, beta=wl.beta, max_step=wl.max_step)
    log(f"[bench] autotune: M2L rows {tune['m2l_rows']}, helpers {tune['helpers']}; warmup {args.warmup}")
    run_chains([ch], args.warmup, wl.seed, wl.beta, wl.max_step, t0=0, mode=args.mode)
    torch.cuda.synchronize()
    pos_before = ch.positions()
    log(f"[bench] timed {args.steps} steps")
    t0 = time.perf_counter()
    st, tr = run_chains([ch], args.steps, wl.seed, wl.beta, wl.max_step, t0=args.warmup, mode=args.mode,
                        traces=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_s = ch.last_timing()[0] * 1e-3
    s0 = st[0]
    value = args.steps / dt
    log(f"[bench] {value:.1f} steps/s (kernel {kern_s:.3f} s, wall {dt:.3f} s), accepted {s0['accepted']}")
    prop_b, acc_b, nu, mean_t = algorithmic_bytes(wl, pos_before, tr["idx"][0], tr["newpos"][0], tr["acc"][0])
    total_bytes = args.steps * prop_b + s0["accepted"] * acc_b
    achieved = total_bytes / kern_s / 1e9
    out = {
        "metric": "MH steps/s at N=1e5 (1 chain) + aggregate over 256 chains; dE err vs Ewald",
        "value": value,
        "unit": "MH steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n, "depth": wl.depth, "p": wl.p, "beta": wl.beta,
                   "max_step": wl.max_step, "chains": 1, "setup_ms": t_setup * 1e3, "setup_m2l_ms": m2l_ms,
                   "autotune": tune,
                   "acceptance": s0["accepted"] / args.steps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.steps, args.warmup),
                     "algorithmic_bytes": total_bytes,
                     "kernel": "k_run_single", "kernel_s": kern_s,
                     "bytes_per_proposal": prop_b, "bytes_per_accept": acc_b,
                     "targets_per_accept": mean_t},
    }
    log("[bench] single chain, mixed precision")
    out["single_mixed"] = run_single_mixed(wl, args.steps, args.warmup)
    log(f"[bench] single chain mixed {out['single_mixed']['value']:.1f} steps/s")
    log("[bench] direct P2L setup (Alg. L.3)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chd = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=4)
    torch.cuda.synchronize()
    out["setup_direct"] = {"wall_ms": (time.perf_counter() - t0) * 1e3, "p2l_ms": chd.last_timing()[1]}
    chd.close()
    log(f"[bench] direct setup {out['setup_direct']['wall_ms']:.1f} ms (P2L {out['setup_direct']['p2l_ms']:.2f} ms)")
    log("[bench] single chain, multipole-based variant")
    out["single_multipole"] = run_single_variant(wl, args.steps // 4, args.warmup, flags=2, tune=True)
    out["single_multipole"]["variant"] = "multipole (Alg. M.1-M.3)"
    log(f"[bench] single chain multipole {out['single_multipole']['value']:.1f} steps/s")
    if not args.no_batched:
        log("[bench] batched 256 chains, FP64")
        out["batched"] = run_batched(steps=args.batched_steps)
        log(f"[bench] batched {out['batched']['value']:.1f} steps/s")
        log("[bench] batched 256 chains, mixed precision")
        out["batched_mixed"] = run_batched(steps=args.batched_steps, flags=1, resetup_every=10000)
        log(f"[bench] batched mixed {out['batched_mixed']['value']:.1f} steps/s")
    if not args.no_sweep:
        log("[bench] scaling sweep")
        out["sweep"] = run_sweep()
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(wl, out["config"]["acceptance"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
