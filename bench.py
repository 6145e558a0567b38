"""Benchmark: Metropolis-Hastings steps per second of the multilevel
local-expansion method on one MI355X.

Headline workload: the jittered rock-salt system of 46^3 = 97336 charges in
the periodic unit cube, octree depth 5, degree p = 12, beta = 1,
displacement uniform in [-0.3/46, 0.3/46)^3, one chain, FP64, on the whole
GPU. An MH step is the proposal energy, the decision and, on acceptance,
the O(189 p^2 L) update of the interaction-list expansions plus the
bookkeeping, all inside one persistent kernel.

A bench step is one fmm_mc_run call of --mh-per-step MH steps (default
10^4) on the resident chain: `--steps K --warmup W` runs W untimed calls,
then times exactly K calls between two device synchronisations. `value` is
the MH steps of the K calls over that wall time; the kernel's own HIP-event
time of the same calls is reported beside it. The algorithmic bytes per
accept come from a traced run of the same chain after the timed region.

Also measured in the same run and reported beside the headline value, each
with its error against the Ewald oracle:
* the rock-salt chain in mixed precision with an FP64 re-setup every 10^4
  accepts, and the drift each re-setup removes;
* the rock-salt chain at p = 19, the smallest degree at which its dE error
  against Ewald falls below 1e-5 of RMS dE, in FP64 and in mixed precision;
* the multipole-based variant (Alg. M.1-M.3) on the rock-salt chain, and
  the direct P2L setup (Alg. L.3);
* the small (N = 10^3) and medium (N = 10^4, with setup time and a mixed
  rerun) single-chain workloads;
* the batched form: 256 independent chains of uneven size and depth, set up
  in one pass and run in one launch (one workgroup per chain), in FP64 and
  in mixed precision, as
  aggregate steps/s, with the dE error of 8 sampled chains against Ewald
  and against the FP64 oracle;
* the scaling sweep N = 10^3 .. 10^6 of the propose and accept times of the
  whole-GPU chain, local method and multipole variant, each fitted to the
  paper's performance model, with the speedup of the local method;
* in the cpu_baseline leg: the FP64 oracle's per-step rate on one host core
  (rock salt) and on all host cores (batched chains, one per thread), and
  the Ewald oracle's.

Prints one JSON line. Usage: python bench.py [--steps K] [--warmup W]
[--mh-per-step M]
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
P_GATE = 19  # smallest degree whose rock-salt dE error against Ewald is below 1e-5 of RMS dE

# HBM bytes per MH step of the timed launches of the default command, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by the counts of a plain 1 GiB
# device copy (FETCH_SIZE reads half the copied bytes, WRITE_SIZE all of
# them): the 20 single-chain launches (k_run_single) and the batched FP64
# launch (k_run_chains, 256 chains x 10^4 steps). The per-step figures depend
# on the acceptance rate, which the fixed proposal stream fixes. Valid only
# for the kernel sources they were taken on; otherwise the traffic is null.
MEASURED_TRAFFIC = {
    "src_sha256": "e36957b51de27a8391df6eba80827545b50f28cb760ebcab00b9f763ab320f8f",
    "fetch_bytes_per_step": 779828.9,
    "write_bytes_per_step": 438489.2,
    "batched_fetch_bytes_per_step": 209943.4,
    "batched_write_bytes_per_step": 188496.3,
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


def measured_traffic(mh_steps, batched=False):
    """HBM bytes (FETCH + WRITE, scaled) of a launch of mh_steps MH steps,
    or None when the kernel sources differ from those the counters came from"""
    m = MEASURED_TRAFFIC
    if m["src_sha256"] is None or kernel_sources_sha256() != m["src_sha256"]:
        return None
    pre = "batched_" if batched else ""
    return mh_steps * (m[pre + "fetch_bytes_per_step"] + m[pre + "write_bytes_per_step"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_rms(de, ref):
    de, ref = np.asarray(de), np.asarray(ref)
    return float(np.sqrt(np.mean((de - ref) ** 2)) / np.sqrt(np.mean(ref ** 2)))


def host_threads():
    """threads for the all-core oracle leg: this process's CPU share, at
    most 16 (the host share of one GPU)"""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


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


def moves_from_stream(wl, count, pos, chain=0):
    import oracle as O
    out = []
    for t in range(count):
        i, d, _ = O.draw(wl.seed, chain, t, wl.n, wl.max_step)
        out.append((i, pos[i] + d))
    return out


def gpu_proposals(wl, moves, flags=0, p=None):
    from paper_2006_16622_amd import Chain
    ch = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p if p is None else p, flags=flags)
    de = np.array([ch.propose(i, r) for i, r in moves])
    ch.close()
    return de


def timed_calls(chains, wl_steps, seed, beta, max_step, calls, mh, t0, resetup_every=0, mode=0):
    """`calls` fmm_mc_run calls of `mh` MH steps each, between two device
    synchronisations: (wall s, kernel s, summed stats per chain)"""
    from paper_2006_16622_amd import run_chains
    import torch
    tot = None
    kern = 0.0
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(calls):
        st = run_chains(chains, mh, seed, beta, max_step, t0=t0 + k * mh, mode=mode,
                        resetup_every=resetup_every)
        kern += chains[0].last_timing()[0] * 1e-3
        if tot is None:
            tot = [dict(s) for s in st]
        else:
            for a, b in zip(tot, st):
                for key in ("proposed", "accepted", "singular", "dE_sum", "t_propose_us", "t_accept_us",
                            "t_wait_us"):
                    a[key] += b[key]
                a["energy"] = b["energy"]
                a["status"] = a["status"] or b["status"]
    torch.cuda.synchronize()
    return time.perf_counter() - t_start, kern, tot


def headline(wl, steps, warmup, mh):
    """the rock-salt chain, FP64, whole GPU: setup, autotune, W warmup and
    K timed calls of mh MH steps, then a traced sample for the bytes"""
    from paper_2006_16622_amd import Chain, run_chains
    import torch
    log(f"[bench] workload {wl.name}: setup")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    m2l_ms = ch.last_timing()[1]
    log(f"[bench] setup {t_setup*1e3:.1f} ms (M2L {m2l_ms:.2f} ms); autotune")
    tune = ch.autotune(steps=2000, beta=wl.beta, max_step=wl.max_step)
    log(f"[bench] autotune: M2L rows {tune['m2l_rows']}, helpers {tune['helpers']}; warmup {warmup} x {mh}")
    tw, _, _ = timed_calls([ch], None, wl.seed, wl.beta, wl.max_step, warmup, mh, 0)
    log(f"[bench] warmup {tw:.2f} s; timed {steps} x {mh} MH steps")
    dt, kern, st = timed_calls([ch], None, wl.seed, wl.beta, wl.max_step, steps, mh, warmup * mh)
    s0 = st[0]
    total = steps * mh
    log(f"[bench] {total / dt:.1f} MH steps/s (kernel {kern:.3f} s, wall {dt:.3f} s), accepted {s0['accepted']}")
    # the bytes each accept touches, from a traced sample of the same chain
    nsamp = 20000
    pos_before = ch.positions()
    _, tr = run_chains([ch], nsamp, wl.seed, wl.beta, wl.max_step, t0=(warmup + steps) * mh, traces=True)
    prop_b, acc_b, nu_s, mean_t = algorithmic_bytes(wl, pos_before, tr["idx"][0], tr["newpos"][0], tr["acc"][0])
    ch.close()
    total_bytes = total * prop_b + s0["accepted"] * acc_b
    achieved = total_bytes / kern / 1e9
    nu = s0["accepted"] / total
    out = {
        "value": total / dt,
        "ms_per_step": dt / steps * 1e3,
        "kernel_ms_per_step": kern / steps * 1e3,
        "us_per_mh_step": dt / total * 1e6,
        "kernel_us_per_mh_step": kern / total * 1e6,
        "nu": nu,
        "status": s0["status"],
        "t_prop_us": s0["t_propose_us"] / total,
        "t_acc_us": (s0["t_accept_us"] + s0["t_wait_us"]) / max(1, s0["accepted"]),
        "setup_ms": t_setup * 1e3, "setup_m2l_ms": m2l_ms, "autotune": tune,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(mh),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)",
                     "algorithmic_bytes_per_launch": total_bytes / steps,
                     "algorithmic_bytes": total_bytes, "kernel": "k_run_single", "kernel_s": kern,
                     "launches": steps, "mh_steps_per_launch": mh,
                     "bytes_per_proposal": prop_b, "bytes_per_accept": acc_b,
                     "targets_per_accept": mean_t, "traced_sample_steps": nsamp, "traced_sample_nu": nu_s},
    }
    return out


def single_line(wl, steps, warmup, mh, flags=0, p=None, resetup_every=0, tune=False):
    """one chain of the workload on the whole GPU: steps x mh MH steps timed"""
    from paper_2006_16622_amd import Chain
    pp = wl.p if p is None else p
    ch = Chain(wl.pos, wl.q, wl.box, wl.depth, pp, flags=flags)
    t = ch.autotune(steps=2000, beta=wl.beta, max_step=wl.max_step) if tune else None
    timed_calls([ch], None, wl.seed, wl.beta, wl.max_step, warmup, mh, 0, resetup_every)
    dt, kern, st = timed_calls([ch], None, wl.seed, wl.beta, wl.max_step, steps, mh, warmup * mh, resetup_every)
    ch.close()
    s0 = st[0]
    total = steps * mh
    out = {"value": total / dt, "unit": "MH steps/s", "mh_steps": total, "kernel_s": kern, "wall_s": dt,
           "p": pp, "accepted": s0["accepted"], "status": s0["status"],
           "t_prop_us": (s0["t_propose_us"] + (s0["t_wait_us"] if flags & 2 else 0)) / total}
    if t is not None:
        out["helpers"] = t["helpers"]
    if resetup_every:
        out["resetup_every"] = resetup_every
    return out


def mixed_drift(wl, mh_steps=20000, count=200):
    """What an FP64 re-setup removes after about 10^4 accepts, measured on
    what the expansions are for: the dE of `count` proposals from the
    state reached (charges and displacements from a fixed numpy stream),
    evaluated on the maintained expansions and again after a fresh FP64
    re-setup, as the RMS and largest difference relative to RMS dE; and the
    running energy against the fresh energy. In mixed precision and, for
    contrast, in FP64 (where the two differ only by the truncation of the
    P2L updates against that of M2L)."""
    from paper_2006_16622_amd import FMM_MC_MIXED, Chain, run_chains
    out = {}
    for name, flags in (("mixed", FMM_MC_MIXED), ("f64", 0)):
        ch = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=flags)
        st = run_chains([ch], mh_steps, wl.seed, wl.beta, wl.max_step)
        pos = ch.positions()
        g = np.random.default_rng(5)
        idx = g.integers(0, wl.n, count)
        moves = [(int(i), pos[i] + g.uniform(-wl.max_step, wl.max_step, 3)) for i in idx]
        kept = np.array([ch.propose(i, r) for i, r in moves])
        u_run = ch.running_energy()
        ch.resetup()
        fresh = np.array([ch.propose(i, r) for i, r in moves])
        u_fresh = ch.running_energy()
        ch.close()
        rms = float(np.sqrt(np.mean(fresh ** 2)))
        out[name] = {"accepts": st[0]["accepted"],
                     "dE_rms_diff_over_rms_dE": float(np.sqrt(np.mean((kept - fresh) ** 2)) / rms),
                     "dE_max_diff_over_rms_dE": float(np.abs(kept - fresh).max() / rms),
                     "energy_diff_over_rms_dE": abs(u_run - u_fresh) / rms}
    return out


def c3_accuracy(wl, ew, count=200):
    """dE of every rock-salt variant against Ewald on the first `count`
    proposals of the stream from the initial state"""
    from paper_2006_16622_amd import FMM_MC_DIRECT_SETUP, FMM_MC_MIXED, FMM_MC_MULTIPOLE
    moves = moves_from_stream(wl, count, wl.pos)
    ref = np.array([ew.propose(i, r) for i, r in moves])
    errs = {}
    for name, flags, p in (("f64", 0, 12), ("mixed", FMM_MC_MIXED, 12), ("direct_setup", FMM_MC_DIRECT_SETUP, 12),
                           ("multipole", FMM_MC_MULTIPOLE, 12), (f"f64_p{P_GATE}", 0, P_GATE),
                           (f"mixed_p{P_GATE}", FMM_MC_MIXED, P_GATE)):
        errs[name] = rel_rms(gpu_proposals(wl, moves, flags, p), ref)
    return errs, moves, ref


def small_configs():
    """the N = 10^3 and N = 10^4 single-chain workloads: all their
    proposals timed from the setup state, and the setup timed"""
    import workloads as W
    from paper_2006_16622_amd import FMM_MC_MIXED, Chain, run_chains
    import torch
    out = {}
    for wl in (W.small(), W.medium()):
        line = {"workload": wl.name, "n": wl.n, "depth": wl.depth, "p": wl.p, "max_step": wl.max_step,
                "proposals": wl.steps}
        for name, flags in (("f64", 0), ("mixed", FMM_MC_MIXED)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ch = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=flags)
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            m2l = ch.last_timing()[1]
            ch.autotune(steps=1000, beta=wl.beta, max_step=wl.max_step)
            # the workload's proposals, once untimed on a clone state (kernel
            # load), then timed from the setup state of a fresh chain
            run_chains([ch], min(wl.steps, 2000), wl.seed, wl.beta, wl.max_step)
            ch.close()
            ch = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=flags)
            resetup = 10000 if flags else 0
            dt, kern, st = timed_calls([ch], None, wl.seed, wl.beta, wl.max_step, 1, wl.steps, 0, resetup)
            ch.close()
            line[name] = {"value": wl.steps / dt, "unit": "MH steps/s", "kernel_s": kern, "wall_s": dt,
                          "nu": st[0]["accepted"] / wl.steps, "status": st[0]["status"],
                          "setup_ms": t_setup * 1e3, "setup_m2l_ms": m2l}
            if flags:
                line[name]["resetup_every"] = resetup
            log(f"[bench] {wl.name} {name}: {line[name]['value']:.0f} MH steps/s, setup {t_setup*1e3:.1f} ms")
        out[wl.name] = line
    return out


def small_configs_accuracy(lines, npre=2000):
    """the chain prefix of npre steps of each small workload, both
    precisions, against the Ewald oracle, whose state follows the accepts"""
    import oracle as O
    import workloads as W
    from paper_2006_16622_amd import FMM_MC_MIXED, Chain, run_chains
    for wl in (W.small(), W.medium()):
        for name, flags in (("f64", 0), ("mixed", FMM_MC_MIXED)):
            ch = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=flags)
            pos0 = ch.positions()
            _, tr = run_chains([ch], npre, wl.seed, wl.beta, wl.max_step, traces=True)
            ch.close()
            ew = O.Ewald(pos0, wl.q, wl.box)
            ref = np.empty(npre)
            for t in range(npre):
                ref[t] = ew.propose(int(tr["idx"][0][t]), tr["newpos"][0][t])
                if tr["acc"][0][t]:
                    ew.accept(int(tr["idx"][0][t]), tr["newpos"][0][t])
            ew.close()
            err = rel_rms(tr["dE"][0], ref)
            if wl.name in lines:
                lines[wl.name][name]["dE_rel_rms_err_vs_ewald"] = err
                lines[wl.name][name]["ewald_sample"] = (f"chain prefix of {npre} steps, the Ewald state follows "
                                                        f"the accepts")
            log(f"[bench] {wl.name} {name}: chain prefix error vs Ewald {err:.2e}")


def run_batched(steps=10000, nchains=256, flags=0, resetup_every=0, seed=4):
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
    steps_c = [w.max_step for w in wls]
    # warmup a few steps (kernel load), then the timed launch
    run_chains(chains, 20, seed, 1.0, steps_c, t0=0, mode=1)
    dt, kern, st = timed_calls(chains, None, seed, 1.0, steps_c, 1, steps, 20, resetup_every, mode=1)
    acc = sum(s["accepted"] for s in st)
    abytes = batched_algorithmic_bytes(wls, st)
    for c in chains:
        c.close()
    return {"value": nchains * steps / dt, "unit": "MH steps/s", "chains": nchains, "steps_per_chain": steps,
            "precision": "mixed" if flags else "f64", "resetup_every": resetup_every,
            "kernel_s": kern, "wall_s": dt, "nu": acc / (nchains * steps), "setup_s": t_setup,
            "setup_m2l_ms": m2l_ms,
            "nu_per_chain": [s["accepted"] / steps for s in st],
            "roofline": {"bound": "hbm", "achieved": abytes / kern / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": abytes / kern / 1e9 / HBM_PEAK_GBS, "kernel": "k_run_chains",
                         "algorithmic_bytes": abytes,
                         "traffic": measured_traffic(nchains * steps, batched=True) if not flags else None,
                         "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)"},
            "n_range": [min(w.n for w in wls), max(w.n for w in wls)],
            "depths": {str(d): sum(1 for w in wls if w.depth == d) for d in sorted({w.depth for w in wls})},
            "status": [s["status"] for s in st if s["status"] != 0][:4]}


def batched_accuracy(count=200):
    """8 sampled chains of the batched workload (depths 2, 3, 4): dE of the
    first `count` proposals from the initial state, both precisions, against
    the Ewald oracle (relative RMS) and the FP64 multilevel oracle (largest
    difference relative to RMS dE)"""
    import oracle as O
    import workloads as W
    from paper_2006_16622_amd import FMM_MC_MIXED
    sizes = W.batched_sizes()
    depth = np.array([s[1] for s in sizes])
    picks = []
    for d, k in ((2, 2), (3, 3), (4, 3)):
        picks += [int(c) for c in np.nonzero(depth == d)[0][:k]]
    rows = []
    for c in picks:
        w = W.batched_chain(c)
        moves = moves_from_stream(w, count, w.pos, chain=c)
        ew = O.Ewald(w.pos, w.q, w.box)
        ref = np.array([ew.propose(i, r) for i, r in moves])
        ew.close()
        orc = O.Multilevel(w.pos, w.q, w.box, w.depth, w.p)
        de_o = np.array([orc.propose(i, r) for i, r in moves])
        orc.close()
        rms = float(np.sqrt(np.mean(de_o ** 2)))
        row = {"chain": c, "n": w.n, "depth": w.depth}
        for name, flags in (("f64", 0), ("mixed", FMM_MC_MIXED)):
            de = gpu_proposals(w, moves, flags)
            row[name] = {"vs_ewald_rel_rms": rel_rms(de, ref),
                         "vs_oracle_max_over_rms": float(np.abs(de - de_o).max() / rms)}
        rows.append(row)
        log(f"[bench] batched accuracy chain {c} (n={w.n}, d={w.depth}): f64 {row['f64']['vs_ewald_rel_rms']:.2e} "
            f"/ {row['f64']['vs_oracle_max_over_rms']:.1e}, mixed {row['mixed']['vs_ewald_rel_rms']:.2e} "
            f"/ {row['mixed']['vs_oracle_max_over_rms']:.1e}")
    return {"sample": f"{count} proposals of each chain's stream from its initial state", "chains": rows,
            "f64_vs_ewald_max": max(r["f64"]["vs_ewald_rel_rms"] for r in rows),
            "mixed_vs_ewald_max": max(r["mixed"]["vs_ewald_rel_rms"] for r in rows),
            "f64_vs_oracle_max": max(r["f64"]["vs_oracle_max_over_rms"] for r in rows),
            "mixed_vs_oracle_max": max(r["mixed"]["vs_oracle_max_over_rms"] for r in rows)}


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


def cpu_baseline(wl, nu, ew, nprop=8000, nacc=1000):
    """The FP64 oracle timed on one host core: proposals and accepts of the
    rock-salt workload timed separately on a state whose expansions are not
    initialised (their values do not change the per-step cost; the
    initialisation of 97336 charges is out of reach of one core here), and
    combined as t_prop + nu t_acc at the acceptance rate of the timed GPU
    run (after its warmup). The Ewald oracle beside it."""
    import oracle as O
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
    m.close()
    step = tp + nu * ta
    out = {"value": 1.0 / step, "unit": "MH steps/s", "cores": 1, "kind": "oracle",
           "sample": f"{nprop} proposals and {nacc} accepts of the rocksalt workload on one core "
                     f"(expansions not initialised; lattice moments formed in {t_setup:.1f} s), "
                     f"t_prop={tp*1e3:.3f} ms, t_acc={ta*1e3:.3f} ms, combined at the timed GPU run's "
                     f"acceptance nu={nu:.3f}"}
    moves = moves_from_stream(wl, 200, wl.pos)
    t0 = time.perf_counter()
    for i, r in moves:
        ew.propose(i, r)
    tpe = (time.perf_counter() - t0) / len(moves)
    t0 = time.perf_counter()
    for i, r in moves[:100]:
        ew.accept(i, r)
    tae = (time.perf_counter() - t0) / 100
    out["ewald"] = {"value": 1.0 / (tpe + nu * tae), "unit": "MH steps/s", "cores": 1, "kind": "oracle",
                    "t_prop_ms": tpe * 1e3, "t_acc_ms": tae * 1e3}
    return out


def cpu_baseline_batched(nu_per_chain, nchains_sample=None, nprop=600, nacc=120):
    """The FP64 oracle on every host core at once, one batched chain per
    thread (the oracle calls release the interpreter lock): each sampled
    chain's proposals and accepts timed separately, as above, and combined
    at that chain's acceptance rate in the GPU run. The aggregate rate is
    threads / mean step time."""
    import threading
    import oracle as O
    import workloads as W
    nt = host_threads()
    ns = 2 * nt if nchains_sample is None else nchains_sample
    res = [None] * ns

    def work(c):
        w = W.batched_chain(c)
        m = O.Multilevel(w.pos, w.q, w.box, w.depth, w.p, setup="none")
        draws = [O.draw(w.seed, c, t, w.n, w.max_step) for t in range(nprop)]
        t0 = time.perf_counter()
        for i, d, _ in draws:
            m.propose(i, w.pos[i] + d)
        tp = (time.perf_counter() - t0) / nprop
        t0 = time.perf_counter()
        for i, d, _ in draws[:nacc]:
            m.accept(i, w.pos[i] + d)
        ta = (time.perf_counter() - t0) / nacc
        m.close()
        res[c] = tp + nu_per_chain[c] * ta

    def worker(k):
        for c in range(k, ns, nt):
            work(c)

    old = os.environ.get("OMP_NUM_THREADS")
    t0 = time.perf_counter()
    th = [threading.Thread(target=worker, args=(k,)) for k in range(nt)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    wall = time.perf_counter() - t0
    mean_step = float(np.mean(res))
    return {"value": nt / mean_step, "unit": "MH steps/s", "cores": nt, "kind": "oracle",
            "sample": f"chains 0..{ns - 1} of the batched workload, {nprop} proposals and {nacc} accepts each, "
                      f"one chain per thread on {nt} threads at once ({wall:.1f} s), expansions not initialised, "
                      f"combined at each chain's acceptance in the GPU run; aggregate = threads / mean step time"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed bench steps (fmm_mc_run calls)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed bench steps before them")
    ap.add_argument("--mh-per-step", type=int, default=10000, help="MH steps per bench step")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the N = 1e3 .. 1e6 scaling sweep")
    ap.add_argument("--no-extra", action="store_true", help="only the headline chain")
    ap.add_argument("--batched-steps", type=int, default=10000)
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
    import torch  # noqa: F401
    import workloads as W
    from paper_2006_16622_amd import FMM_MC_MIXED, FMM_MC_MULTIPOLE
    from paper_2006_16622_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    wl = W.rocksalt()
    mh = args.mh_per_step
    h = headline(wl, args.steps, args.warmup, mh)
    out = {
        "metric": "MH steps/s at N=1e5 (1 chain) + aggregate over 256 chains; dE err vs Ewald",
        "value": h["value"],
        "unit": "MH steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n, "depth": wl.depth, "p": wl.p, "beta": wl.beta,
                   "max_step": wl.max_step, "chains": 1, "mh_steps_per_step": mh,
                   "step": f"one fmm_mc_run call of {mh} MH steps on the resident chain",
                   "setup_ms": h["setup_ms"], "setup_m2l_ms": h["setup_m2l_ms"], "autotune": h["autotune"],
                   "acceptance": h["nu"]},
        "kernel_ms_per_step": h["kernel_ms_per_step"],
        "us_per_mh_step": h["us_per_mh_step"],
        "kernel_us_per_mh_step": h["kernel_us_per_mh_step"],
        "t_prop_us": h["t_prop_us"], "t_acc_us": h["t_acc_us"],
        "status": h["status"],
        "roofline": h["roofline"],
    }
    ew = None
    if not args.no_extra:
        log("[bench] rock salt, mixed precision, FP64 re-setup every 10^4 accepts")
        out["single_mixed"] = single_line(wl, args.steps, 1, mh, flags=FMM_MC_MIXED, resetup_every=10000)
        out["single_mixed"]["drift_removed_by_resetup"] = mixed_drift(wl)
        log(f"[bench] mixed {out['single_mixed']['value']:.0f} MH steps/s")
        log(f"[bench] rock salt at p = {P_GATE} (the smallest degree whose dE meets the 1e-5 Ewald gate), "
            "FP64 and mixed")
        out[f"single_p{P_GATE}"] = single_line(wl, max(1, args.steps // 4), 1, mh, p=P_GATE, tune=True)
        out[f"single_p{P_GATE}_mixed"] = single_line(wl, max(1, args.steps // 4), 1, mh, flags=FMM_MC_MIXED,
                                                     p=P_GATE, resetup_every=10000)
        log(f"[bench] p{P_GATE} {out[f'single_p{P_GATE}']['value']:.0f} / "
            f"mixed {out[f'single_p{P_GATE}_mixed']['value']:.0f}")
        log("[bench] direct P2L setup (Alg. L.3)")
        from paper_2006_16622_amd import Chain
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        chd = Chain(wl.pos, wl.q, wl.box, wl.depth, wl.p, flags=4)
        torch.cuda.synchronize()
        out["setup_direct"] = {"wall_ms": (time.perf_counter() - t0) * 1e3, "p2l_ms": chd.last_timing()[1]}
        chd.close()
        log("[bench] multipole-based variant")
        out["single_multipole"] = single_line(wl, max(1, args.steps // 4), 1, mh, flags=FMM_MC_MULTIPOLE, tune=True)
        out["single_multipole"]["variant"] = "multipole (Alg. M.1-M.3)"
        log(f"[bench] multipole {out['single_multipole']['value']:.0f} MH steps/s")
        log("[bench] small and medium workloads")
        out["configs"] = small_configs()
    if not args.no_batched:
        log("[bench] batched 256 chains, FP64")
        out["batched"] = run_batched(steps=args.batched_steps)
        log(f"[bench] batched {out['batched']['value']:.1f} MH steps/s")
        log("[bench] batched 256 chains, mixed precision")
        out["batched_mixed"] = run_batched(steps=args.batched_steps, flags=FMM_MC_MIXED, resetup_every=10000)
        log(f"[bench] batched mixed {out['batched_mixed']['value']:.1f} MH steps/s")
    if not args.no_sweep and not args.no_extra:
        log("[bench] scaling sweep")
        out["sweep"] = run_sweep()
    if not args.no_cpu:
        # the cpu_baseline leg: the oracles' rates, and every error figure
        # above measured against them
        import oracle as O
        if "batched" in out and not args.no_extra:
            log("[bench] accuracy of 8 batched chains against Ewald and the oracle")
            acc = batched_accuracy()
            out["batched"]["accuracy"] = acc
            out["batched_mixed"]["accuracy"] = acc
        if "configs" in out:
            small_configs_accuracy(out["configs"])
        log("[bench] accuracy of the rock-salt variants against Ewald")
        t0 = time.perf_counter()
        ew = O.Ewald(wl.pos, wl.q, wl.box)
        t_ew = time.perf_counter() - t0
        errs, _, _ = c3_accuracy(wl, ew)
        out["dE_rel_rms_err_vs_ewald"] = errs
        out["dE_err_sample"] = ("200 proposals of the Philox stream from the initial rock-salt state; "
                                "direct_setup: local expansions by Alg. L.3; multipole: Alg. M.1-M.3")
        for key, line in (("f64", out), ("mixed", out.get("single_mixed")),
                          (f"f64_p{P_GATE}", out.get(f"single_p{P_GATE}")),
                          (f"mixed_p{P_GATE}", out.get(f"single_p{P_GATE}_mixed")),
                          ("multipole", out.get("single_multipole"))):
            if line is not None:
                line["dE_rel_rms_err_vs_ewald"] = errs[key]
        log(f"[bench] errors vs Ewald: {errs}")
        log("[bench] cpu baseline (oracle), one core")
        out["cpu_baseline"] = cpu_baseline(wl, h["nu"], ew)
        out["cpu_baseline"]["ewald"]["setup_s"] = t_ew
        ew.close()
        if "batched" in out:
            log("[bench] cpu baseline (oracle), batched chains on all host cores")
            out["cpu_baseline"]["batched_all_cores"] = cpu_baseline_batched(out["batched"]["nu_per_chain"])
    out.pop("status") if out.get("status") == 0 else None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
