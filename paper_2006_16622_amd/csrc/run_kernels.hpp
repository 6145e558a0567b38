// run_kernels.hpp -- Metropolis-Hastings chains on the device.
//
//  * k_run_chains (16-lane groups) and k_run_batched (32-lane groups, and
//    the multipole variant): one workgroup per chain, every chain its own
//    state; the workgroup proposes, decides and, on accept, walks every
//    update block itself. No inter-workgroup communication: hundreds of
//    independent chains of uneven size and depth in one launch (independent
//    chains run side by side, one of the routes to parallelism named in
//    Sec. 6). k_run_chains runs the loop of k_run_single's workgroup 0
//    (run_chain_wg) without helpers.
//  * k_run_single: one chain on many workgroups (cooperative launch, all
//    co-resident). Workgroup 0 proposes, decides and keeps the bookkeeping;
//    it posts every move in a mailbox, and the update blocks of Alg. L.2,
//    each owning distinct target cells, are shared out over the other
//    workgroups, which form them speculatively and store them on accept;
//    the next proposal waits for their completion only before it reads the
//    local expansions. The per-level work is spread as the paper suggests
//    for parallelism (Sec. 6).
//
// A step draws (idx, delta, u) from Philox4x64-10 (key = (seed, chain),
// counter = (t, 0|1, 0, 0)) or reads them from fixed lists; the move is
// accepted iff u < exp(-beta dE) and it is not singular. The next move is
// drawn, located and (for the helpers) posted by the last wavefront while
// the current one is being proposed.
#pragma once

#include "mp_step.hpp"

namespace fmmdev {

// A run is `steps` MH steps per chain; a launch may cover part of it: slot
// k of the launch (blockIdx.x, or the single chain) is chain chain_id[k] of
// the run and resumes at step first[k]. A chain stops early once it has
// accepted acc_limit moves in this launch (the caller then re-sets it up
// and launches the rest).
struct RunParams {
  int64_t steps, t0;
  uint64_t seed;
  double beta;
  const double *max_step;  // per chain of the run, null: max_step0 for every chain
  const int64_t *first;    // per slot, null: first0 for every slot
  const int *chain_id;     // per slot, null: the slot
  double max_step0;
  int64_t first0;
  int64_t acc_limit;       // 0: none
  // fixed-list source (replay) when list_idx != nullptr
  const int64_t *list_idx;
  const double *list_pos;
  const double *list_u;
  // traces, [chain * steps + t], may be null
  int64_t *tr_idx;
  double *tr_pos, *tr_dE;
  uint8_t *tr_acc;
  int32_t *tr_leaf;
  double *stats;           // per slot RUN_NSTAT doubles: proposed, accepted, singular, dE_sum, status,
                           // three times, running energy at the end of the launch
};

constexpr int RUN_NSTAT = 10;

__device__ __forceinline__ double run_max_step(const RunParams &rp, int c) {
  return rp.max_step ? rp.max_step[c] : rp.max_step0;
}
__device__ __forceinline__ int64_t run_first(const RunParams &rp, int slot) {
  return rp.first ? rp.first[slot] : rp.first0;
}

// the draw of one step and the record of its particle (LDS)
struct NextDraw {
  int64_t idx;
  double d[3];   // displacement (Philox) or absolute new position (list)
  double u;
  double r[3];   // particle position when fetched
  double q;
};

__device__ __forceinline__ void draw_into(const RunParams &rp, int c, int64_t t, const Chain &ch, double D,
                                          NextDraw &nd) {
  if (rp.list_idx) {
    nd.idx = rp.list_idx[t];
    for (int k = 0; k < 3; ++k) nd.d[k] = rp.list_pos[3 * t + k];
    nd.u = rp.list_u[t];
  } else {
    mh_draw(rp.seed, (uint64_t)c, (uint64_t)(rp.t0 + t), ch.N, D, nd.idx, nd.d, nd.u);
  }
  nd.r[0] = glb(ch.px)[nd.idx];
  nd.r[1] = glb(ch.py)[nd.idx];
  nd.r[2] = glb(ch.pz)[nd.idx];
  nd.q = glb(ch.pq)[nd.idx];
}

// The random part of a draw (no memory of the chain's state): lane 0 forms
// idx and the displacement (Philox counter (t, 0)), lane 1 the uniform
// (counter (t, 1)), side by side; in list mode lane 0 reads the lists.
struct RngDraw {
  int64_t idx;
  double d[3];
  double u;
};

__device__ __forceinline__ void rng_into(const RunParams &rp, int c, int64_t t, int64_t N, double D, int lane,
                                         RngDraw &out) {
#pragma clang fp contract(off)
  if (rp.list_idx) {
    if (lane == 0) {
      out.idx = rp.list_idx[t];
      for (int k = 0; k < 3; ++k) out.d[k] = rp.list_pos[3 * t + k];
      out.u = rp.list_u[t];
    }
    return;
  }
  if (lane >= 2) return;
  // both counters in one instruction stream (lane 0: (t, 0), lane 1: (t, 1))
  uint64_t w[4] = {(uint64_t)(rp.t0 + t), (uint64_t)lane, 0, 0};
  philox4x64_10(w, rp.seed, (uint64_t)c);
  const double two53 = 1.0 / 9007199254740992.0;
  if (lane == 0) {
    out.idx = (int64_t)__umul64hi(w[0], (uint64_t)N);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double f = (double)(w[k + 1] >> 11) * two53;
      double two_f = 2.0 * f;
      double centred = two_f - 1.0;
      out.d[k] = D * centred;
    }
  } else {
    out.u = (double)(w[0] >> 11) * two53;
  }
}

// Build the move of a step from its draw (thread 0). If the previous step
// accepted a move of the same particle after the draw was fetched, its new
// position replaces the fetched one.
__device__ __forceinline__ void move_from_draw(const RunParams &rp, const Chain &ch, const NextDraw &nd,
                                               bool prev_acc, int prev_idx, const double prev_rn[3],
                                               Move &mv) {
#pragma clang fp contract(off)
  double r[3];
  const bool moved = prev_acc && prev_idx == (int)nd.idx;
  for (int k = 0; k < 3; ++k) r[k] = moved ? prev_rn[k] : nd.r[k];
  mv.idx = (int)nd.idx;
  mv.q = nd.q;
  for (int k = 0; k < 3; ++k) {
    mv.r[k] = r[k];
    double rn_abs = rp.list_idx ? nd.d[k] : r[k] + nd.d[k];
    mv.rn[k] = ch.free_space ? rn_abs : wrap_coord(rn_abs, ch.a);
  }
}

// one workgroup per CU is the shape of the batched launch (256 chains), so
// a workgroup may use the whole register file (2 wavefronts per SIMD)
// The Metropolis test u < exp(-beta dE), u in [0, 1). With beta > 0 a move
// with dE <= 0 passes it whatever u is (exp(-beta dE) >= 1 > u), so the
// exponential is formed only for the others; every decision is the one
// the comparison itself gives.
__device__ __forceinline__ bool mh_accept(double u, double beta, double dE) {
  return (beta > 0.0 && dE <= 0.0) || u < exp(-beta * dE);
}

template <int GS, int PM, typename R, bool MP = false>
__global__ void __launch_bounds__(WG_BATCH) __attribute__((amdgpu_waves_per_eu(1, 2)))
k_run_batched(const Chain *chains, Tabs tb, RunParams rp) {
  constexpr int NT = WG_BATCH;
  constexpr int NG = NT / GS;
  extern __shared__ double lds[];
  __shared__ Move mv;
  __shared__ NextDraw nd;
  __shared__ int s_acc, s_ovf;
  __shared__ double s_u;
  __shared__ Chain chl;  // the chain's descriptor, indexed by level without scratch
  const int slot = blockIdx.x, t = threadIdx.x;
  const int c = rp.chain_id ? rp.chain_id[slot] : slot;
  const int64_t s0 = run_first(rp, slot);
  if (t == 0) chl = chains[slot];
  __syncthreads();
  const Chain &ch = chl;
  Lds<GS, NT> sm(lds, tb.Cs, tb.lat_lds ? tb.lat_w : 0);
  stage_lds(ch, tb, sm, true);
  const double D = run_max_step(rp, c);
  double nprop = 0, nacc = 0, nsing = 0, dEsum = 0;
  uint64_t tick_prop = 0, tick_acc = 0;
  int status = 0;
  bool prev_acc = false;
  int prev_idx = -1;
  double prev_rn[3] = {0, 0, 0};
  int64_t acc_launch = 0;
  if (t == 0 && s0 < rp.steps) draw_into(rp, c, s0, ch, D, nd);
  __syncthreads();
  for (int64_t step = s0; step < rp.steps; ++step) {
    uint64_t t_0 = __builtin_amdgcn_s_memrealtime();
    if (t == 0) {
      move_from_draw(rp, ch, nd, prev_acc, prev_idx, prev_rn, mv);
      s_u = nd.u;
    }
    __syncthreads();
    locate_move_par(ch, mv);
    __syncthreads();
    const double u = s_u;
    auto fetch = [&](int lane) {
      if (lane == 0 && step + 1 < rp.steps) draw_into(rp, c, step + 1, ch, D, nd);
    };
    ProposeOut po;
    if constexpr (MP)
      po = propose_mp_wg<GS, PM>(ch, tb, mv, sm, fetch);
    else
      po = propose_wg<GS, PM, R>(ch, tb, mv, sm, fetch);
    uint64_t t_1 = __builtin_amdgcn_s_memrealtime();
    tick_prop += t_1 - t_0;
    if (t == 0) {
      int acc = !po.singular && mh_accept(u, rp.beta, po.dE);
      // a move that would overflow its new leaf bin is not taken: the chain
      // stops with the error and its state is that before the move
      s_ovf = acc && move_overflows(ch, mv, sm.ints);
      if (s_ovf) acc = 0;
      s_acc = acc;
      nprop += 1;
      nsing += po.singular;
      int64_t o = (int64_t)c * rp.steps + step;
      if (rp.tr_idx) glb(rp.tr_idx)[o] = mv.idx;
      if (rp.tr_pos)
        for (int k = 0; k < 3; ++k) glb(rp.tr_pos)[3 * o + k] = mv.rn[k];
      if (rp.tr_dE) glb(rp.tr_dE)[o] = po.dE;
      if (rp.tr_acc) glb(rp.tr_acc)[o] = (uint8_t)acc;
      if (rp.tr_leaf) {
        int n = 1 << (ch.L - 1);
        glb(rp.tr_leaf)[o] = lin3(n, mv.c1[ch.L][0], mv.c1[ch.L][1], mv.c1[ch.L][2]);
      }
    }
    __syncthreads();
    prev_acc = s_acc;
    if (s_ovf) {
      status = -7;
      break;
    }
    prev_idx = mv.idx;
    for (int k = 0; k < 3; ++k) prev_rn[k] = mv.rn[k];
    if (prev_acc) {
      if constexpr (MP)
        accept_mp_wg<GS, PM, NT>(ch, tb, mv, sm.rec);
      else
        accept_all_wg<GS, PM, R, NT>(ch, tb, mv, sm);
      int ovf = accept_bookkeeping<GS, PM, !MP>(ch, tb, mv, po.dE, sm);
      if (t == 0) {
        nacc += 1;
        dEsum += po.dE;
      }
      tick_acc += __builtin_amdgcn_s_memrealtime() - t_1;
      if (ovf) {
        status = -7;
        break;
      }
      if (rp.acc_limit && ++acc_launch >= rp.acc_limit) break;
    }
  }
  __syncthreads();
  writeback_lds(ch, tb, sm);
  if (t == 0) {
    const auto st = glb(rp.stats) + RUN_NSTAT * slot;
    st[0] = nprop;
    st[1] = nacc;
    st[2] = nsing;
    st[3] = dEsum;
    st[4] = status;
    st[5] = tick_prop * 0.01;  // microseconds (100 MHz clock)
    st[6] = tick_acc * 0.01;
    st[7] = 0.0;
    st[8] = sm.st[3];
  }
}

// ---------------------------------------------------------------- single chain
// Polling uses relaxed agent-scope loads (no cache invalidation per poll);
// the caller issues one acquire fence after the awaited value is seen.
__device__ __forceinline__ unsigned ld_relaxed(unsigned *p) {
  return __hip_atomic_load(glb(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(unsigned *p, unsigned v) {
  __hip_atomic_store(glb(p), v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(unsigned *p, unsigned v) {
  __hip_atomic_store(glb(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every spin is bounded: it returns false after `limit` ticks of the
// 100 MHz clock.
// spin until the counter *p has reached `target` (counters of one launch
// stay far below 2^31, so the signed difference orders them)
__device__ __forceinline__ bool spin_until_reached(unsigned *p, unsigned target, uint64_t limit) {
  uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  while (true) {
    if ((int)(ld_relaxed(p) - target) >= 0) return true;
    if (__builtin_amdgcn_s_memrealtime() - t0 > limit) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}
// spin by a whole wavefront until *p differs from `old`: the value is made
// uniform, so every lane takes the same exit
__device__ __forceinline__ bool wave_spin_until_ne(unsigned *p, unsigned old, unsigned &val, uint64_t limit) {
  uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  while (true) {
    val = __builtin_amdgcn_readfirstlane(ld_relaxed(p));
    if (val != old) return true;
    if (__builtin_amdgcn_s_memrealtime() - t0 > limit) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}
// wavefront 0 waits until flags[1..G-1] all equal `target` (one flag per
// helper workgroup, so the completions do not contend on one address)
__device__ __forceinline__ bool spin_all_equal(unsigned *flags, int G, unsigned target, uint64_t limit) {
  const int lane = threadIdx.x & 63;
  uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  while (true) {
    // the first four flags of this lane are all requested before any is
    // compared, so a poll whose flags are already set takes one round trip
    unsigned v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int w = 1 + lane + 64 * i;
      v[i] = w < G ? ld_relaxed(&flags[w]) : target;
    }
    bool mine = v[0] == target && v[1] == target && v[2] == target && v[3] == target;
    for (int w = 257 + lane; w < G; w += 64) mine = mine && (ld_relaxed(&flags[w]) == target);
    if (__all(mine)) return true;
    if (__builtin_amdgcn_s_memrealtime() - t0 > limit) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}

// The order in which the H helpers of the whole-GPU run take the nblk accept
// blocks: helper w takes the positions w - 1, w - 1 + H, ... The blocks
// differ in weight: a level-2 cell has some 47 candidate terms, a level-3
// cell a few, and a fine block of bpl blocks per level holds its level's
// old-side items (its first jh blocks, two terms per active item) or
// new-side ones (mostly owned by the old side, when r and r' share a cell).
// With two blocks per helper (nblk = 2 H) the first H positions hold the
// level-2 cells, the old-side fine blocks and level-3 cells, the second H the
// level-3 cells that pair with the level-2 ones, the new-side fine blocks
// that pair with the old-side ones, and the other level-3 cells. Otherwise
// the level-2 cells come first, then the fine blocks with 8 level-3 cells at
// positions H .. H + 7 (the second block of a level-2 holder), then the other
// level-3 cells. Without fine blocks the order is the block order.
// Returns the block at position v.
__host__ __device__ inline int block_at(int v, int H, int nblk, int bpl, int jh) {
  if (v < 8 || nblk <= 72) return v;
  const int F = nblk - 72;  // fine blocks: F / bpl levels, jh old-side blocks on each
  if (2 * H == nblk) {
    const int Fh = F / bpl * jh, Fl = F - Fh, x = H - 8 - Fh;
    if (v < 8 + Fh) {
      const int i = v - 8;
      return 72 + i / jh * bpl + i % jh;
    }
    if (v < H) return 16 + (v - 8 - Fh);
    if (v < H + 8) return 8 + (v - H);
    if (v < H + 8 + Fl) {
      const int i = v - H - 8, nl = bpl - jh;
      return 72 + i / nl * bpl + jh + i % nl;
    }
    return 16 + x + (v - H - 8 - Fl);
  }
  const int A = H - 8 < 0 ? 0 : (H - 8 > F ? F : H - 8);  // fine blocks before the 8 level-3 cells
  if (v < 8 + A) return 72 + (v - 8);
  if (v < 16 + A) return 8 + (v - 8 - A);
  if (v < 16 + F) return 72 + (v - 16);
  return 16 + (v - 16 - F);
}
// the helper (1 .. H) that holds fine block b >= 72
__host__ __device__ inline int helper_of_fine(int b, int H, int nblk, int bpl, int jh) {
  const int F = nblk - 72, f = b - 72;
  int v;
  if (2 * H == nblk) {
    const int li = f / bpl, j = f % bpl;
    v = j < jh ? 8 + li * jh + j : H + 8 + li * (bpl - jh) + (j - jh);
  } else {
    const int A = H - 8 < 0 ? 0 : (H - 8 > F ? F : H - 8);
    v = f < A ? 8 + f : 16 + f;
  }
  return 1 + v % H;
}

// a helper's wait before it reads target rows: wavefront 0 polls the done
// flags of the helpers holding fine-level blocks (levels 4..L, bpl blocks
// each; fine block b belongs to helper_of_fine(b)) of the levels in `lvmask`
// until all have reached `target` (a flag may already be past it)
__device__ __forceinline__ bool spin_level_helpers(unsigned *flags, int G, int nblk, unsigned lvmask, int bpl, int jh,
                                                   unsigned target, uint64_t limit) {
  const int lane = threadIdx.x & 63;
  uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  while (true) {
    bool mine = true;
    for (int l = 4; l < 32; ++l) {
      if (!((lvmask >> l) & 1u)) continue;
      const int b0 = 72 + (l - 4) * bpl;
      for (int b = b0 + lane; b < b0 + bpl; b += 64)
        mine = mine && ((int)(ld_relaxed(&flags[helper_of_fine(b, G - 1, nblk, bpl, jh)]) - target) >= 0);
    }
    if (__all(mine)) return true;
    if (__builtin_amdgcn_s_memrealtime() - t0 > limit) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}

constexpr uint64_t SPIN_LIMIT = 100000000ull * 20;  // 20 s of the 100 MHz clock
constexpr int SPEC_MAX = 8;  // accept blocks one helper of the whole-GPU run can hold

// dynamic LDS a helper of the whole-GPU run needs beyond the standard
// layout when the busiest helper holds k accept blocks
__host__ __device__ inline size_t spec_extra_bytes(int k, int NG, int Cs) {
  return (size_t)(k - 1) * NG * Cs * sizeof(double) + (size_t)k * NG * sizeof(double *);
}

// post move `num` in its mailbox slot (one thread). The slot is written with
// agent-scope atomic stores, which write through this XCD's L2; once they
// have completed, the number is stored, and a helper that sees it acquires
// at agent scope (its L2 is invalidated) before it reads the slot. A release
// fence would add a write-back of the whole L2 for plain stores, which the
// helpers do not read.
__device__ __forceinline__ void post_move(double *mb, unsigned *mvseq, unsigned num, const Move &mv) {
  const auto slot = glb(mb) + 8 * (num & 3);
  const double v[8] = {(double)mv.idx, mv.q, mv.r[0], mv.r[1], mv.r[2], mv.rn[0], mv.rn[1], mv.rn[2]};
#pragma unroll
  for (int k = 0; k < 8; ++k) __hip_atomic_store(slot + k, v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  st_relaxed(mvseq, num);
}

// the same in two halves, so that the wavefront does not wait for its
// stores where it would hold up the workgroup: post_issue writes the slot,
// post_publish (later) waits for those stores and stores the number
__device__ __forceinline__ void post_issue(double *mb, unsigned num, const Move &mv) {
  const auto slot = glb(mb) + 8 * (num & 3);
  const double v[8] = {(double)mv.idx, mv.q, mv.r[0], mv.r[1], mv.r[2], mv.rn[0], mv.rn[1], mv.rn[2]};
#pragma unroll
  for (int k = 0; k < 8; ++k) __hip_atomic_store(slot + k, v[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void post_publish(unsigned *mvseq, unsigned num) {
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  st_relaxed(mvseq, num);
}

// the whole workgroup: wavefront 0 waits until every helper has finished
// move `target`, then every thread acquires their rows; false on time-out
// (flag: LDS word, 0 or 1)
__device__ __forceinline__ bool wait_helpers(unsigned *doneflag, int G, unsigned target, int *flag) {
  if (threadIdx.x < 64) {
    bool ok = spin_all_equal(doneflag, G, target, SPIN_LIMIT);
    if (threadIdx.x == 0) *flag = ok ? 0 : 1;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const bool ok = *flag == 0;
  __syncthreads();
  return ok;
}

// gate of a proposal that follows an accepted move (active when `on`):
// wait for the helpers' rows of move num - 1. ticks: LDS, the time of the
// wait (thread 0).
struct HelperGate {
  bool on;
  int G;
  unsigned num;
  unsigned *doneflag;
  int *flag;
  uint64_t *ticks;
  __device__ bool active() const { return on; }
  __device__ void operator()() const {
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    wait_helpers(doneflag, G, num - 1, flag);
    if (threadIdx.x == 0) *ticks = __builtin_amdgcn_s_memrealtime() - t0;
  }
};

// Protocol of the whole-GPU chain (sync words of the workspace):
//   sync[0] mvseq   number of the latest posted move (1, 2, ... per launch)
//   sync[1] dec     2 * number + accepted, once that move is decided
//   sync[2] stop, sync[3] error, sync[64 + w] done flag of helper w (the
//                   number of the last accepted move whose rows it stored)
//   mailbox         two slots of 8 doubles (idx, q, r, r'), slot = number & 1
// Workgroup 0 posts each move at the start of its proposal. Every helper
// takes the moves in order; for each it reads the move, locates it and
// forms, in LDS, the updated rows of its accept blocks without writing them
// (speculation), then waits for the decision. If accepted, it stores those
// rows and raises its done flag; else they are dropped. A fine-level target
// row may belong to another helper on the next move, so before a
// speculation reads any row the helper waits until the done flags of the
// helpers holding blocks of its fine levels have reached the last accepted
// move. Workgroup 0 does its bookkeeping meanwhile; its next
// proposal forms every term that does not read a local expansion and then
// waits for all done flags (the gate).
// Hence the decision of a move m is published only after every helper has
// stored the accepted move before it: a helper that finds the decision word
// already past m knows m was rejected, and a mailbox slot, rewritten two
// moves later, can only have changed under a helper still reading a
// rejected move (whose rows are dropped). A helper that finds a move
// already decided rejected skips it. Every wait is bounded; on time-out the
// chain stops with an error status.
template <int GS, int PM, typename R, bool BATCH>
__device__ __forceinline__ void run_chain_wg(const Chain &ch_arg, const Tabs &tb, const RunParams &rp) {
  constexpr int NT = WG_SINGLE;
  constexpr int NG = NT / GS;
  // groups of 16 lanes: the proposal of propose_fast, with the next move
  // formed one step ahead (two move buffers); otherwise propose_wg
  constexpr bool FAST = GS == 16;
  extern __shared__ double lds[];
  __shared__ Move mvs[2];  // workgroup 0: this step's move and the next; helpers use mvs[0]
  Move &mv = mvs[0];
  __shared__ NextDraw nd;
  __shared__ RngDraw s_rng[2];  // workgroup 0: random part of the draws of the next steps, by step parity
  __shared__ int s_flag, s_acc, s_ovf, s_sing;
  __shared__ unsigned s_seq;
  __shared__ double s_u, s_dE;
  __shared__ uint64_t s_ticks;
  __shared__ Chain chl;  // the chain's descriptor, indexed by level without scratch
  // BATCH: every workgroup runs its own chain alone (slot blockIdx.x)
  const int t = threadIdx.x, w = BATCH ? 0 : (int)blockIdx.x, G = BATCH ? 1 : (int)gridDim.x;
  const int slot = BATCH ? (int)blockIdx.x : 0;
  if (t == 0) chl = ch_arg;
  __syncthreads();
  const Chain &ch = chl;
  const int nblk = accept_blocks(ch.L, NG);
  unsigned *mvseq = ch.sync, *dec = ch.sync + 1, *stop = ch.sync + 2, *err = ch.sync + 3;
  unsigned *doneflag = ch.sync + 64;
  double *mb = ch.mbox;
  Lds<GS, NT> sm(lds, tb.Cs, tb.lat_lds ? tb.lat_w : 0);
  stage_lds(ch, tb, sm, w == 0);
  __syncthreads();
  if (w == 0) {
    const int c = rp.chain_id ? rp.chain_id[slot] : slot;
    const double D = run_max_step(rp, c);
    double nprop = 0, nacc = 0, nsing = 0, dEsum = 0;
    int status = 0;
    unsigned num = 0;  // move number of this launch
    uint64_t tick_prop = 0, tick_acc = 0, tick_wait = 0;
    bool prev_acc = false;
    int prev_idx = -1;
    double prev_rn[3] = {0, 0, 0};
    const int64_t s0 = run_first(rp, slot);
    int64_t acc_launch = 0;
    // the rows of the last accepted move may still be in flight (helpers
    // finish them while the next proposal forms its other terms)
    bool pending = false;
    if constexpr (FAST) {
      // the move of the first step, posted at once, and the random part of
      // the next draw
      if (s0 < rp.steps) {
        if (t == 0) {
          draw_into(rp, c, s0, ch, D, nd);
          move_from_draw(rp, ch, nd, false, -1, prev_rn, mvs[0]);
          mvs[0].u = nd.u;
        }
        if (t < 64 && s0 + 1 < rp.steps) rng_into(rp, c, s0 + 1, ch.N, D, t, s_rng[(s0 + 1) & 1]);
        __syncthreads();
        locate_move_par(ch, mvs[0]);
        __syncthreads();
        if (t == 0 && G > 1) post_move(mb, mvseq, 1u, mvs[0]);
      }
    } else {
      if (t == 0 && s0 < rp.steps) draw_into(rp, c, s0, ch, D, nd);
      __syncthreads();
    }
    int cur = 0;
    double nxr[3] = {0, 0, 0}, nxq = 0;  // the last wavefront's lane 0: position and charge of the next draw
    for (int64_t step = s0; step < rp.steps; ++step) {
      uint64_t t_0 = __builtin_amdgcn_s_memrealtime();
      ++num;  // every thread keeps the move number
      const bool more = step + 1 < rp.steps;
      HelperGate gate{pending, G, num, doneflag, &s_flag, &s_ticks};
      double dE_step;
      if constexpr (FAST) {
        const Move &mc = mvs[cur];
        Move &mn = mvs[cur ^ 1];
        // The next move is formed during this proposal from the position
        // its draw reads now (a later fix-up covers an accept of the same
        // charge), posted (stores only) and published with this move's
        // decision, so the helpers find it waiting when they finish this
        // one. The random part of the draw after it is formed meanwhile.
        RngDraw &rn1 = s_rng[(step + 1) & 1];
        propose_fast<GS, PM, R, NT>(
            ch, tb, mc, sm,
            [&](int lane) {  // the position of the next draw; the draw after it
              if (lane == 0 && more) {
                const int64_t i = rn1.idx;
                nxr[0] = glb(ch.px)[i];
                nxr[1] = glb(ch.py)[i];
                nxr[2] = glb(ch.pz)[i];
                nxq = glb(ch.pq)[i];
              }
              if (step + 2 < rp.steps) rng_into(rp, c, step + 2, ch.N, D, lane, s_rng[step & 1]);
            },
            [&](int lane) {  // the next move, located and posted
              if (!more) return;
              if (lane == 0) {
                nd.idx = rn1.idx;
                for (int k = 0; k < 3; ++k) {
                  nd.d[k] = rn1.d[k];
                  nd.r[k] = nxr[k];
                }
                nd.u = rn1.u;
                nd.q = nxq;
                move_from_draw(rp, ch, nd, false, -1, prev_rn, mn);
                mn.u = nd.u;
              }
              __builtin_amdgcn_wave_barrier();
              __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
              locate_move_level(ch, mn, lane + 1);
              if (lane == 0 && G > 1) post_issue(mb, num + 1, mn);
            },
            gate,
            [&](double dE, int sing) {  // one thread (lane 0 of the last wavefront)
              int acc = !sing && mh_accept(mc.u, rp.beta, dE);
              // a move that would overflow its new leaf bin is published as
              // rejected (the helpers drop its rows) and the chain stops
              s_ovf = acc && move_overflows(ch, mc, sm.ints);
              if (s_ovf) acc = 0;
              s_acc = acc;
              s_dE = dE;
              s_sing = sing;
            });
        dE_step = s_dE;
        if (t == 0) {  // the counters live in thread 0, which writes the results
          nprop += 1;
          nsing += s_sing;
        }
      } else {
        if (t == 0) {
          move_from_draw(rp, ch, nd, prev_acc, prev_idx, prev_rn, mv);
          s_u = nd.u;
        }
        __syncthreads();
        locate_move_par(ch, mv);
        __syncthreads();
        const double u = s_u;
        // the last wavefront of the proposal posts the move to the helpers
        // first and later fetches the next draw
        ProposeOut po = propose_wg<GS, PM, R>(
            ch, tb, mv, sm,
            [&](int lane) {
              if (lane == 0 && more) draw_into(rp, c, step + 1, ch, D, nd);
            },
            [&](int lane) {
              if (lane == 0 && G > 1) post_move(mb, mvseq, num, mv);
            },
            gate);
        if (t == 0) {
          int acc = !po.singular && mh_accept(u, rp.beta, po.dE);
          s_ovf = acc && move_overflows(ch, mv, sm.ints);
          if (s_ovf) acc = 0;
          s_acc = acc;
          nprop += 1;
          nsing += po.singular;
        }
        __syncthreads();
        dE_step = po.dE;
      }
      const Move &m = mvs[FAST ? cur : 0];
      uint64_t t_1 = __builtin_amdgcn_s_memrealtime();
      const uint64_t gate_ticks = pending ? s_ticks : 0;
      tick_prop += t_1 - t_0 - gate_ticks;
      tick_wait += gate_ticks;
      if (pending) {
        pending = false;
        if (s_flag) {  // a helper did not finish the last accepted move
          status = -8;
          break;
        }
      }
      prev_acc = s_acc;
      // the decision (a relaxed store: it publishes no data) and the traces
      // are stored by the last wavefront, so that the wavefront that starts
      // the next step has no store outstanding
      if (t == NT - 64) {
        // the next move, posted during the proposal, is published first
        // (its stores are long complete), unless this accepted move moved
        // the same charge
        if (FAST && G > 1 && more && !(prev_acc && (int)nd.idx == m.idx)) post_publish(mvseq, num + 1);
        if (G > 1) st_relaxed(dec, 2u * num + (unsigned)prev_acc);
        const int64_t o = (int64_t)c * rp.steps + step;
        if (rp.tr_idx) glb(rp.tr_idx)[o] = m.idx;
        if (rp.tr_pos)
          for (int k = 0; k < 3; ++k) glb(rp.tr_pos)[3 * o + k] = m.rn[k];
        if (rp.tr_dE) glb(rp.tr_dE)[o] = dE_step;
        if (rp.tr_acc) glb(rp.tr_acc)[o] = (uint8_t)prev_acc;
        if (rp.tr_leaf) {
          int n = 1 << (ch.L - 1);
          glb(rp.tr_leaf)[o] = lin3(n, m.c1[ch.L][0], m.c1[ch.L][1], m.c1[ch.L][2]);
        }
      }
      if (s_ovf) {
        status = -7;
        break;
      }
      prev_idx = m.idx;
      for (int k = 0; k < 3; ++k) prev_rn[k] = m.rn[k];
      if (prev_acc) {
        if (G == 1) accept_all_wg<GS, PM, R>(ch, tb, m, sm);
        int ovf = accept_bookkeeping<GS, PM, true>(ch, tb, m, dE_step, sm);
        if (t == 0) {
          nacc += 1;
          dEsum += dE_step;
        }
        tick_acc += __builtin_amdgcn_s_memrealtime() - t_1;
        // the next proposal waits for the helpers (gate) only where it
        // reads the expansions
        pending = G > 1;
        if (ovf) {
          status = -7;
          break;
        }
        if (rp.acc_limit && ++acc_launch >= rp.acc_limit) break;
      }
      if constexpr (FAST) {
        // the next move was formed from the position the draw read; if this
        // accepted move moved the same charge, it is formed again from the
        // new position (a uniform condition: LDS values)
        if (more) {
          if (prev_acc && (int)nd.idx == prev_idx) {
            if (t == 0) {
              move_from_draw(rp, ch, nd, true, prev_idx, prev_rn, mvs[cur ^ 1]);
              mvs[cur ^ 1].u = nd.u;
            }
            __syncthreads();
            locate_move_par(ch, mvs[cur ^ 1]);
            __syncthreads();
            if (t == 0 && G > 1) post_move(mb, mvseq, num + 1, mvs[cur ^ 1]);
          }
          cur ^= 1;
        }
      }
    }
    // a helper must have stored the last accepted move before it is stopped
    if (pending) {
      uint64_t t_2 = __builtin_amdgcn_s_memrealtime();
      if (!wait_helpers(doneflag, G, num, &s_flag) && status == 0) status = -8;
      tick_wait += __builtin_amdgcn_s_memrealtime() - t_2;
    }
    if (G > 1 && t == 0) {
      st_release(stop, 1u);
      st_release(mvseq, num + 1);
    }
    __syncthreads();
    writeback_lds(ch, tb, sm);
    if (t == 0) {
      const auto st = glb(rp.stats) + RUN_NSTAT * slot;
      st[0] = nprop;
      st[1] = nacc;
      st[2] = nsing;
      st[3] = dEsum;
      st[4] = status;
      st[5] = tick_prop * 0.01;  // microseconds (100 MHz clock)
      st[6] = tick_acc * 0.01;
      st[7] = tick_wait * 0.01;
      st[8] = sm.st[3];
    }
    return;
  }
  // ---- helper workgroups: block k of this helper (positions w-1, w-1+G-1, ...
  // of block_at's order)
  // forms its rows in spec(k): the group buffers for k = 0, then the dynamic
  // LDS after the standard layout; then the row pointers of all its blocks
  const int kmax = (nblk + G - 2) / (G - 1);  // blocks of the busiest helper
  double *xbuf = lds + Lds<GS, NT>::bytes(tb.Cs, tb.lat_lds ? tb.lat_w : 0) / sizeof(double);
  double **sdst = (double **)(xbuf + (size_t)(kmax - 1) * NG * tb.Cs);
  auto spec = [&](int k) { return k == 0 ? sm.gbuf : xbuf + (size_t)(k - 1) * NG * tb.Cs; };
  __shared__ bool s_coarse[SPEC_MAX];
  __shared__ int s_skip;
  unsigned cur = 0;        // number of the last move taken
  unsigned last_acc = 0;   // the last accepted move this helper stored
  unsigned confirmed = 0;  // the rows this helper reads hold the accepted moves up to this one
  // levels of this helper's fine blocks: their rows change owner from move
  // to move (the coarse blocks of levels 2 and 3 always belong to the same
  // helper, which stores and re-reads them itself)
  const int bpl = (378 + NG - 1) / NG;
  const int jh = (189 + NG - 1) / NG;  // the blocks of a level holding its old-side items
  unsigned lvmask = 0;
  for (int v = w - 1; v < nblk; v += G - 1) {
    const int b = block_at(v, G - 1, nblk, bpl, jh);
    if (b >= 72) lvmask |= 1u << (4 + (b - 72) / bpl);
  }
  while (true) {
    const unsigned num = cur + 1;
    // wait until move `num` is posted; the stop flag is stored before the
    // number that follows the last move
    if (t == 0) {
      bool ok = spin_until_reached(mvseq, num, SPIN_LIMIT);
      s_flag = ok ? 0 : 1;
      if (ok) {
        // ordered after the number by the fence: the stop flag, the
        // decision word and the move itself, requested together
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const unsigned sp = ld_relaxed(stop);
        const unsigned d = ld_relaxed(dec);
        const auto slot = glb(mb) + 8 * (num & 3);
        double m[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) m[k] = slot[k];
        if (sp) s_flag = 2;
        // a move already decided rejected (its decision, or a later one, is out) is skipped
        s_skip = (d >> 1) > num || ((d >> 1) == num && !(d & 1u));
        mv.idx = (int)m[0];
        mv.q = m[1];
        for (int k = 0; k < 3; ++k) {
          mv.r[k] = m[2 + k];
          mv.rn[k] = m[5 + k];
        }
      }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int f = s_flag;
    const bool skip = s_skip;
    __syncthreads();
    if (f == 1) {
      if (t == 0) st_relaxed(err, 1u);
      return;
    }
    if (f == 2) return;
    cur = num;
    if (skip) continue;
    // the speculation reads target rows: the fine-level rows of the last
    // accepted move, stored by the helpers of those levels, must be in place
    if (confirmed != last_acc && lvmask) {
      if (t < 64) {
        bool ok = spin_level_helpers(doneflag, G, nblk, lvmask, bpl, jh, last_acc, SPIN_LIMIT);
        if (t == 0) s_flag = ok ? 0 : 1;
      }
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const int f2 = s_flag;
      __syncthreads();
      if (f2) {
        if (t == 0) st_relaxed(err, 1u);
        return;
      }
      confirmed = last_acc;
    }
    locate_move_par(ch, mv);
    __syncthreads();
    // speculation: the updated rows of every own block, in LDS
    for (int k = 0, v = w - 1; v < nblk; ++k, v += G - 1) {
      bool coarse =
          accept_block_compute<GS, PM, R>(ch, tb, mv, block_at(v, G - 1, nblk, bpl, jh), sm, spec(k), sdst + (size_t)k * NG);
      if (t == 0) s_coarse[k] = coarse;
      __syncthreads();
    }
    // the decision of this move (a later one means rejected). A move never
    // decided (workgroup 0 stopped on an error) ends the wait at the stop
    // flag: an accepted move is stored by every helper before the stop.
    if (t == 0) {
      uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      int res = 0;  // 0 rejected, 1 accepted, 2 time-out, 3 stopped
      while (true) {
        const unsigned d = ld_relaxed(dec), sp = ld_relaxed(stop);  // one round trip
        if ((d >> 1) == num) {
          res = (int)(d & 1u);
          break;
        }
        if ((d >> 1) > num) break;
        if (sp) {
          res = 3;
          break;
        }
        if (__builtin_amdgcn_s_memrealtime() - t0 > SPIN_LIMIT) {
          res = 2;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      s_flag = res;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int res = s_flag;
    __syncthreads();
    if (res == 2) {
      if (t == 0) st_relaxed(err, 1u);
      return;
    }
    if (res == 3) return;
    if (res == 1) {
      for (int k = 0, v = w - 1; v < nblk; ++k, v += G - 1)
        accept_block_store<GS, NT>(tb, s_coarse[k], spec(k), sdst + (size_t)k * NG);
      // The rows are agent-scope atomic stores, which write through this
      // XCD's L2; once they have completed (the wait below) they are
      // visible to every reader that acquires at agent scope (its L2 is
      // invalidated). An agent-scope release fence would add a write-back
      // of the whole L2 for plain stores, of which this workgroup makes
      // none that another one reads.
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __syncthreads();
      if (t == 0) st_relaxed(&doneflag[w], num);
      last_acc = num;
    }
  }
}

// The whole-GPU chain of the multipole-based variant (Sec. 3.3). Its
// expensive loops are in the proposal (Alg. M.1), so the helpers share the
// proposal instead of the accept: workgroup 0 draws the move, posts it at
// the start of its proposal and forms the near-field, self-image, lattice
// and tin-foil terms; helper w evaluates the far-field items of its groups
// (items (w-1) NG + g, stepping by (G-1) NG), adds them by a fixed tree and
// posts the sum in part[w] with its done flag. Workgroup 0 adds the partial
// sums in helper order, decides, and on accept updates the 2(L-1)
// multipoles and the bookkeeping itself (Alg. M.2), releasing every store
// before it posts the next move, so a helper always reads the multipoles
// of the current state. Protocol words: sync[0] number of the latest move,
// sync[2] stop, sync[3] error, sync[64 + w] done flag of helper w; the move
// is in mailbox slot number & 1, which is rewritten only after every helper
// has finished the move after it. Every wait is bounded.
template <int GS, int PM, typename R>
__global__ void __launch_bounds__(WG_SINGLE) k_run_single(Chain ch_arg, Tabs tb, RunParams rp) {
  run_chain_wg<GS, PM, R, false>(ch_arg, tb, rp);
}

// Many independent chains, one workgroup each: the loop of the whole-GPU
// chain's workgroup 0 without helpers (its proposal, then the whole update
// of an accepted move by the workgroup itself).
template <int GS, int PM, typename R>
__global__ void __launch_bounds__(WG_SINGLE) k_run_chains(const Chain *chains, Tabs tb, RunParams rp) {
  run_chain_wg<GS, PM, R, true>(chains[blockIdx.x], tb, rp);
}

template <int GS, int PM>
__global__ void __launch_bounds__(WG_SINGLE) k_run_single_mp(Chain ch_arg, Tabs tb, RunParams rp) {
  constexpr int NT = WG_SINGLE;
  constexpr int NG = NT / GS;
  extern __shared__ double lds[];
  __shared__ Move mvs[2];  // the move of this step and the next (workgroup 0); helpers use mvs[0]
  __shared__ NextDraw nd;
  __shared__ int s_flag, s_acc, s_ovf;
  __shared__ unsigned s_seq;
  __shared__ double s_u, s_far;
  __shared__ Chain chl;  // the chain's descriptor, indexed by level without scratch
  const int t = threadIdx.x, w = blockIdx.x, G = gridDim.x;
  if (t == 0) chl = ch_arg;
  __syncthreads();
  const Chain &ch = chl;
  unsigned *mvseq = ch.sync, *stop = ch.sync + 2, *err = ch.sync + 3;
  unsigned *doneflag = ch.sync + 64;
  double *mb = ch.mbox;
  Lds<GS, NT> sm(lds, tb.Cs, tb.lat_lds ? tb.lat_w : 0);
  stage_lds(ch, tb, sm, w == 0);
  __syncthreads();
  if (w == 0) {
    const int c = rp.chain_id ? rp.chain_id[0] : 0;
    const double D = run_max_step(rp, c);
    double nprop = 0, nacc = 0, nsing = 0, dEsum = 0;
    int status = 0;
    unsigned num = 0;  // move number of this launch
    uint64_t tick_prop = 0, tick_acc = 0, tick_wait = 0;
    const int64_t s0 = run_first(rp, 0);
    int64_t acc_launch = 0;
    int cur = 0;  // mvs[cur]: the move of this step, located and posted
    // the move of step s0 (no move accepted before it in this launch)
    auto next_move = [&](bool acc, int prev_idx, const double *prev_rn, int slot) {
      if (t == 0) {
        move_from_draw(rp, ch, nd, acc, prev_idx, prev_rn, mvs[slot]);
        s_u = nd.u;
      }
      __syncthreads();
      locate_move_par(ch, mvs[slot]);
      __syncthreads();
      ++num;
      if (t == 0 && G > 1) {
        const auto sl = glb(mb) + 8 * (num & 1);
        const Move &m = mvs[slot];
        sl[0] = (double)m.idx;
        sl[1] = m.q;
        for (int k = 0; k < 3; ++k) {
          sl[2 + k] = m.r[k];
          sl[5 + k] = m.rn[k];
        }
        st_release(mvseq, num);
      }
    };
    if (s0 < rp.steps) {
      if (t == 0) draw_into(rp, c, s0, ch, D, nd);
      __syncthreads();
      const double none[3] = {0, 0, 0};
      next_move(false, -1, none, 0);
    }
    for (int64_t step = s0; step < rp.steps; ++step) {
      uint64_t t_0 = __builtin_amdgcn_s_memrealtime();
      const Move &mv = mvs[cur];
      const double u = s_u;
      // near field, self-image, lattice and tin-foil terms; the last
      // wavefront fetches the next draw meanwhile
      ProposeOut po = propose_wg<GS, PM, double, false>(ch, tb, mv, sm, [&](int lane) {
        if (lane == 0 && step + 1 < rp.steps) draw_into(rp, c, step + 1, ch, D, nd);
      });
      uint64_t t_w = __builtin_amdgcn_s_memrealtime();
      if (G > 1) {
        // the helpers' partial sums, added in helper order
        if (t < 64) {
          const bool ok = spin_all_equal(doneflag, G, num, SPIN_LIMIT);
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          double v = 0.0;
          if (ok)
            for (int hw = 1 + t; hw < G; hw += 64) v += glb(ch.part)[hw];
          {
            double a[1] = {v};
            sum_allreduce<64, 1>(a);
            v = a[0];
          }
          if (t == 0) {
            s_far = v;
            s_flag = ok ? 0 : 1;
          }
        }
        __syncthreads();
      } else {
        // no helpers: the workgroup evaluates every item itself
        double f = m2p_far_part<GS, PM>(ch, tb, sm.rec, sm.il32, mv, 0, NG);
        f = wg_sum<NT>(f, sm.red);
        if (t == 0) {
          s_far = f;
          s_flag = 0;
        }
        __syncthreads();
      }
      if (s_flag) {
        status = -8;
        break;
      }
      const double dE = po.dE + mv.q * s_far;
      uint64_t t_1 = __builtin_amdgcn_s_memrealtime();
      tick_prop += t_w - t_0;
      tick_wait += t_1 - t_w;
      if (t == 0) {
        int acc = !po.singular && mh_accept(u, rp.beta, dE);
        s_ovf = acc && move_overflows(ch, mv, sm.ints);
        if (s_ovf) acc = 0;
        s_acc = acc;
        nprop += 1;
        nsing += po.singular;
        const int64_t o = (int64_t)c * rp.steps + step;
        if (rp.tr_idx) glb(rp.tr_idx)[o] = mv.idx;
        if (rp.tr_pos)
          for (int k = 0; k < 3; ++k) glb(rp.tr_pos)[3 * o + k] = mv.rn[k];
        if (rp.tr_dE) glb(rp.tr_dE)[o] = dE;
        if (rp.tr_acc) glb(rp.tr_acc)[o] = (uint8_t)acc;
        if (rp.tr_leaf) {
          int n = 1 << (ch.L - 1);
          glb(rp.tr_leaf)[o] = lin3(n, mv.c1[ch.L][0], mv.c1[ch.L][1], mv.c1[ch.L][2]);
        }
      }
      __syncthreads();
      const bool acc = s_acc;
      if (s_ovf) {
        status = -7;
        break;
      }
      const bool last = acc && rp.acc_limit && acc_launch + 1 >= rp.acc_limit;
      if (acc) {
        // the multipoles first: the next move may be posted only when every
        // thread's stores are released
        accept_mp_wg<GS, PM, NT>(ch, tb, mv, sm.rec);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      }
      // the next move is posted before this move's bookkeeping, so the
      // helpers evaluate its far field while the bookkeeping runs
      if (step + 1 < rp.steps && !last) next_move(acc, mv.idx, mv.rn, cur ^ 1);
      if (acc) {
        int ovf = accept_bookkeeping<GS, PM>(ch, tb, mv, dE, sm);
        if (t == 0) {
          nacc += 1;
          dEsum += dE;
        }
        tick_acc += __builtin_amdgcn_s_memrealtime() - t_1;
        if (ovf) {
          status = -7;
          break;
        }
        ++acc_launch;
        if (last) break;
      } else {
        tick_prop += __builtin_amdgcn_s_memrealtime() - t_1;  // forming the next move
      }
      cur ^= 1;
      // every step ends at a barrier (see the helper loop)
      __syncthreads();
    }
    if (G > 1 && t == 0) {
      st_release(stop, 1u);
      st_release(mvseq, num + 1);
    }
    __syncthreads();
    writeback_lds(ch, tb, sm);
    if (t == 0) {
      glb(rp.stats)[0] = nprop;
      glb(rp.stats)[1] = nacc;
      glb(rp.stats)[2] = nsing;
      glb(rp.stats)[3] = dEsum;
      glb(rp.stats)[4] = status;
      glb(rp.stats)[5] = tick_prop * 0.01;  // microseconds (100 MHz clock)
      glb(rp.stats)[6] = tick_acc * 0.01;
      glb(rp.stats)[7] = tick_wait * 0.01;
      glb(rp.stats)[8] = sm.st[3];
    }
    return;
  }
  // ---- helper workgroups. The whole of wavefront 0 waits (a condition
  // uniform over each wavefront) and every iteration ends at a barrier, so
  // no per-thread branch at the end of one iteration can be merged by the
  // compiler with the wait of the next.
  Move &mv = mvs[0];
  unsigned cur = 0;
  while (true) {
    if (t < 64) {
      unsigned v;
      const bool ok = wave_spin_until_ne(mvseq, cur, v, SPIN_LIMIT);
      int fl = ok ? 0 : 1;
      if (ok) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the stop flag is stored before the number
        const unsigned sv = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(glb(stop), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
        if (sv) fl = 2;
      }
      if (t == 0) {
        s_seq = v;
        s_flag = fl;
      }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int f = s_flag;
    const unsigned num = s_seq;
    __syncthreads();
    if (f == 1) {
      if (t == 0) st_relaxed(err, 1u);
      return;
    }
    if (f == 2) return;
    cur = num;
    if (t == 0) {
      const auto slot = glb(mb) + 8 * (num & 1);
      double m[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) m[k] = slot[k];
      mv.idx = (int)m[0];
      mv.q = m[1];
      for (int k = 0; k < 3; ++k) {
        mv.r[k] = m[2 + k];
        mv.rn[k] = m[5 + k];
      }
    }
    __syncthreads();
    locate_move_par(ch, mv);
    __syncthreads();
    double fsum = m2p_far_part<GS, PM>(ch, tb, sm.rec, sm.il32, mv, (w - 1) * NG, (G - 1) * NG);
    fsum = wg_sum<NT>(fsum, sm.red);
    if (t == 0) {
      glb(ch.part)[w] = fsum;
      st_release(&doneflag[w], num);
    }
    __syncthreads();
  }
}

// single-call entry points (one proposal / one accept)
__device__ __forceinline__ void move_direct(const Chain &ch, int64_t idx, double x, double y, double z,
                                            Move &mv) {
  if (threadIdx.x == 0) {
    mv.idx = (int)idx;
    mv.q = glb(ch.pq)[idx];
    mv.r[0] = glb(ch.px)[idx];
    mv.r[1] = glb(ch.py)[idx];
    mv.r[2] = glb(ch.pz)[idx];
    mv.rn[0] = ch.free_space ? x : wrap_coord(x, ch.a);
    mv.rn[1] = ch.free_space ? y : wrap_coord(y, ch.a);
    mv.rn[2] = ch.free_space ? z : wrap_coord(z, ch.a);
  }
  __syncthreads();
  locate_move_par(ch, mv);
  __syncthreads();
}

template <int GS, int PM, typename R, bool MP = false>
__global__ void __launch_bounds__(WG_SINGLE) k_propose_one(Chain ch, Tabs tb, int64_t idx, double x, double y,
                                                    double z) {
  constexpr int NT = WG_SINGLE;
  extern __shared__ double lds[];
  __shared__ Move mv;
  Lds<GS, NT> sm(lds, tb.Cs, tb.lat_lds ? tb.lat_w : 0);
  stage_lds(ch, tb, sm, true);
  move_direct(ch, idx, x, y, z, mv);
  ProposeOut po;
  if constexpr (MP)
    po = propose_mp_wg<GS, PM>(ch, tb, mv, sm, [](int) {});
  else
    po = propose_wg<GS, PM, R>(ch, tb, mv, sm, [](int) {});
  if (threadIdx.x == 0) {
    glb(ch.scratch)[0] = po.dE;
    glb(ch.scratch)[1] = po.singular;
  }
}

template <int GS, int PM, typename R>
__global__ void __launch_bounds__(WG_SINGLE) k_accept_blocks(Chain ch, Tabs tb, int64_t idx, double x, double y,
                                                      double z) {
  constexpr int NT = WG_SINGLE;
  extern __shared__ double lds[];
  __shared__ Move mv;
  Lds<GS, NT> sm(lds, tb.Cs, tb.lat_lds ? tb.lat_w : 0);
  stage_lds(ch, tb, sm, false);
  move_direct(ch, idx, x, y, z, mv);
  if (move_overflows_mem(ch, mv)) return;  // uniform over the workgroup
  accept_block<GS, PM, R>(ch, tb, mv, blockIdx.x, sm);
}

// the bookkeeping of one accepted move; in the multipole-based variant
// (MP) also its multipole updates (Alg. M.2)
template <int GS, int PM, bool MP = false>
__global__ void __launch_bounds__(WG_SINGLE) k_accept_book(Chain ch, Tabs tb, int64_t idx, double x, double y,
                                                    double z, double dE) {
  constexpr int NT = WG_SINGLE;
  extern __shared__ double lds[];
  __shared__ Move mv;
  Lds<GS, NT> sm(lds, tb.Cs, tb.lat_lds ? tb.lat_w : 0);
  stage_lds(ch, tb, sm, true);
  move_direct(ch, idx, x, y, z, mv);
  // status word 0 of the single-call accept: FMM_MC_EOVERFLOW, with the
  // state unchanged, when the move would overflow its new leaf bin
  if (move_overflows_mem(ch, mv)) {
    if (threadIdx.x == 0) glb(ch.status)[0] = -7;
    return;
  }
  if constexpr (MP) accept_mp_wg<GS, PM, NT>(ch, tb, mv, sm.rec);
  load_bin_records(ch, mv, sm);
  __syncthreads();
  int ovf = accept_bookkeeping<GS, PM>(ch, tb, mv, dE, sm);
  writeback_lds(ch, tb, sm);
  if (threadIdx.x == 0) glb(ch.status)[0] = ovf ? -7 : 0;
}

}  // namespace fmmdev
