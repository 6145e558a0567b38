// run_kernels.hpp -- Metropolis-Hastings chains on the device.
//
//  * k_run_batched: one workgroup per chain, every chain its own state; the
//    workgroup proposes, decides and, on accept, walks every update block
//    itself. No inter-workgroup communication: hundreds of independent
//    chains of uneven size and depth in one launch (the paper's "several
//    Markov chains in parallel", Sec. 6).
//  * k_run_single: one chain on many workgroups (cooperative launch, all
//    co-resident). Workgroup 0 proposes and decides; on accept it posts the
//    move in a mailbox and the update blocks of Alg. L.2 are shared out over
//    all workgroups, each owning distinct target cells, then workgroup 0
//    waits for their completion before the next proposal. The per-level
//    work is spread as the paper suggests for parallelism (Sec. 6).
//
// A step draws (idx, delta, u) from Philox4x64-10 (key = (seed, chain),
// counter = (t, 0|1, 0, 0)) or reads them from fixed lists; the move is
// accepted iff u < exp(-beta dE) and it is not singular.
#pragma once

#include "mc_step.hpp"

namespace fmmdev {

struct RunParams {
  int64_t steps, t0;
  uint64_t seed;
  double beta;
  const double *max_step;  // per chain
  // fixed-list source (replay) when list_idx != nullptr
  const int64_t *list_idx;
  const double *list_pos;
  const double *list_u;
  // traces, [chain * steps + t], may be null
  int64_t *tr_idx;
  double *tr_pos, *tr_dE;
  uint8_t *tr_acc;
  int32_t *tr_leaf;
  double *stats;           // per chain 8 doubles: proposed, accepted, singular, dE_sum, status
};

__device__ __forceinline__ void draw_step(const RunParams &rp, int c, int64_t t, int64_t N, double D,
                                          int64_t &idx, double rn_abs[3], const Chain &ch,
                                          double &u) {
#pragma clang fp contract(off)
  if (rp.list_idx) {
    idx = rp.list_idx[t];
    for (int k = 0; k < 3; ++k) rn_abs[k] = rp.list_pos[3 * t + k];
    u = rp.list_u[t];
  } else {
    double delta[3];
    mh_draw(rp.seed, (uint64_t)c, (uint64_t)(rp.t0 + t), N, D, idx, delta, u);
    double r[3] = {ch.px[idx], ch.py[idx], ch.pz[idx]};
    for (int k = 0; k < 3; ++k) rn_abs[k] = r[k] + delta[k];
  }
}

__device__ __forceinline__ void fill_move(const Chain &ch, Move &mv, int64_t idx, const double rn_abs[3]) {
  mv.idx = (int)idx;
  mv.q = ch.pq[idx];
  mv.r[0] = ch.px[idx];
  mv.r[1] = ch.py[idx];
  mv.r[2] = ch.pz[idx];
  for (int k = 0; k < 3; ++k) mv.rn[k] = wrap_coord(rn_abs[k], ch.a);
  locate_move(ch, mv);
}

template <int GS>
__global__ void __launch_bounds__(NT) k_run_batched(const Chain *chains, Tabs tb, RunParams rp) {
  constexpr int NG = NT / GS;
  extern __shared__ double lds[];
  __shared__ Move mv;
  __shared__ int s_acc, s_ovf;
  __shared__ double s_dE;
  const int c = blockIdx.x, t = threadIdx.x;
  const Chain ch = chains[c];
  Lds<GS> sm(lds, tb.Cs);
  stage_rec(tb, sm);
  const double D = rp.max_step[c];
  const int nblk = accept_blocks(ch.L, NG);
  double nprop = 0, nacc = 0, nsing = 0, dEsum = 0;
  uint64_t tick_prop = 0, tick_acc = 0;
  int status = 0;
  for (int64_t step = 0; step < rp.steps; ++step) {
    uint64_t t_0 = __builtin_amdgcn_s_memrealtime();
    if (t == 0) {
      int64_t idx;
      double rn_abs[3], u;
      draw_step(rp, c, step, ch.N, D, idx, rn_abs, ch, u);
      fill_move(ch, mv, idx, rn_abs);
      s_dE = u;  // park u
    }
    __syncthreads();
    double u = s_dE;
    ProposeOut po = propose_wg<GS>(ch, tb, mv, sm);
    uint64_t t_1 = __builtin_amdgcn_s_memrealtime();
    tick_prop += t_1 - t_0;
    if (t == 0) {
      int acc = !po.singular && (u < exp(-rp.beta * po.dE));
      s_acc = acc;
      nprop += 1;
      nsing += po.singular;
      int64_t o = (int64_t)c * rp.steps + step;
      if (rp.tr_idx) rp.tr_idx[o] = mv.idx;
      if (rp.tr_pos)
        for (int k = 0; k < 3; ++k) rp.tr_pos[3 * o + k] = mv.rn[k];
      if (rp.tr_dE) rp.tr_dE[o] = po.dE;
      if (rp.tr_acc) rp.tr_acc[o] = (uint8_t)acc;
      if (rp.tr_leaf) {
        int n = 1 << (ch.L - 1);
        rp.tr_leaf[o] = lin3(n, mv.c1[ch.L][0], mv.c1[ch.L][1], mv.c1[ch.L][2]);
      }
    }
    __syncthreads();
    if (s_acc) {
      for (int b = 0; b < nblk; ++b) {
        accept_block<GS>(ch, tb, mv, b, sm);
        __syncthreads();
      }
      int ovf = accept_bookkeeping<GS>(ch, tb, mv, po.dE, sm);
      if (t == 0) {
        nacc += 1;
        dEsum += po.dE;
      }
      tick_acc += __builtin_amdgcn_s_memrealtime() - t_1;
      if (ovf) {
        status = -7;
        break;
      }
    }
  }
  if (t == 0) {
    double *st = rp.stats + 8 * c;
    st[0] = nprop;
    st[1] = nacc;
    st[2] = nsing;
    st[3] = dEsum;
    st[4] = status;
    st[5] = tick_prop * 0.01;  // microseconds (100 MHz clock)
    st[6] = tick_acc * 0.01;
    st[7] = 0.0;
  }
}

// ---------------------------------------------------------------- single chain
// Polling uses relaxed agent-scope loads (no cache invalidation per poll);
// the caller issues one acquire fence after the awaited value is seen.
__device__ __forceinline__ unsigned ld_relaxed(unsigned *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(unsigned *p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// bounded spin: returns false after `limit` ticks of the 100 MHz clock
__device__ __forceinline__ bool spin_until_ne(unsigned *p, unsigned old, unsigned &val, uint64_t limit) {
  uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  while (true) {
    val = ld_relaxed(p);
    if (val != old) return true;
    if (__builtin_amdgcn_s_memrealtime() - t0 > limit) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}
__device__ __forceinline__ bool spin_until_ge(unsigned *p, unsigned target, uint64_t limit) {
  uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  while (true) {
    unsigned v = ld_relaxed(p);
    if ((int)(v - target) >= 0) return true;
    if (__builtin_amdgcn_s_memrealtime() - t0 > limit) return false;
    __builtin_amdgcn_s_sleep(1);
  }
}

constexpr uint64_t SPIN_LIMIT = 100000000ull * 20;  // 20 s of the 100 MHz clock

template <int GS>
__global__ void __launch_bounds__(NT) k_run_single(Chain ch, Tabs tb, RunParams rp) {
  constexpr int NG = NT / GS;
  extern __shared__ double lds[];
  __shared__ Move mv;
  __shared__ int s_flag, s_acc;
  __shared__ double s_u;
  const int t = threadIdx.x, w = blockIdx.x, G = gridDim.x;
  Lds<GS> sm(lds, tb.Cs);
  stage_rec(tb, sm);
  __syncthreads();
  const int nblk = accept_blocks(ch.L, NG);
  unsigned *seq = ch.sync, *done = ch.sync + 1, *stop = ch.sync + 2, *err = ch.sync + 3;
  double *mb = ch.mbox;
  if (w == 0) {
    const double D = rp.max_step[0];
    double nprop = 0, nacc = 0, nsing = 0, dEsum = 0;
    int status = 0;
    unsigned myseq = 0, expect = 0;
    uint64_t tick_prop = 0, tick_acc = 0, tick_wait = 0;
    for (int64_t step = 0; step < rp.steps; ++step) {
      uint64_t t_0 = __builtin_amdgcn_s_memrealtime();
      if (t == 0) {
        int64_t idx;
        double rn_abs[3], u;
        draw_step(rp, 0, step, ch.N, D, idx, rn_abs, ch, u);
        fill_move(ch, mv, idx, rn_abs);
        s_u = u;
      }
      __syncthreads();
      ProposeOut po = propose_wg<GS>(ch, tb, mv, sm);
      uint64_t t_1 = __builtin_amdgcn_s_memrealtime();
      tick_prop += t_1 - t_0;
      if (t == 0) {
        int acc = !po.singular && (s_u < exp(-rp.beta * po.dE));
        s_acc = acc;
        nprop += 1;
        nsing += po.singular;
        if (rp.tr_idx) rp.tr_idx[step] = mv.idx;
        if (rp.tr_pos)
          for (int k = 0; k < 3; ++k) rp.tr_pos[3 * step + k] = mv.rn[k];
        if (rp.tr_dE) rp.tr_dE[step] = po.dE;
        if (rp.tr_acc) rp.tr_acc[step] = (uint8_t)acc;
        if (rp.tr_leaf) {
          int n = 1 << (ch.L - 1);
          rp.tr_leaf[step] = lin3(n, mv.c1[ch.L][0], mv.c1[ch.L][1], mv.c1[ch.L][2]);
        }
        if (acc) {
          mb[0] = (double)mv.idx;
          mb[1] = mv.q;
          for (int k = 0; k < 3; ++k) {
            mb[2 + k] = mv.r[k];
            mb[5 + k] = mv.rn[k];
          }
        }
      }
      __syncthreads();
      if (s_acc) {
        if (G > 1) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __syncthreads();
          if (t == 0) st_release(seq, ++myseq);
        }
        for (int b = 0; b < nblk; b += G) {
          accept_block<GS>(ch, tb, mv, b, sm);
          __syncthreads();
        }
        int ovf = accept_bookkeeping<GS>(ch, tb, mv, po.dE, sm);
        if (t == 0) {
          nacc += 1;
          dEsum += po.dE;
        }
        uint64_t t_2 = __builtin_amdgcn_s_memrealtime();
        tick_acc += t_2 - t_1;
        if (G > 1) {
          expect += (unsigned)(G - 1);
          if (t == 0) s_flag = spin_until_ge(done, expect, SPIN_LIMIT) ? 0 : 1;
          __syncthreads();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          if (s_flag) {
            status = -8;
            break;
          }
        }
        tick_wait += __builtin_amdgcn_s_memrealtime() - t_2;
        if (ovf) {
          status = -7;
          break;
        }
      }
    }
    if (G > 1 && t == 0) {
      st_release(stop, 1u);
      st_release(seq, ++myseq);
    }
    if (t == 0) {
      rp.stats[0] = nprop;
      rp.stats[1] = nacc;
      rp.stats[2] = nsing;
      rp.stats[3] = dEsum;
      rp.stats[4] = status;
      rp.stats[5] = tick_prop * 0.01;  // microseconds (100 MHz clock)
      rp.stats[6] = tick_acc * 0.01;
      rp.stats[7] = tick_wait * 0.01;
    }
    return;
  }
  // helper workgroups: wait for a posted move, do their share of the blocks
  unsigned myseq = 0;
  while (true) {
    if (t == 0) {
      unsigned v;
      bool ok = spin_until_ne(seq, myseq, v, SPIN_LIMIT);
      s_flag = ok ? 0 : 1;
      if (ok) {
        myseq = v;
        if (__hip_atomic_load(stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) s_flag = 2;
      }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    int f = s_flag;
    __syncthreads();
    if (f == 1) {
      if (t == 0) __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    if (f == 2) return;
    if (t == 0) {
      double rn_abs[3];
      mv.idx = (int)mb[0];
      mv.q = mb[1];
      for (int k = 0; k < 3; ++k) {
        mv.r[k] = mb[2 + k];
        mv.rn[k] = mb[5 + k];
        rn_abs[k] = mv.rn[k];
      }
      (void)rn_abs;
      locate_move(ch, mv);
    }
    __syncthreads();
    for (int b = w; b < nblk; b += G) {
      accept_block<GS>(ch, tb, mv, b, sm);
      __syncthreads();
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (t == 0) __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// single-call entry points (one proposal / one accept)
template <int GS>
__global__ void __launch_bounds__(NT) k_propose_one(Chain ch, Tabs tb, int64_t idx, double x, double y,
                                                    double z) {
  extern __shared__ double lds[];
  __shared__ Move mv;
  Lds<GS> sm(lds, tb.Cs);
  stage_rec(tb, sm);
  if (threadIdx.x == 0) {
    double rn_abs[3] = {x, y, z};
    fill_move(ch, mv, idx, rn_abs);
  }
  __syncthreads();
  ProposeOut po = propose_wg<GS>(ch, tb, mv, sm);
  if (threadIdx.x == 0) {
    ch.scratch[0] = po.dE;
    ch.scratch[1] = po.singular;
  }
}

template <int GS>
__global__ void __launch_bounds__(NT) k_accept_blocks(Chain ch, Tabs tb, int64_t idx, double x, double y,
                                                      double z) {
  extern __shared__ double lds[];
  __shared__ Move mv;
  Lds<GS> sm(lds, tb.Cs);
  stage_rec(tb, sm);
  if (threadIdx.x == 0) {
    double rn_abs[3] = {x, y, z};
    fill_move(ch, mv, idx, rn_abs);
  }
  __syncthreads();
  accept_block<GS>(ch, tb, mv, blockIdx.x, sm);
}

template <int GS>
__global__ void __launch_bounds__(NT) k_accept_book(Chain ch, Tabs tb, int64_t idx, double x, double y,
                                                    double z, double dE) {
  extern __shared__ double lds[];
  __shared__ Move mv;
  Lds<GS> sm(lds, tb.Cs);
  stage_rec(tb, sm);
  if (threadIdx.x == 0) {
    double rn_abs[3] = {x, y, z};
    fill_move(ch, mv, idx, rn_abs);
  }
  __syncthreads();
  int ovf = accept_bookkeeping<GS>(ch, tb, mv, dE, sm);
  if (threadIdx.x == 0 && ovf) ch.status[0] = -7;
}

}  // namespace fmmdev
