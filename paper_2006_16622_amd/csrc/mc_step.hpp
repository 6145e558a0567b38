// mc_step.hpp -- the per-step device work of the multilevel Monte Carlo
// method: the proposal energy (Alg. L.1 + Alg. 1 with the periodic
// modifications of Sec. 3.4) evaluated by one workgroup, and the accepted-
// move update (Alg. L.2 with images, Sec. 3.4) split into independent
// blocks, each owning distinct target cells (no atomics, deterministic).
#pragma once

#include "device_common.hpp"

namespace fmmdev {

// A proposed or accepted move, known to every thread of a workgroup (LDS).
struct Move {
  int idx;
  double q;
  double r[3], rn[3];   // old and new (wrapped) positions
  double u;             // uniform of the decision (whole-GPU run)
  int c0[MAXL + 1][3];  // cell of r on each level
  int c1[MAXL + 1][3];  // cell of rn on each level
};

__device__ __forceinline__ int lin3(int n, int x, int y, int z) { return x + n * (y + n * z); }
__device__ __forceinline__ int imod(int i, int n) { return ((i % n) + n) % n; }
__device__ __forceinline__ int ifloordiv(int i, int n) { return (i - imod(i, n)) / n; }
// the same for n a power of two (cells per side of a level): a mask and an
// arithmetic shift instead of integer divisions
__device__ __forceinline__ int pmod(int i, int n) { return i & (n - 1); }
__device__ __forceinline__ int pfloordiv(int i, int n) { return i >> __builtin_ctz((unsigned)n); }

// cells of r and rn on level l (1..L)
__device__ __forceinline__ void locate_move_level(const Chain &ch, Move &mv, int l) {
  if (l <= ch.L) {
    int n = 1 << (l - 1);
    for (int k = 0; k < 3; ++k) {
      mv.c0[l][k] = cell_coord(mv.r[k], ch.inv_h[l], n);
      mv.c1[l][k] = cell_coord(mv.rn[k], ch.inv_h[l], n);
    }
  }
}

// cells of r and rn on every level, one level per thread (caller syncs)
__device__ __forceinline__ void locate_move_par(const Chain &ch, Move &mv) {
  locate_move_level(ch, mv, threadIdx.x + 1);
}

// indices into Lds::ints
enum : int {
  I_NCELL = 0,     // 54 near cells
  I_NSHIFT = 54,   // 54 image shifts
  I_MASK = 108,    // images of the moving charge met in the new near region
  I_SLOTK = 109,   // slot of the moving charge in its leaf bin
  I_CNTOLD = 110,  // occupancy of the old leaf bin
  I_CNTNEW = 111,  // occupancy of the new leaf bin
  I_IDLAST = 112,  // particle in the last slot of the old leaf bin
  I_FLAG = 113,
  I_SING = 114,    // a new-side near-field distance was zero (propose_fast)
  I_LIST = 128     // candidate list of a coarse accept block (55 entries)
};

// Load the constant tables and the chain's small state into LDS (all
// threads; caller syncs).
template <int GS, int NT>
__device__ __forceinline__ void stage_lds(const Chain &ch, const Tabs &tb, Lds<GS, NT> &sm, bool state) {
  const int Cs = tb.Cs;
  for (int i = threadIdx.x; i < 3 * Cs; i += NT) {
    sm.rec[i] = tb.rec[i];
    sm.rec32[i] = (float)tb.rec[i];
  }
  for (int i = threadIdx.x; i < 8 * 189; i += NT) sm.il32[i] = il_pack(tb.il_off + 3 * i);
  for (int i = threadIdx.x; i < Cs; i += NT) {
    sm.wl2p[i] = tb.wl2p[i];
    sm.wdot[i] = tb.wdot[i];
    sm.sgnc[i] = tb.sgnc[i];
    if (state) {
      sm.H[i] = ch.H[i];
      sm.K[i] = ch.K[i];
    }
  }
  if (tb.lat_lds)
    for (int i = threadIdx.x; i < tb.lat_w * Cs; i += NT) {
      sm.lat_val[i] = tb.lat_val[i];
      sm.lat_col[i] = tb.lat_col[i];
    }
  if (threadIdx.x >= NT - 32) fill_p2l_cols(threadIdx.x - (NT - 32), tb, sm.p2lg, sm.p2la);
  if (state && threadIdx.x < 3) sm.st[threadIdx.x] = ch.dip[threadIdx.x];
  if (state && threadIdx.x == 3) sm.st[3] = ch.U[0];
  // the image mask of the first proposal starts empty (each proposal clears
  // it again after its last barrier)
  if (threadIdx.x == 0) {
    sm.ints[I_MASK] = 0;
    sm.ints[I_SING] = 0;
  }
}

// write the chain's small state back to global memory (all threads)
template <int GS, int NT>
__device__ __forceinline__ void writeback_lds(const Chain &ch, const Tabs &tb, Lds<GS, NT> &sm) {
  for (int i = threadIdx.x; i < tb.C; i += NT) {
    ch.H[i] = sm.H[i];
    ch.K[i] = sm.K[i];
  }
  if (threadIdx.x < 3) ch.dip[threadIdx.x] = sm.st[threadIdx.x];
  if (threadIdx.x == 3) ch.U[0] = sm.st[3];
}

// f(values, columns) of the lattice operator's ELL layout: the LDS copy
// when it is resident, else the tables in global memory. The two calls keep
// each access in its own address space (a pointer that may be either would
// make every access a flat one, which the LDS wait counter also waits for).
template <int GS, int NT, typename F>
__device__ __forceinline__ void with_lattice(const Tabs &tb, Lds<GS, NT> &sm, F &&f) {
  if (tb.lat_lds)
    f(sm.lat_val, sm.lat_col);
  else
    f(glb(tb.lat_val), glb(tb.lat_col));
}

struct ProposeOut {
  double dE;
  int singular;
};

// ------------------------------------------------------------------ propose
// Energy change of the move mv, by one whole workgroup:
//   dE = sum_{l=2..L} q [Psi^D_{l,a'_l}(r') - Psi^D_{l,a_l}(r)]        (Alg. L.1)
//      + q [sum_{near(a'_L)} q_j/|r'-r_j-a nu| - sum_{near(a_L)} ...]  (Alg. 1)
//      - sum_{nu in {-1,0,1}^3} q^2/|r'-r-a nu| + (q^2/a)(6+8/sqrt3+12/sqrt2)
//      + q [Psi^inf(r') - Psi^inf(r)] + 1/2 dk.R(dk)                   (far lattice)
//      - (2 pi/3V)(|D + q(r'-r)|^2 - |D|^2)                            (tin-foil)
// The new-side direct sum leaves out every image of the moving charge in
// the near region together with the matching self term (they cancel). The
// bin records the bookkeeping of an accept needs are kept in LDS. `early`
// is run by the last wavefront at the start, `spare` by the last wavefront
// while the others evaluate the expansions. With LOCAL false the first sum
// (the local expansions) is left out: the multipole-based variant adds its
// own far field. When gate.active() holds, the local expansions may still be
// being updated by other workgroups: everything that does not read them (the
// near field, the harmonics of every point, the two lattice values, the
// quadratic lattice term and the partial sums) is formed first, then every
// thread calls gate(), which returns once the expansions are current, and
// only then are they read. The quadratic lattice term leaves dk in sm.dk and
// R(dk) in sm.latO for the bookkeeping of an accept of this move.
struct NoWork {
  __device__ void operator()(int) const {}
};
struct NoGate {
  __device__ bool active() const { return false; }
  __device__ void operator()() const {}
};

template <int GS, int PM, typename R, bool LOCAL = true, int NT, typename Spare, typename Early = NoWork,
          typename Gate = NoGate>
__device__ __forceinline__ ProposeOut propose_wg(const Chain &ch, const Tabs &tb, const Move &mv, Lds<GS, NT> &sm,
                                 Spare &&spare, Early &&early = NoWork{}, Gate &&gate = NoGate{}) {
  constexpr int NG = NT / GS;
  constexpr int NJ = (PM + 1) * (PM + 1) / GS + 1;
  const int Cs = tb.Cs, C = tb.C;
  const int t = threadIdx.x, g = t / GS, lane = t % GS;
  int *ints = sm.ints;
  const double a = ch.a, q = mv.q;
  const int L = ch.L, d = ch.d, B = ch.B;
  const int npts = LOCAL ? 2 * d + 2 : 2;
  const int nL = 1 << (L - 1);
  const bool gated = gate.active();

  if (t >= NT - 64) early(t - (NT - 64));

  // The loads stay in flight across the lattice term in the whole-GPU
  // chain's workgroups; in the wider batched workgroup the registers this
  // holds would spill. There, too, loaded values are not selected or masked
  // where they are loaded (that would make the wavefront wait for them at
  // once): every load reads a valid address, and what is not needed is left
  // out where it is used.
  constexpr bool overlap = NT == WG_SINGLE;

  // ---- the level coefficients of the points are requested first (one
  // point per group), so that their memory latency overlaps the rest
  const bool one_round = npts <= NG;
  double lv0[NJ];
  if (!gated && g >= 2 && g < npts) {
    const int l = 2 + (g - 2) / 2, side = (g - 2) % 2, n = 1 << (l - 1);
    const int *c = side ? mv.c1[l] : mv.c0[l];
    const auto src = glb(ch.Ld) + ch.ld_off[l] + (size_t)lin3(n, c[0], c[1], c[2]) * Cs;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      int s = lane + j * GS;
      if constexpr (overlap)
        lv0[j] = src[min(s, Cs - 1)];  // slots >= C are not used
      else
        lv0[j] = s < C ? src[s] : 0.0;
    }
  }

  // ---- near field: 4 threads per near cell. The count and the first two
  // slots of each thread are requested here (bins of up to 8 charges take
  // one round of loads; the capacity is at least 32 slots) and used later.
  double dold = 0.0, dnew = 0.0;
  int singular = 0;
  const int e = t >> 2, j0 = t & 3;
  const int side = e / 27, ee = e % 27;
  int w = 13, cnt = 0, id = -1, id1 = -1;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  size_t base = 0;
  double4 pj = make_double4(0.0, 0.0, 0.0, 0.0), pj1 = pj;
  if (t < 216) {
    const int *c = side ? mv.c1[L] : mv.c0[L];
    int b[3] = {c[0] + ee % 3 - 1, c[1] + (ee / 3) % 3 - 1, c[2] + ee / 9 - 1};
    const int cell = lin3(nL, pmod(b[0], nL), pmod(b[1], nL), pmod(b[2], nL));
    const int fx = pfloordiv(b[0], nL), fy = pfloordiv(b[1], nL), fz = pfloordiv(b[2], nL);
    w = (fx + 1) + 3 * (fy + 1) + 9 * (fz + 1);
    sx = fx * a;
    sy = fy * a;
    sz = fz * a;
    base = (size_t)cell * B;
    if constexpr (overlap)
      cnt = glb(ch.bin_cnt)[cell];
    else
      cnt = (ch.free_space && w != 13) ? 0 : glb(ch.bin_cnt)[cell];  // free space: no images
    id = glb(ch.bin_id)[base + j0];
    pj = ld_rec(ch.bin_p, base + j0);
    id1 = glb(ch.bin_id)[base + j0 + 4];
    pj1 = ld_rec(ch.bin_p, base + j0 + 4);
  }
  auto near_sum = [&]() __attribute__((always_inline)) {
    if (t >= 216) return;
    if (overlap && ch.free_space && w != 13) cnt = 0;  // free space: no images
    if (ee == 13 && j0 == 0) ints[side ? I_CNTNEW : I_CNTOLD] = cnt;
    const double *x = side ? mv.rn : mv.r;
    for (int j = j0; j < cnt; j += 4) {
      if (j == j0 + 4) {
        id = id1;
        pj = pj1;
      } else if (j != j0) {
        id = glb(ch.bin_id)[base + j];
        pj = ld_rec(ch.bin_p, base + j);
      }
      if (side == 0 && ee == 13) {  // the moving charge's own leaf bin
        if (id == mv.idx) ints[I_SLOTK] = j;
        if (j == cnt - 1) {
          ints[I_IDLAST] = id;
          sm.stash[0] = pj;
        }
      }
      if (id == mv.idx) {
        if (side) atomicOr(&ints[I_MASK], 1 << w);
        if (side || w == 13) continue;  // w == 13: no image shift
      }
      double dx = x[0] - (pj.x + sx), dy = x[1] - (pj.y + sy), dz = x[2] - (pj.z + sz);
      double r2 = dx * dx + dy * dy + dz * dz;
      if (side && r2 == 0.0) singular = 1;
      double v;
      if constexpr (sizeof(R) == 4)
        v = pj.w * (double)rsqrtf((float)r2);  // FP32 inverse distance of an FP64 difference
      else
        v = pj.w / sqrt(r2);
      if (side) dnew += v; else dold += v;
    }
  };

  // ---- one expansion point per group: the local expansion of level
  // l = 2 + (pt - 2) / 2 about the old (even pt) or new (odd pt) cell, or
  // for pt < 2 the lattice expansion about the box centre, scaled by a.
  // geom: the point in cell units, the cell size, the group's harmonics
  // buffer and the coefficients; harm: the harmonics of the point into the
  // buffer; dot: the expansion's value from the coefficients and the buffer.
  auto geom = [&](int pt, double x[3], double &hh, double *&buf, const double *&src) __attribute__((always_inline)) {
    if (pt < 2) {
      buf = pt ? sm.latN : sm.latO;
      const double *r = pt ? mv.rn : mv.r;
      hh = a;
      for (int k = 0; k < 3; ++k) x[k] = (r[k] - 0.5 * a) / a;
      src = sm.H;
    } else {
      int l = 2 + (pt - 2) / 2, side = (pt - 2) % 2;
      buf = sm.gbuf + (size_t)g * Cs;
      int n = 1 << (l - 1);
      hh = a / n;
      const int *c = side ? mv.c1[l] : mv.c0[l];
      const double *r = side ? mv.rn : mv.r;
      for (int k = 0; k < 3; ++k) x[k] = (r[k] - (c[k] + 0.5) * hh) / hh;
      src = ch.Ld + ch.ld_off[l] + (size_t)lin3(n, c[0], c[1], c[2]) * Cs;
    }
  };
  auto load = [&](int pt, const double *src, double lv[NJ]) __attribute__((always_inline)) {
    if (pt < 2) {  // the lattice vector H, in LDS (read from sm.H itself: no flat access)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        int s = lane + j * GS;
        if constexpr (overlap)
          lv[j] = sm.H[min(s, Cs - 1)];
        else
          lv[j] = s < C ? sm.H[s] : 0.0;
      }
    } else {
      const auto gsrc = glb(src);
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        int s = lane + j * GS;
        if constexpr (overlap)
          lv[j] = gsrc[min(s, Cs - 1)];
        else
          lv[j] = s < C ? gsrc[s] : 0.0;
      }
    }
  };
  auto harm = [&](int pt, const double x[3], double *buf) __attribute__((always_inline)) {
    if (pt < 2)  // the periodic lattice term stays in FP64
      group_harmonics<GS, PM, 0, false>(lane, tb, sm.rec, x[0], x[1], x[2], 1.0, buf);
    else
      group_harmonics<GS, PM, 0, false, R>(lane, tb, sm.template rec_of<R>(), (R)x[0], (R)x[1], (R)x[2],
                                           R(1), buf);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  };
  auto dot = [&](int pt, const double lv[NJ], const double *buf, double hh) __attribute__((always_inline)) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      int s = lane + j * GS;
      if (s < C) acc += lv[j] * sm.wl2p[s] * buf[s];
    }
    acc = group_sum<GS>(acc);
    if (lane == 0) sm.vals[pt] = acc / hh;
  };
  // the whole point; the coefficients are loaded while the harmonics are formed
  auto point = [&](int pt, bool preloaded) __attribute__((always_inline)) {
    double x[3], hh, *buf;
    const double *src;
    geom(pt, x, hh, buf, src);
    double lv[NJ];
    if (preloaded) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) lv[j] = lv0[j];
    } else {
      load(pt, src, lv);
    }
    harm(pt, x, buf);
    dot(pt, lv, buf, hh);
  };

  // ---- far lattice quadratic term: dk = q (conj T(r') - conj T(r)), 1/2 dk.R(dk)
  // (this thread's share; needs both lattice points). dk stays in sm.dk and
  // R(dk) replaces sm.latO: an accept of this move adds them to K and H.
  auto lattice_quad = [&]() __attribute__((always_inline)) {
    for (int s = t; s < C; s += NT) sm.dk[s] = q * sm.sgnc[s] * (sm.latN[s] - sm.latO[s]);
    __syncthreads();
    double v = 0.0;
    with_lattice(tb, sm, [&](auto val, auto col) {
      lattice_rows<NT>(tb, val, col, sm.dk, [&](int s, double y) {
        v += sm.wdot[s] * sm.dk[s] * y;
        sm.latO[s] = y;
      });
    });
    return v;
  };
  // self-interaction with the old position's images (Sec. 3.4)
  auto self_term = [&]() __attribute__((always_inline)) {
    double self = 0.0;
    if (t < 27 && !((ints[I_MASK] >> t) & 1) && (!ch.free_space || t == 13)) {
      double sx = (t % 3 - 1) * a, sy = ((t / 3) % 3 - 1) * a, sz = (t / 9 - 1) * a;
      double dx = mv.rn[0] - (mv.r[0] + sx), dy = mv.rn[1] - (mv.r[1] + sy), dz = mv.rn[2] - (mv.r[2] + sz);
      self = q * q / sqrt(dx * dx + dy * dy + dz * dz);
    }
    return self;
  };

  const bool spare_in_loop = npts <= NG - 64 / GS;  // the last wavefront holds no point
  double part[4];
  int sing;
  if (overlap && one_round) {
    // while the near-field and coefficient loads are in flight: the two
    // lattice points and the quadratic lattice term (LDS only)
    double x[3], hh, *buf;
    const double *src;
    if (g < 2) {
      double lv[NJ];
      geom(g, x, hh, buf, src);
      load(g, src, lv);
      harm(g, x, buf);
      dot(g, lv, buf, hh);
    }
    __syncthreads();
    part[3] = lattice_quad();
    near_sum();
    // the harmonics of the level points (and their values, when the
    // coefficients are current); the last wavefront fetches the next draw
    if (g >= 2 && g < npts) {
      geom(g, x, hh, buf, src);
      harm(g, x, buf);
      if (!gated) dot(g, lv0, buf, hh);
    } else if (g >= npts && spare_in_loop && t >= NT - 64) {
      spare(t - (NT - 64));
    }
    __syncthreads();
    if (!spare_in_loop && t >= NT - 64) spare(t - (NT - 64));
    part[0] = dold;
    part[1] = dnew;
    part[2] = self_term();
    wg_sum4<NT>(part, sm.red);
    sing = __syncthreads_or(singular);
    if (gated) {
      // the local expansions are read only after the gate
      gate();
      if (g >= 2 && g < npts) {
        double lv[NJ];
        load(g, src, lv);
        dot(g, lv, buf, hh);
      }
      __syncthreads();
    }
  } else {
    // the direct sum, then the points round by round (no overlap)
    near_sum();
    if (gated) gate();
    for (int base = 0; base < npts; base += NG) {
      int pt = base + g;
      if (pt < npts)
        point(pt, !gated && base == 0 && pt >= 2);
      else if (base == 0 && spare_in_loop && t >= NT - 64)
        spare(t - (NT - 64));
      __syncthreads();
    }
    if (!spare_in_loop && t >= NT - 64) spare(t - (NT - 64));
    part[0] = dold;
    part[1] = dnew;
    part[3] = lattice_quad();
    part[2] = self_term();
    wg_sum4<NT>(part, sm.red);
    sing = __syncthreads_or(singular);
  }

  ProposeOut out;
  double dE = 0.0;
  for (int l = 2; l <= L && LOCAL; ++l) {
    int po = 2 + 2 * (l - 2);
    dE += q * (sm.vals[po + 1] - sm.vals[po]);
  }
  dE += q * (part[1] - part[0]);
  dE += -part[2];
  if (!ch.free_space) {
    // periodic images of the moving charge, far lattice, tin-foil (Sec. 3.4)
    dE += q * q / a * tb.self_const;
    dE += q * (sm.vals[1] - sm.vals[0]) + 0.5 * part[3] / a;
    double dr[3] = {mv.rn[0] - mv.r[0], mv.rn[1] - mv.r[1], mv.rn[2] - mv.r[2]};
    double Ddot = sm.st[0] * dr[0] + sm.st[1] * dr[1] + sm.st[2] * dr[2];
    double dd = dr[0] * dr[0] + dr[1] * dr[1] + dr[2] * dr[2];
    dE += -2.0 * M_PI / (3.0 * a * a * a) * (2.0 * q * Ddot + q * q * dd);
  } else if (!(mv.rn[0] >= 0.0 && mv.rn[0] < a && mv.rn[1] >= 0.0 && mv.rn[1] < a && mv.rn[2] >= 0.0 &&
               mv.rn[2] < a)) {
    dE = INFINITY;  // free space: a move out of the box is never taken
  }
  out.dE = dE;
  out.singular = sing;
  __syncthreads();
  // every read of the image mask is behind the barrier above and every
  // write of the next proposal behind at least one more: clearing it here
  // needs no barrier of its own
  if (t == 0) ints[I_MASK] = 0;
  return out;
}

// One group of GS lanes: the table of T_n^m(x) (KIND 0) into the real-layout
// buffer, through harmonics_core: each lane requests all the recurrence
// constants of its column before the arithmetic starts and runs its rows to
// the uniform bound, so the evaluation waits once for LDS instead of once
// per row. The values are those of group_harmonics<GS, PM, 0, false>.
// Stores are not branched on: a row beyond p is written to a slot of the
// lane's own in `spare` (16 doubles per group lane, never read), and the
// imaginary part is written before the real one, so that for m = 0 the
// real part is the one that stays in the shared slot.
template <int GS, int PM, typename R>
__device__ __forceinline__ void group_harmonics_store(int lane, const Tabs &tb, const R *__restrict__ rec, R x, R y,
                                                      R z, double *buf, double *spare) {
  const int m = lane;
  harmonics_core<GS, PM, 0, R, true>(lane, tb, rec, x, y, z, R(1),
                                     [&](int, int n, double re, double im, bool valid) {
                                       double *pi = valid ? buf + (n * n + n - m) : spare + (lane & 15);
                                       double *pr = valid ? buf + (n * n + n + m) : spare + 16 + (lane & 15);
                                       *pi = im;
                                       *pr = re;
                                     });
}

// The proposal of the whole-GPU chain's proposing workgroup (256 threads,
// groups of 16 lanes, 2d + 2 <= 16 points): the terms of propose_wg, in
// fewer phases.
// Level point pt (2..2d+1) is held by group pt - 2; the two lattice points
// by the two groups after them when those lie in the first three
// wavefronts (d <= 5), else by groups 14 and 15. The last wavefront also
// runs early() and forms the self-image terms.
//   1. the coefficient rows of the level points and the first near-field
//      records are requested;
//   2. the harmonics of every point at once (red[64..95] takes the rows
//      beyond p); early(); the self-image terms, whose images are known
//      from the cells alone: image nu of the old position is in the new near
//      region exactly when the old leaf cell shifted by nu cells lies within
//      one cell of the new leaf cell (the near field skips the same images);
//   3. (barrier) dk is formed, and the terms of the two lattice values H.T,
//      one slot per thread;
//   4. (barrier) the rows of R dk (unrolled to the ELL width) with the
//      quadratic lattice term, the near field, the level values from the
//      requested rows, and spare() in the last wavefront;
//   5. (barrier) after an accepted move the level rows are read only after
//      gate() and their values formed then (one more barrier);
//   6. lane 0 of the last wavefront adds the wavefront sums in order,
//      assembles dE and calls decide(dE, singular); a last barrier makes
//      the decision visible.
// The sums are butterflies inside each wavefront, then the wavefront
// totals in order, as in propose_wg; the lattice values are summed the same
// way here (group sums there), so dE agrees with propose_wg to rounding.
template <int GS, int PM, typename R, int NT, typename Early, typename Spare, typename Gate, typename Decide>
__device__ __forceinline__ void propose_fast(const Chain &ch, const Tabs &tb, const Move &mv, Lds<GS, NT> &sm,
                                             Early &&early, Spare &&spare, Gate &&gate, Decide &&decide) {
  constexpr int NG = NT / GS;
  constexpr int NJ = (PM + 1) * (PM + 1) / GS + 1;
  static_assert(NT == WG_SINGLE && GS == 16, "the whole-GPU proposal shape");
  const int Cs = tb.Cs, C = tb.C;
  const int t = threadIdx.x, g = t / GS, lane = t % GS, wv = t >> 6, wl = t & 63;
  int *ints = sm.ints;
  const double a = ch.a, q = mv.q;
  const int L = ch.L, d = ch.d, B = ch.B;
  const int npts = 2 * d + 2;
  const int nL = 1 << (L - 1);
  const bool gated = gate.active();
  const int lat0 = npts <= 12 ? npts - 2 : NG - 2;  // group of lattice point 0
  // the point of this group: level points first, then the lattice points
  const int pt = g < npts - 2 ? g + 2 : (g == lat0 ? 0 : (g == lat0 + 1 ? 1 : -1));
  const bool last_free = npts <= 12;  // the last wavefront holds no point

  // ---- 1. requests
  double lv0[NJ];
  if (!gated && pt >= 2) {
    const int l = 2 + (pt - 2) / 2, sd = (pt - 2) % 2, n = 1 << (l - 1);
    const int *c = sd ? mv.c1[l] : mv.c0[l];
    const auto src = glb(ch.Ld) + ch.ld_off[l] + (size_t)lin3(n, c[0], c[1], c[2]) * Cs;
#pragma unroll
    for (int j = 0; j < NJ; ++j) lv0[j] = src[min(lane + j * GS, Cs - 1)];  // slots >= C are not used
  }
  double dold = 0.0, dnew = 0.0;
  const int e = t >> 2, j0 = t & 3;
  const int side = e / 27, ee = e % 27;
  int w = 13, cnt = 0, id = -1, id1 = -1;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  size_t base = 0;
  double4 pj = make_double4(0.0, 0.0, 0.0, 0.0), pj1 = pj;
  if (t < 216) {
    const int *c = side ? mv.c1[L] : mv.c0[L];
    int b[3] = {c[0] + ee % 3 - 1, c[1] + (ee / 3) % 3 - 1, c[2] + ee / 9 - 1};
    const int cell = lin3(nL, pmod(b[0], nL), pmod(b[1], nL), pmod(b[2], nL));
    const int fx = pfloordiv(b[0], nL), fy = pfloordiv(b[1], nL), fz = pfloordiv(b[2], nL);
    w = (fx + 1) + 3 * (fy + 1) + 9 * (fz + 1);
    sx = fx * a;
    sy = fy * a;
    sz = fz * a;
    base = (size_t)cell * B;
    cnt = glb(ch.bin_cnt)[cell];
    id = glb(ch.bin_id)[base + j0];
    pj = ld_rec(ch.bin_p, base + j0);
    id1 = glb(ch.bin_id)[base + j0 + 4];
    pj1 = ld_rec(ch.bin_p, base + j0 + 4);
  }

  // ---- 2. the harmonics of every point; early(); the self-image terms
  double ihh = 1.0, *buf = nullptr;  // ihh: 1 / (side of the point's cell)
  const double *src = nullptr;
  if (pt >= 0) {
    double x[3];
    if (pt < 2) {
      buf = pt ? sm.latN : sm.latO;
      const double *r = pt ? mv.rn : mv.r;
      ihh = 1.0 / a;
      for (int k = 0; k < 3; ++k) x[k] = (r[k] - 0.5 * a) * ihh;
    } else {
      const int l = 2 + (pt - 2) / 2, sd = (pt - 2) % 2, n = 1 << (l - 1);
      buf = sm.gbuf + (size_t)g * Cs;
      const double hh = a / n;
      ihh = n / a;
      const int *c = sd ? mv.c1[l] : mv.c0[l];
      const double *r = sd ? mv.rn : mv.r;
      for (int k = 0; k < 3; ++k) x[k] = (r[k] - (c[k] + 0.5) * hh) * ihh;
      src = ch.Ld + ch.ld_off[l] + (size_t)lin3(n, c[0], c[1], c[2]) * Cs;
    }
    if (pt < 2 || sizeof(R) == 8)  // the lattice term is FP64 in every mode
      group_harmonics_store<GS, PM, double>(lane, tb, sm.rec, x[0], x[1], x[2], buf, sm.red + 64);
    else
      group_harmonics_store<GS, PM, R>(lane, tb, sm.template rec_of<R>(), (R)x[0], (R)x[1], (R)x[2], buf,
                                       sm.red + 64);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
  auto dot = [&](const double lv[NJ]) __attribute__((always_inline)) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {  // loads at a valid slot, the term selected: no branch
      const int s2 = lane + j * GS, sc = s2 < C ? s2 : C - 1;
      const double term = lv[j] * sm.wl2p[sc] * buf[sc];
      acc += s2 < C ? term : 0.0;
    }
    acc = group_sum<GS>(acc);
    if (lane == 0) sm.vals[pt] = acc * ihh;
  };
  double self = 0.0;  // the last wavefront: sum of the self-image terms
  if (wv == NT / 64 - 1) {
    early(wl);
    const int k = wl - 32;  // image k of the old position, lanes 32..58
    if (k >= 0 && k < 27 && (!ch.free_space || k == 13)) {
      const int f[3] = {k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1};
      bool near = true;
      for (int c = 0; c < 3; ++c) {
        const int b = mv.c0[L][c] + f[c] * nL;
        near = near && b >= mv.c1[L][c] - 1 && b <= mv.c1[L][c] + 1;
      }
      if (!near) {
        const double dx = mv.rn[0] - (mv.r[0] + f[0] * a), dy = mv.rn[1] - (mv.r[1] + f[1] * a),
                     dz = mv.rn[2] - (mv.r[2] + f[2] * a);
        self = q * q / sqrt(dx * dx + dy * dy + dz * dz);
      }
    }
    {
      double a[1] = {self};
      sum_allreduce<64, 1>(a);
      self = a[0];
    }
  }
  __syncthreads();

  // ---- 3. dk = q (conj T(r') - conj T(r)); the two lattice values H . T,
  // one slot per thread, summed with the wavefront sums below
  double lato = 0.0, latn = 0.0;
  for (int s2 = t; s2 < C; s2 += NT) {
    sm.dk[s2] = q * sm.sgnc[s2] * (sm.latN[s2] - sm.latO[s2]);
    lato += sm.H[s2] * sm.wl2p[s2] * sm.latO[s2];
    latn += sm.H[s2] * sm.wl2p[s2] * sm.latN[s2];
  }
  __syncthreads();

  // ---- 4. R dk, near field, level values, spare
  double latq = 0.0;
  with_lattice(tb, sm, [&](auto val, auto col) {
    lattice_rows_w<NT, ell_width(PM)>(tb, val, col, sm.dk, [&](int s2, double y) {
      latq += sm.wdot[s2] * sm.dk[s2] * y;
      sm.latO[s2] = y;  // R(dk), for the bookkeeping of an accept of this move
    });
  });
  int singular = 0;
  if (t < 216) {
    if (ch.free_space && w != 13) cnt = 0;  // free space: no images
    if (ee == 13 && j0 == 0) ints[side ? I_CNTNEW : I_CNTOLD] = cnt;
    const double *xp = side ? mv.rn : mv.r;
    for (int j = j0; j < cnt; j += 4) {
      if (j == j0 + 4) {
        id = id1;
        pj = pj1;
      } else if (j != j0) {
        id = glb(ch.bin_id)[base + j];
        pj = ld_rec(ch.bin_p, base + j);
      }
      if (side == 0 && ee == 13) {  // the moving charge's own leaf bin
        if (id == mv.idx) ints[I_SLOTK] = j;
        if (j == cnt - 1) {
          ints[I_IDLAST] = id;
          sm.stash[0] = pj;
        }
      }
      // the moving charge itself: on the new side each of its images here
      // goes with its self-image term (both left out), on the old side the
      // charge without shift is not its own partner
      if (id == mv.idx && (side || w == 13)) continue;
      double dx = xp[0] - (pj.x + sx), dy = xp[1] - (pj.y + sy), dz = xp[2] - (pj.z + sz);
      double r2 = dx * dx + dy * dy + dz * dz;
      if (side && r2 == 0.0) singular = 1;
      double v;
      if constexpr (sizeof(R) == 4)
        v = pj.w * (double)rsqrtf((float)r2);  // FP32 inverse distance of an FP64 difference
      else  // 1/r by the refined estimate; r = 0 gives the infinity a division would
        v = pj.w * (r2 > 0.0 ? rsqrt_nr(r2) : INFINITY);
      if (side) dnew += v; else dold += v;
    }
  }
  if (singular) ints[I_SING] = 1;
  if (!gated && pt >= 2) dot(lv0);
  if (last_free && wv == NT / 64 - 1) spare(wl);
  // wavefront partial sums (the butterflies of wg_sum4)
  {
    double a[5] = {dold, dnew, latq, lato, latn};
    sum_allreduce<64, 5>(a);
    dold = a[0];
    dnew = a[1];
    latq = a[2];
    lato = a[3];
    latn = a[4];
  }
  if (wl == 0) {
    sm.red[4 * wv + 0] = dold;
    sm.red[4 * wv + 1] = dnew;
    sm.red[4 * wv + 3] = latq;
    sm.red[16 + 2 * wv] = lato;
    sm.red[17 + 2 * wv] = latn;
  }
  __syncthreads();
  if (!last_free && wv == NT / 64 - 1) spare(wl);

  // ---- 5. after an accepted move: the level values once its rows are in place
  if (gated) {
    gate();
    if (pt >= 2) {
      double lv[NJ];
      const auto gsrc = glb(src);
#pragma unroll
      for (int j = 0; j < NJ; ++j) lv[j] = gsrc[min(lane + j * GS, Cs - 1)];
      dot(lv);
    }
    __syncthreads();
  }

  // ---- 6. assembly and decision (lane 0 of the last wavefront)
  if (t == NT - 64) {
    double part[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double sum = 0.0;
      for (int w2 = 0; w2 < NT / 64; ++w2) sum += k == 2 ? (w2 == NT / 64 - 1 ? self : 0.0) : sm.red[4 * w2 + k];
      part[k] = sum;
    }
    double dE = 0.0;
    for (int l = 2; l <= L; ++l) {
      const int po = 2 + 2 * (l - 2);
      dE += q * (sm.vals[po + 1] - sm.vals[po]);
    }
    dE += q * (part[1] - part[0]);
    dE += -part[2];
    if (!ch.free_space) {
      const double ia = 1.0 / a;  // one division; the terms below multiply by it
      dE += q * q * ia * tb.self_const;
      double vo = 0.0, vn = 0.0;
      for (int w2 = 0; w2 < NT / 64; ++w2) {
        vo += sm.red[16 + 2 * w2];
        vn += sm.red[17 + 2 * w2];
      }
      dE += q * (vn * ia - vo * ia) + 0.5 * part[3] * ia;
      const double dr[3] = {mv.rn[0] - mv.r[0], mv.rn[1] - mv.r[1], mv.rn[2] - mv.r[2]};
      const double Ddot = sm.st[0] * dr[0] + sm.st[1] * dr[1] + sm.st[2] * dr[2];
      const double dd = dr[0] * dr[0] + dr[1] * dr[1] + dr[2] * dr[2];
      dE += -(2.0 * M_PI / 3.0) * (ia * ia * ia) * (2.0 * q * Ddot + q * q * dd);
    } else if (!(mv.rn[0] >= 0.0 && mv.rn[0] < a && mv.rn[1] >= 0.0 && mv.rn[1] < a && mv.rn[2] >= 0.0 &&
                 mv.rn[2] < a)) {
      dE = INFINITY;  // free space: a move out of the box is never taken
    }
    decide(dE, ints[I_SING]);
    ints[I_SING] = 0;
  }
  __syncthreads();
}

// An accepted move of a charge into another leaf cell whose bin is full
// would overflow the bin (fixed-capacity cell arrays, Sec. 4.1). The run
// kernels test it at the decision, from the occupancy the proposal read, and
// stop with FMM_MC_EOVERFLOW before any state changes; the single-call
// accept tests it from memory.
__device__ __forceinline__ bool move_overflows(const Chain &ch, const Move &mv, const int *ints) {
  const int L = ch.L;
  const bool same = mv.c0[L][0] == mv.c1[L][0] && mv.c0[L][1] == mv.c1[L][1] && mv.c0[L][2] == mv.c1[L][2];
  return !same && ints[I_CNTNEW] >= ch.B;
}
__device__ __forceinline__ bool move_overflows_mem(const Chain &ch, const Move &mv) {
  const int L = ch.L, n = 1 << (L - 1);
  const int oldc = lin3(n, mv.c0[L][0], mv.c0[L][1], mv.c0[L][2]);
  const int newc = lin3(n, mv.c1[L][0], mv.c1[L][1], mv.c1[L][2]);
  return oldc != newc && glb(ch.bin_cnt)[newc] >= ch.B;
}

// ------------------------------------------------------------------ accept
// Work of one accepted move, split into blocks that own distinct target
// cells. Level 2 (2 cells per side) and level 3 (4 per side): one block per
// stored cell, summing every image of it in IL(a_l) (charge -q at r) and in
// IL(a'_l) (+q at r'). Levels 4..L (>= 8 cells per side, so an interaction
// list never holds two images of one cell): blocks of NG items, one item per
// offset of IL(a_l) and IL(a'_l); a stored cell lying in both lists is
// handled by the old-side item.
__host__ __device__ inline int accept_blocks(int L, int NG) {
  int nb = 0;
  if (L >= 2) nb += 8;
  if (L >= 3) nb += 64;
  if (L >= 4) nb += (L - 3) * ((378 + NG - 1) / NG);
  return nb;
}

// is some image of stored cell s (on a level of n >= 8 cells per side) in the
// interaction list of cell c? returns the image in b. In free space only the
// cell itself counts.
__device__ __forceinline__ bool image_in_il(const int s[3], const int c[3], int n, int b[3], bool free_space) {
  int mx = 0;
  for (int k = 0; k < 3; ++k) {
    int lo = 2 * (c[k] >> 1) - 2;
    int v = lo + pmod(s[k] - lo, n);
    if (v >= lo + 6 || (free_space && v != s[k])) return false;
    b[k] = v;
    int dd = v - c[k];
    dd = dd < 0 ? -dd : dd;
    mx = dd > mx ? dd : mx;
  }
  return mx >= 2;
}

// One fine-level item (level l >= 4, index in 0..377 over the two
// interaction lists): the stored target cell it owns and the one or two
// point contributions (scaled displacement and charge) it adds there.
struct FineItem {
  int active;  // 0: the target is owned by the other list's item
  int two;     // the old-side target also lies in the new list
  double *dst;
  double v0[3], v1[3];
  double q0, q1;
};

// the quantities of fine level l that every item of a move shares, read
// once per level instead of once per item
struct FineLevel {
  int n;
  double inv_h;
  int c0[3], c1[3];  // cells of r and r'
  int oc0, oc1;      // their octants
  double *rows;      // the level's local expansions
};

__device__ __forceinline__ FineLevel fine_level(const Chain &ch, const Move &mv, int l) {
  FineLevel fl;
  fl.n = 1 << (l - 1);
  fl.inv_h = ch.inv_h[l];
  for (int k = 0; k < 3; ++k) {
    fl.c0[k] = mv.c0[l][k];
    fl.c1[k] = mv.c1[l][k];
  }
  fl.oc0 = (fl.c0[0] & 1) | ((fl.c0[1] & 1) << 1) | ((fl.c0[2] & 1) << 2);
  fl.oc1 = (fl.c1[0] & 1) | ((fl.c1[1] & 1) << 1) | ((fl.c1[2] & 1) << 2);
  fl.rows = ch.Ld + ch.ld_off[l];
  return fl;
}

__device__ __forceinline__ FineItem fine_item(const Chain &ch, const Tabs &tb, const int *il32, const Move &mv,
                                              const FineLevel &fl, int item) {
  FineItem it;
  it.active = 0;
  it.two = 0;
  // without a second point: a zero charge at unit distance (zero terms)
  it.v1[0] = 1.0;
  it.v1[1] = it.v1[2] = 0.0;
  it.q1 = 0.0;
  const int n = fl.n;
  const int side = item >= 189, k189 = side ? item - 189 : item;
  int c[3], co[3], o[3];
  for (int k = 0; k < 3; ++k) {
    c[k] = side ? fl.c1[k] : fl.c0[k];
    co[k] = side ? fl.c0[k] : fl.c1[k];
  }
  il_unpack(il32[(side ? fl.oc1 : fl.oc0) * 189 + k189], o);
  int b[3] = {c[0] + o[0], c[1] + o[1], c[2] + o[2]};
  int s[3] = {pmod(b[0], n), pmod(b[1], n), pmod(b[2], n)};
  if (ch.free_space && (b[0] != s[0] || b[1] != s[1] || b[2] != s[2])) return it;  // outside the box
  int b_other[3];
  const bool other = image_in_il(s, co, n, b_other, ch.free_space);
  if (side == 1 && other) return it;  // owned by the old-side item
  it.active = 1;
  it.dst = fl.rows + (size_t)lin3(n, s[0], s[1], s[2]) * tb.Cs;
  const double *x = side ? mv.rn : mv.r;
  for (int k = 0; k < 3; ++k) it.v0[k] = fma(x[k], fl.inv_h, -(b[k] + 0.5));
  it.q0 = side ? mv.q : -mv.q;
  if (side == 0 && other) {
    it.two = 1;
    for (int k = 0; k < 3; ++k) it.v1[k] = fma(mv.rn[k], fl.inv_h, -(b_other[k] + 0.5));
    it.q1 = mv.q;
  }
  return it;
}

// Contributions of the move to stored cell s of a coarse level (n = 2 or 4
// cells per side): bit (27 side + image) of the result is set when image
// s + n w, w in {-1,0,1}^3, lies in the interaction list of the old (side 0)
// or new (side 1) cell. Computed by the GS lanes of a group.
template <int GS>
__device__ __forceinline__ uint64_t coarse_mask(const Move &mv, int l, const int s[3], int lane, bool free_space) {
  const int n = 1 << (l - 1);
  uint64_t m = 0;
  for (int cand = lane; cand < 54; cand += GS) {
    const int side = cand / 27, e = cand % 27;
    if (free_space && e != 13) continue;  // images only under periodicity
    const int *c = side ? mv.c1[l] : mv.c0[l];
    const int w[3] = {e % 3 - 1, (e / 3) % 3 - 1, e / 9 - 1};
    int mx = 0;
    bool valid = true;
    for (int k = 0; k < 3; ++k) {
      const int bb = s[k] + n * w[k];
      const int lo = 2 * (c[k] >> 1) - 2;
      if (bb < lo || bb >= lo + 6) valid = false;
      int dd = bb - c[k];
      dd = dd < 0 ? -dd : dd;
      mx = dd > mx ? dd : mx;
    }
    if (valid && mx >= 2) m |= 1ull << cand;
  }
  const unsigned lo = or_steps<GS, GS / 2>((unsigned)m), hi = or_steps<GS, GS / 2>((unsigned)(m >> 32));
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// The updated target rows of accept block blk of move mv, formed in LDS
// without writing the targets: out (NG x Cs doubles) receives the old
// values read now plus the block's additions, and dst[g] the row that
// group g's result replaces (null: none). A coarse block (level 2 or 3)
// sums its groups' partial contributions in out itself and forms one row,
// in out[0..C), for dst[0]. The arithmetic and its order are those of an
// immediate update. Returns whether the block is coarse.
template <int GS, int PM, typename R, int NT>
__device__ __forceinline__ bool accept_block_compute(const Chain &ch, const Tabs &tb, const Move &mv, int blk, Lds<GS, NT> &sm,
                                     double *out, double **dst) {
  constexpr int NG = NT / GS;
  constexpr int NJ = (PM + 1) * (PM + 1) / GS + 1;
  const int Cs = tb.Cs, C = tb.C;
  const int t = threadIdx.x, g = t / GS, lane = t % GS;
  double *acc = out;  // NG * Cs partial sums of a coarse block
  int *lst = sm.ints + I_LIST;
  const double a = ch.a, q = mv.q;
  const int L = ch.L;

  int coarse_l = 0, s_lin = 0;
  if (blk < 8) {
    coarse_l = 2;
    s_lin = blk;
  } else if (blk < 72 && L >= 3) {
    coarse_l = 3;
    s_lin = blk - 8;
  }
  if (coarse_l) {
    // ---- one stored cell of level 2 or 3: all its images in both lists
    const int l = coarse_l, n = 1 << (l - 1);
    int s[3] = {s_lin % n, (s_lin / n) % n, s_lin / (n * n)};
    double *row = ch.Ld + ch.ld_off[l] + (size_t)s_lin * Cs;
    double old = glb(row)[min(t, Cs - 1)];  // used for t < C (C <= NT for the 16-lane groups)
    if (t < NG) dst[t] = t == 0 ? row : nullptr;
    if (t < 64) {
      bool valid = false;
      int side = t / 27, e = t % 27;
      if (t < 54 && (!ch.free_space || e == 13)) {
        const int *c = side ? mv.c1[l] : mv.c0[l];
        int w[3] = {e % 3 - 1, (e / 3) % 3 - 1, e / 9 - 1};
        int mx = 0;
        valid = true;
        for (int k = 0; k < 3; ++k) {
          int b = s[k] + n * w[k];
          int lo = 2 * (c[k] >> 1) - 2;
          if (b < lo || b >= lo + 6) valid = false;
          int dd = b - c[k];
          dd = dd < 0 ? -dd : dd;
          mx = dd > mx ? dd : mx;
        }
        if (mx < 2) valid = false;
      }
      uint64_t bal = __ballot(valid);
      if (valid) {
        int pos = __popcll(bal & ((1ULL << t) - 1ULL));
        lst[1 + pos] = t;
      }
      if (t == 0) lst[0] = __popcll(bal);
    }
    __syncthreads();
    // each group sums its candidates in registers (P2L by columns, two at a
    // time) and writes its column sums once
    const int nv = lst[0];
    P2LCols<PM, R> cols;
    load_p2l_cols<PM, R>(lane, tb, sm.p2lg, cols);
    auto cand_pt = [&](int cand, R v[3], R &c) __attribute__((always_inline)) {
      const int side = cand / 27, e = cand % 27;
      const int w[3] = {e % 3 - 1, (e / 3) % 3 - 1, e / 9 - 1};
      const double *x = side ? mv.rn : mv.r;
      for (int k = 0; k < 3; ++k) v[k] = (R)fma(x[k], ch.inv_h[l], -((s[k] + n * w[k]) + 0.5));
      c = (R)(side ? q : -q);
    };
    ColSum<PM> cs;
    cs.zero();
    int i = g;
    for (; i + NG < nv; i += 4 * NG) {  // up to four at a time; a missing point is a zero charge
      R v[4][3], c[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (i + k * NG < nv) {
          cand_pt(lst[1 + i + k * NG], v[k], c[k]);
        } else {
          v[k][0] = R(1);
          v[k][1] = v[k][2] = c[k] = R(0);
        }
      }
      p2l_sum<GS, PM, R, 4>(lane, cols, v, c, cs);
    }
    if (i < nv) {
      R v[1][3], c[1];
      cand_pt(lst[1 + i], v[0], c[0]);
      p2l_sum<GS, PM, R, 1>(lane, cols, v, c, cs);
    }
    flush_p2l<PM>(lane, tb, sm.p2la, cs, acc + (size_t)g * Cs, sm.red + 64);
    __syncthreads();
    for (int k = t; k < C; k += NT) {
      double sum = 0.0;
      for (int gg = 0; gg < NG; ++gg) sum += acc[(size_t)gg * Cs + k];
      out[k] = (k == t ? old : glb(row)[k]) + sum;
    }
    return true;
  }
  // ---- fine levels: item = (level, side, IL offset)
  int b2 = blk - 72;
  const int bpl = (378 + NG - 1) / NG;
  const int l = 4 + b2 / bpl;
  const int item = (b2 % bpl) * NG + g;
  FineItem it;
  it.active = 0;
  if (l <= L && item < 378) it = fine_item(ch, tb, sm.il32, mv, fine_level(ch, mv, l), item);
  if (lane == 0) dst[g] = it.active ? it.dst : nullptr;
  if (!it.active) return false;
  double *buf = out + (size_t)g * Cs;
  // the target's coefficients are loaded while the harmonics are formed
  double old[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    int k = lane + j * GS;
    old[j] = glb(it.dst)[min(k, Cs - 1)];
  }
  // the one or two contributions are summed in registers, then written once
  P2LCols<PM, R> cols;
  load_p2l_cols<PM, R>(lane, tb, sm.p2lg, cols);
  ColSum<PM> cs;
  cs.zero();
  {
    // one pass for one or two points (a missing second point has zero
    // charge), so that the lane groups of a wavefront do not branch apart
    const R v[2][3] = {{(R)it.v0[0], (R)it.v0[1], (R)it.v0[2]}, {(R)it.v1[0], (R)it.v1[1], (R)it.v1[2]}};
    const R c[2] = {(R)it.q0, (R)it.q1};
    p2l_sum<GS, PM, R, 2>(lane, cols, v, c, cs);
  }
  flush_p2l<PM>(lane, tb, sm.p2la, cs, buf, sm.red + 64);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    int k = lane + j * GS;
    if (k < C) buf[k] = old[j] + buf[k];
  }
  return false;
}

// write the rows formed by accept_block_compute (all threads; the caller
// synchronises the workgroup between the two). The stores are device-coherent
// (agent scope): they are written through the XCD's L2, so the release that
// publishes them finds few dirty lines to write back; with plain stores the
// release of every helper wrote back the rows of all helpers on its XCD.
template <int GS, int NT>
__device__ __forceinline__ void accept_block_store(const Tabs &tb, bool coarse, const double *out,
                                                   double *const *dst) {
  const int C = tb.C, Cs = tb.Cs, t = threadIdx.x;
  if (coarse) {
    const auto row = glb(dst[0]);
    for (int k = t; k < C; k += NT) __hip_atomic_store(row + k, out[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const int g = t / GS, lane = t % GS;
  if (dst[g]) {
    const auto row = glb(dst[g]);
    for (int k = lane; k < C; k += GS)
      __hip_atomic_store(row + k, out[(size_t)g * Cs + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// the update of accept block blk, applied at once
template <int GS, int PM, typename R, int NT>
__device__ void accept_block(const Chain &ch, const Tabs &tb, const Move &mv, int blk, Lds<GS, NT> &sm) {
  double **dst = sm.dstp;
  bool coarse = accept_block_compute<GS, PM, R>(ch, tb, mv, blk, sm, sm.gbuf, dst);
  __syncthreads();
  accept_block_store<GS, NT>(tb, coarse, sm.gbuf, dst);
  __syncthreads();
}

// The whole update of an accepted move by one workgroup (one chain per
// workgroup): every group works through its own share of targets without
// workgroup barriers between them. Level 2: each of the 8 stored cells is
// split over NG/8 groups (candidates taken round robin, partial sums added
// in a fixed order); level 3: 64 stored cells over the groups; levels >= 4:
// the items of both interaction lists over the groups. A group sums the
// terms of a target in registers (P2L by columns, two points at a time),
// writes the sums once to its LDS buffer and adds them to the target row,
// whose loads are issued before the terms are formed.
template <int GS, int PM, typename R, int NT>
__device__ __forceinline__ void accept_all_wg(const Chain &ch, const Tabs &tb, const Move &mv, Lds<GS, NT> &sm) {
  constexpr int NG = NT / GS;
  constexpr int NJ = (PM + 1) * (PM + 1) / GS + 1;
  constexpr int SPLIT2 = NG / 8;  // NG is 32, 16 or 8
  static_assert(NG % 8 == 0 && SPLIT2 <= 4, "groups per workgroup");
  const int Cs = tb.Cs, C = tb.C;
  const int t = threadIdx.x, g = t / GS, lane = t % GS;
  const int L = ch.L;
  double *buf = sm.gbuf + (size_t)g * Cs;
  // rows stored without branches (finish_row) up to the p <= 12 variant; the
  // larger variants keep branched stores, whose addresses take no registers
  // of their own (the unbranched form spilled there and slowed the proposal)
  constexpr bool UNBRANCHED = PM <= 12;
  P2LCols<PM, R> cols;
  load_p2l_cols<PM, R>(lane, tb, sm.p2lg, cols);
  // the point of candidate `cand` (side 27 side + image) of stored cell s3
  // of coarse level l, in cell units from the image's centre
  auto coarse_pt = [&](int l, const int s3[3], int cand, R v[3], R &c) __attribute__((always_inline)) {
    const int n = 1 << (l - 1);
    const int side = cand / 27, e = cand % 27;
    const int w[3] = {e % 3 - 1, (e / 3) % 3 - 1, e / 9 - 1};
    const double *x = side ? mv.rn : mv.r;
    for (int k = 0; k < 3; ++k) v[k] = (R)fma(x[k], ch.inv_h[l], -((s3[k] + n * w[k]) + 0.5));
    c = (R)(side ? mv.q : -mv.q);
  };
  // the terms of every candidate in mask m, two at a time (four at a time
  // measured slower on one wavefront per SIMD); an odd last candidate is
  // paired with a zero charge at unit distance, so that the lane groups of a
  // wavefront run one pass
  auto coarse_sum = [&](int l, const int s3[3], uint64_t m, ColSum<PM> &cs) __attribute__((always_inline)) {
    while (m) {
      const int c0 = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      R v[2][3], q[2];
      coarse_pt(l, s3, c0, v[0], q[0]);
      if (m) {
        const int c1 = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        coarse_pt(l, s3, c1, v[1], q[1]);
      } else {
        v[1][0] = R(1);
        v[1][1] = v[1][2] = q[1] = R(0);
      }
      p2l_sum<GS, PM, R, 2>(lane, cols, v, q, cs);
    }
  };
  // row := old + sums (old read slot by slot before the sums were formed,
  // slots >= C as slot C - 1). UNBRANCHED: no store is branched on, a lane
  // whose slot lies beyond C stores slot C - 1 again, with the same value.
  // (With the stores under a branch the wavefront cannot count its
  // outstanding loads and stores, and waits for this row's stores before it
  // requests the next target's row.)
  auto finish_row = [&](gptr<double> dst, const double old[NJ], const ColSum<PM> &cs) __attribute__((always_inline)) {
    flush_p2l<PM>(lane, tb, sm.p2la, cs, buf, sm.red + 64);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      if constexpr (UNBRANCHED) {
        const int k = min(lane + j * GS, C - 1);
        dst[k] = old[j] + buf[k];
      } else {
        const int k = lane + j * GS;
        if (k < C) dst[k] = old[j] + buf[k];
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  };
  // ---- level 2: group g sums the candidates cand = part (mod SPLIT2) of cell g % 8
  {
    const int cell = g % 8, part = g / 8;
    const int s3[3] = {cell % 2, (cell / 2) % 2, cell / 4};
    const uint64_t every = SPLIT2 == 4 ? 0x1111111111111111ull : SPLIT2 == 2 ? 0x5555555555555555ull : ~0ull;
    const uint64_t m = coarse_mask<GS>(mv, 2, s3, lane, ch.free_space) & (every << part);
    ColSum<PM> cs;
    cs.zero();
    coarse_sum(2, s3, m, cs);
    flush_p2l<PM>(lane, tb, sm.p2la, cs, buf, sm.red + 64);
  }
  __syncthreads();
  if constexpr (!UNBRANCHED) {
    for (int i = t; i < 8 * C; i += NT) {
      const int cell = i / C, k = i % C;
      double sum = 0.0;
      for (int part = 0; part < SPLIT2; ++part) sum += sm.gbuf[(size_t)(cell + 8 * part) * Cs + k];
      const auto dst = glb(ch.Ld) + ch.ld_off[2] + (size_t)cell * Cs;
      dst[k] += sum;
    }
  } else {
    // the 8 rows: every value requested before any is stored (index i
    // beyond 8 C takes the last slot again, with the same value)
    constexpr int NR2 = (8 * (PM + 1) * (PM + 1) + NT - 1) / NT;
    const auto dst = glb(ch.Ld) + ch.ld_off[2];
    double old2[NR2];
#pragma unroll
    for (int r = 0; r < NR2; ++r) {
      const int i = min(t + r * NT, 8 * C - 1), cell = i / C, k = i % C;
      old2[r] = dst[(size_t)cell * Cs + k];
    }
#pragma unroll
    for (int r = 0; r < NR2; ++r) {
      const int i = min(t + r * NT, 8 * C - 1), cell = i / C, k = i % C;
      double sum = 0.0;
      for (int part = 0; part < SPLIT2; ++part) sum += sm.gbuf[(size_t)(cell + 8 * part) * Cs + k];
      dst[(size_t)cell * Cs + k] = old2[r] + sum;
    }
  }
  __syncthreads();
  // ---- level 3
  if (L >= 3) {
    for (int cell = g; cell < 64; cell += NG) {
      const int s3[3] = {cell % 4, (cell / 4) % 4, cell / 16};
      const auto dst = glb(ch.Ld) + ch.ld_off[3] + (size_t)cell * Cs;
      double old[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) old[j] = dst[min(lane + j * GS, C - 1)];
      const uint64_t m = coarse_mask<GS>(mv, 3, s3, lane, ch.free_space);
      ColSum<PM> cs;
      cs.zero();
      coarse_sum(3, s3, m, cs);
      finish_row(dst, old, cs);
    }
  }
  // ---- levels >= 4: one or two terms per item's own target
  // On a level where r and r' share their cell the two interaction lists
  // coincide and every new-side item belongs to the old side: such a level
  // contributes its 189 old-side items only.
  auto level_items = [&](int l) __attribute__((always_inline)) {
    const bool same = mv.c0[l][0] == mv.c1[l][0] && mv.c0[l][1] == mv.c1[l][1] && mv.c0[l][2] == mv.c1[l][2];
    return same ? 189 : 378;
  };
  int nfine = 0;
  for (int l = 4; l <= L; ++l) nfine += level_items(l);
  int fl_l = 4, fl_base = 0, fl_n = L >= 4 ? level_items(4) : 0;  // level of fl, its first index, its items
  FineLevel fl;
  if (L >= 4) fl = fine_level(ch, mv, 4);
  for (int i = g; i < nfine; i += NG) {
    while (i - fl_base >= fl_n) {  // the items of the next level (uniform over the group)
      fl_base += fl_n;
      ++fl_l;
      fl_n = level_items(fl_l);
      fl = fine_level(ch, mv, fl_l);
    }
    const FineItem it = fine_item(ch, tb, sm.il32, mv, fl, i - fl_base);
    if (!it.active) continue;
    const auto dst = glb(it.dst);
    double old[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) old[j] = dst[min(lane + j * GS, C - 1)];
    ColSum<PM> cs;
    cs.zero();
    {
      // one pass for one or two points, without a branch between the lane
      // groups of a wavefront (a missing second point has zero charge)
      const R v[2][3] = {{(R)it.v0[0], (R)it.v0[1], (R)it.v0[2]}, {(R)it.v1[0], (R)it.v1[1], (R)it.v1[2]}};
      const R q[2] = {(R)it.q0, (R)it.q1};
      p2l_sum<GS, PM, R, 2>(lane, cols, v, q, cs);
    }
    finish_row(dst, old, cs);
  }
  __syncthreads();
}

// Bookkeeping of an accepted move by one workgroup, on the LDS copies of
// K, H, dipole and running energy: K += dk, H += R(dk) (Sec. 3.4), and the
// position and leaf bins (the particle to cell map of Sec. 5.2), from the
// bin records kept in LDS (I_SLOTK, I_CNTOLD, I_CNTNEW, I_IDLAST, stash[0]).
// Returns nonzero on bin overflow.
template <int GS, int PM, bool REUSE = false, int NT>
__device__ __forceinline__ int accept_bookkeeping(const Chain &ch, const Tabs &tb, const Move &mv, double dE, Lds<GS, NT> &sm) {
  const int C = tb.C;
  const int t = threadIdx.x, g = t / GS, lane = t % GS;
  int *ints = sm.ints;
  const double a = ch.a, q = mv.q;
  if (!REUSE && g < 2) {
    const double *r = g ? mv.rn : mv.r;
    group_harmonics<GS, PM, 1, false>(lane, tb, sm.rec, (r[0] - 0.5 * a) / a, (r[1] - 0.5 * a) / a,
                                      (r[2] - 0.5 * a) / a, 1.0, g ? sm.latN : sm.latO);
  }
  if (t == NT - 1) {  // bins and position: stores only
    int ovf = 0;
    const int L = ch.L, n = 1 << (L - 1), B = ch.B;
    const int k = mv.idx;
    const int oldc = lin3(n, mv.c0[L][0], mv.c0[L][1], mv.c0[L][2]);
    const int newc = lin3(n, mv.c1[L][0], mv.c1[L][1], mv.c1[L][2]);
    const int sl = ints[I_SLOTK];
    const double4 rec = make_double4(mv.rn[0], mv.rn[1], mv.rn[2], q);
    if (oldc == newc) {
      st_rec(ch.bin_p, (size_t)oldc * B + sl, rec);
    } else {
      const int cnt = ints[I_CNTNEW];
      if (cnt >= B) {
        ovf = 1;
      } else {
        const int last = ints[I_CNTOLD] - 1;
        if (sl != last) {
          const int moved = ints[I_IDLAST];
          glb(ch.bin_id)[(size_t)oldc * B + sl] = moved;
          st_rec(ch.bin_p, (size_t)oldc * B + sl, sm.stash[0]);
          glb(ch.slot_of)[moved] = sl;
        }
        glb(ch.bin_cnt)[oldc] = last;
        glb(ch.bin_id)[(size_t)newc * B + cnt] = k;
        st_rec(ch.bin_p, (size_t)newc * B + cnt, rec);
        glb(ch.bin_cnt)[newc] = cnt + 1;
        glb(ch.slot_of)[k] = cnt;
        glb(ch.leaf_of)[k] = newc;
      }
    }
    if (!ovf) {
      glb(ch.px)[k] = mv.rn[0];
      glb(ch.py)[k] = mv.rn[1];
      glb(ch.pz)[k] = mv.rn[2];
      for (int j = 0; j < 3; ++j) sm.st[j] += q * (mv.rn[j] - mv.r[j]);
      sm.st[3] += dE;
    }
    ints[I_FLAG] = ovf;
  }
  __syncthreads();
  const int ovf = ints[I_FLAG];
  if (ovf) {  // unreachable after the decision-time test; the state is left as it was
    __syncthreads();
    return ovf;
  }
  if (REUSE) {
    // the proposal of this move left dk in sm.dk and R(dk) in sm.latO; its
    // conj T is the P2M term (the conjugate harmonics are a sign change per
    // slot), so these are bit for bit the values formed below
    for (int s = t; s < C; s += NT) {
      sm.K[s] += sm.dk[s];
      sm.H[s] += sm.latO[s];
    }
  } else {
    for (int s = t; s < C; s += NT) {
      sm.dk[s] = q * (sm.latN[s] - sm.latO[s]);
      sm.K[s] += sm.dk[s];
    }
    __syncthreads();
    with_lattice(tb, sm, [&](auto val, auto col) {
      lattice_rows<NT>(tb, val, col, sm.dk, [&](int s, double v) { sm.H[s] += v; });
    });
  }
  __syncthreads();
  return 0;
}

// the bin records of the bookkeeping, read from global memory (for an
// accept that was not preceded by this workgroup's proposal)
template <int GS, int NT>
__device__ void load_bin_records(const Chain &ch, const Move &mv, Lds<GS, NT> &sm) {
  if (threadIdx.x == 0) {
    const int L = ch.L, n = 1 << (L - 1), B = ch.B;
    const int oldc = lin3(n, mv.c0[L][0], mv.c0[L][1], mv.c0[L][2]);
    const int newc = lin3(n, mv.c1[L][0], mv.c1[L][1], mv.c1[L][2]);
    int *ints = sm.ints;
    ints[I_SLOTK] = glb(ch.slot_of)[mv.idx];
    ints[I_CNTOLD] = glb(ch.bin_cnt)[oldc];
    ints[I_CNTNEW] = glb(ch.bin_cnt)[newc];
    int last = ints[I_CNTOLD] - 1;
    ints[I_IDLAST] = glb(ch.bin_id)[(size_t)oldc * B + last];
    sm.stash[0] = ld_rec(ch.bin_p, (size_t)oldc * B + last);
  }
}

}  // namespace fmmdev
