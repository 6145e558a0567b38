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
  int c0[MAXL + 1][3];  // cell of r on each level
  int c1[MAXL + 1][3];  // cell of rn on each level
};

__device__ __forceinline__ void locate_move(const Chain &ch, Move &mv) {
  for (int l = 1; l <= ch.L; ++l) {
    int n = 1 << (l - 1);
    for (int k = 0; k < 3; ++k) {
      mv.c0[l][k] = cell_coord(mv.r[k], ch.a, n);
      mv.c1[l][k] = cell_coord(mv.rn[k], ch.a, n);
    }
  }
}

__device__ __forceinline__ int lin3(int n, int x, int y, int z) { return x + n * (y + n * z); }
__device__ __forceinline__ int imod(int i, int n) { return ((i % n) + n) % n; }
__device__ __forceinline__ int ifloordiv(int i, int n) { return (i - imod(i, n)) / n; }

// copy the recurrence constants into LDS (all threads; caller syncs)
template <int GS>
__device__ __forceinline__ void stage_rec(const Tabs &tb, Lds<GS> &sm) {
  for (int i = threadIdx.x; i < 3 * tb.Cs; i += NT) sm.rec[i] = tb.rec[i];
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
// the near region together with the matching self term (they cancel).
template <int GS>
__device__ ProposeOut propose_wg(const Chain &ch, const Tabs &tb, const Move &mv, Lds<GS> &sm) {
  constexpr int NG = NT / GS, PM = PmaxOf<GS>::v;
  const int Cs = tb.Cs, C = tb.C;
  const int t = threadIdx.x, g = t / GS, lane = t % GS;
  int *ncell = sm.ints, *nshift = sm.ints + 54, *npre = sm.ints + 108, *nmask = sm.ints + 164;

  const double a = ch.a, q = mv.q;
  const int L = ch.L, d = ch.d;
  const int npts = 2 * d + 2;

  // near-field cell list (54 entries: 27 around the old leaf, 27 around the new)
  if (t < 54) {
    int side = t / 27, e = t % 27;
    int ex = e % 3 - 1, ey = (e / 3) % 3 - 1, ez = e / 9 - 1;
    const int *c = side ? mv.c1[L] : mv.c0[L];
    int n = 1 << (L - 1);
    int b[3] = {c[0] + ex, c[1] + ey, c[2] + ez};
    int s = lin3(n, imod(b[0], n), imod(b[1], n), imod(b[2], n));
    int w = (ifloordiv(b[0], n) + 1) + 3 * (ifloordiv(b[1], n) + 1) + 9 * (ifloordiv(b[2], n) + 1);
    ncell[t] = s;
    nshift[t] = w;
    int cnt = ch.bin_cnt[s];
    npre[t + 1] = cnt;  // counts, turned into a prefix sum below
  }
  if (t == 0) nmask[0] = 0;
  __syncthreads();
  if (t < 64) {  // inclusive scan of the 54 counts in wave 0
    int v = t < 54 ? npre[t + 1] : 0;
    for (int o = 1; o < 64; o <<= 1) {
      int u = __shfl_up(v, o, 64);
      if (t >= o) v += u;
    }
    if (t < 54) npre[t + 1] = v;
    if (t == 0) npre[0] = 0;
  }

  // local expansions at the 2d level points and the two lattice points
  for (int base = 0; base < npts; base += NG) {
    int pt = base + g;
    if (pt < npts) {
      double *buf;
      double x[3], hh;
      const double *src;
      if (pt < 2) {  // lattice: expansion about the box centre, scaled by a
        buf = pt ? sm.latN : sm.latO;
        const double *r = pt ? mv.rn : mv.r;
        hh = a;
        for (int k = 0; k < 3; ++k) x[k] = (r[k] - 0.5 * a) / a;
        src = ch.H;
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
      // the expansion coefficients are loaded while the harmonics are formed
      double lv[(PmaxOf<GS>::v + 1) * (PmaxOf<GS>::v + 1) / GS + 1];
#pragma unroll
      for (int j = 0; j < (PM + 1) * (PM + 1) / GS + 1; ++j) {
        int s = lane + j * GS;
        lv[j] = s < C ? src[s] * tb.wl2p[s] : 0.0;
      }
      group_harmonics<GS, PM, 0, false>(lane, tb, sm.rec, x[0], x[1], x[2], 1.0, buf);
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < (PM + 1) * (PM + 1) / GS + 1; ++j) {
        int s = lane + j * GS;
        if (s < C) acc += lv[j] * buf[s];
      }
      acc = group_sum<GS>(acc);
      if (lane == 0) sm.vals[pt] = acc / hh;
    }
    __syncthreads();
  }

  // direct near field
  double dold = 0.0, dnew = 0.0;
  int singular = 0;
  const int total = npre[54];
  for (int i = t; i < total; i += NT) {
    int lo = 0, hi = 54;  // entry e with npre[e] <= i < npre[e+1]
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (npre[mid] <= i) lo = mid; else hi = mid;
    }
    int e = lo, j = i - npre[e];
    int side = e / 27, cell = ncell[e], w = nshift[e];
    double sx = (w % 3 - 1) * a, sy = ((w / 3) % 3 - 1) * a, sz = (w / 9 - 1) * a;
    int id = ch.bin_id[(size_t)cell * ch.B + j];
    double4 pj = ch.bin_p[(size_t)cell * ch.B + j];
    const double *x = side ? mv.rn : mv.r;
    if (id == mv.idx) {
      if (side) atomicOr(&nmask[0], 1 << w);
      if (side || w == 13) continue;  // w == 13: no image shift
    }
    double dx = x[0] - (pj.x + sx), dy = x[1] - (pj.y + sy), dz = x[2] - (pj.z + sz);
    double r2 = dx * dx + dy * dy + dz * dz;
    if (side && r2 == 0.0) singular = 1;
    double v = pj.w / sqrt(r2);
    if (side) dnew += v; else dold += v;
  }
  // far lattice quadratic term: dk = q (conj T(r') - conj T(r)), 1/2 dk.R(dk)
  for (int s = t; s < C; s += NT) sm.dk[s] = q * tb.sgnc[s] * (sm.latN[s] - sm.latO[s]);
  __syncthreads();
  // self-interaction with the old position's images (Sec. 3.4)
  double self = 0.0;
  if (t < 27 && !((nmask[0] >> t) & 1)) {
    double sx = (t % 3 - 1) * a, sy = ((t / 3) % 3 - 1) * a, sz = (t / 9 - 1) * a;
    double dx = mv.rn[0] - (mv.r[0] + sx), dy = mv.rn[1] - (mv.r[1] + sy), dz = mv.rn[2] - (mv.r[2] + sz);
    self = q * q / sqrt(dx * dx + dy * dy + dz * dz);
  }
  double quad = 0.0;
  lattice_rows(tb, sm.dk, [&](int s, double v) { quad += tb.wdot[s] * sm.dk[s] * v; });
  double part[4] = {dold, dnew, self, quad};
  wg_sum4(part, sm.red);
  int sing = __syncthreads_or(singular);

  ProposeOut out;
  double dE = 0.0;
  for (int l = 2; l <= L; ++l) {
    int po = 2 + 2 * (l - 2);
    dE += q * (sm.vals[po + 1] - sm.vals[po]);
  }
  dE += q * (part[1] - part[0]);
  dE += -part[2] + q * q / a * tb.self_const;
  dE += q * (sm.vals[1] - sm.vals[0]) + 0.5 * part[3] / a;
  double dr[3] = {mv.rn[0] - mv.r[0], mv.rn[1] - mv.r[1], mv.rn[2] - mv.r[2]};
  double Ddot = ch.dip[0] * dr[0] + ch.dip[1] * dr[1] + ch.dip[2] * dr[2];
  double dd = dr[0] * dr[0] + dr[1] * dr[1] + dr[2] * dr[2];
  dE += -2.0 * M_PI / (3.0 * a * a * a) * (2.0 * q * Ddot + q * q * dd);
  out.dE = dE;
  out.singular = sing;
  __syncthreads();
  return out;
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
// interaction list of cell c? returns the image in b
__device__ __forceinline__ bool image_in_il(const int s[3], const int c[3], int n, int b[3]) {
  int mx = 0;
  for (int k = 0; k < 3; ++k) {
    int lo = 2 * (c[k] >> 1) - 2;
    int v = lo + imod(s[k] - lo, n);
    if (v >= lo + 6) return false;
    b[k] = v;
    int dd = v - c[k];
    dd = dd < 0 ? -dd : dd;
    mx = dd > mx ? dd : mx;
  }
  return mx >= 2;
}

template <int GS>
__device__ void accept_block(const Chain &ch, const Tabs &tb, const Move &mv, int blk, Lds<GS> &sm) {
  constexpr int NG = NT / GS, PM = PmaxOf<GS>::v;
  const int Cs = tb.Cs, C = tb.C;
  const int t = threadIdx.x, g = t / GS, lane = t % GS;
  double *acc = sm.gbuf;  // NG * Cs
  int *lst = sm.ints;     // candidate list
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
    const double h = a / n;
    int s[3] = {s_lin % n, (s_lin / n) % n, s_lin / (n * n)};
    if (t < 64) {
      bool valid = false;
      int side = t / 27, e = t % 27;
      if (t < 54) {
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
    for (int i = t; i < NG * Cs; i += NT) acc[i] = 0.0;
    __syncthreads();
    int nv = lst[0];
    for (int i = g; i < nv; i += NG) {
      int cand = lst[1 + i];
      int side = cand / 27, e = cand % 27;
      int w[3] = {e % 3 - 1, (e / 3) % 3 - 1, e / 9 - 1};
      const double *x = side ? mv.rn : mv.r;
      double v[3];
      for (int k = 0; k < 3; ++k) v[k] = (x[k] - ((s[k] + n * w[k]) + 0.5) * h) / h;
      group_harmonics<GS, PM, 2, true>(lane, tb, sm.rec, v[0], v[1], v[2], side ? q : -q,
                                       acc + (size_t)g * Cs);
    }
    __syncthreads();
    double *dst = ch.Ld + ch.ld_off[l] + (size_t)s_lin * Cs;
    for (int k = t; k < C; k += NT) {
      double sum = 0.0;
      for (int gg = 0; gg < NG; ++gg) sum += acc[(size_t)gg * Cs + k];
      dst[k] += sum;
    }
    __syncthreads();
    return;
  }
  // ---- fine levels: item = (level, side, IL offset)
  int b2 = blk - 72;
  const int bpl = (378 + NG - 1) / NG;
  const int l = 4 + b2 / bpl;
  const int item = (b2 % bpl) * NG + g;
  if (l <= L && item < 378) {
    const int n = 1 << (l - 1);
    const double h = a / n;
    int side = item / 189, k189 = item % 189;
    const int *c = side ? mv.c1[l] : mv.c0[l];
    const int *co = side ? mv.c0[l] : mv.c1[l];
    int oc = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2);
    const int8_t *o = tb.il_off + (oc * 189 + k189) * 3;
    int b[3] = {c[0] + o[0], c[1] + o[1], c[2] + o[2]};
    int s[3] = {imod(b[0], n), imod(b[1], n), imod(b[2], n)};
    int b_other[3];
    bool other = image_in_il(s, co, n, b_other);
    if (side == 1 && other) return;  // owned by the old-side item
    double *buf = acc + (size_t)g * Cs;
    const double *dstc = ch.Ld + ch.ld_off[l] + (size_t)lin3(n, s[0], s[1], s[2]) * Cs;
    // the target's coefficients are loaded while the harmonics are formed
    double old[(PmaxOf<GS>::v + 1) * (PmaxOf<GS>::v + 1) / GS + 1];
#pragma unroll
    for (int j = 0; j < (PM + 1) * (PM + 1) / GS + 1; ++j) {
      int k = lane + j * GS;
      old[j] = k < C ? dstc[k] : 0.0;
    }
    const double *x = side ? mv.rn : mv.r;
    double v[3];
    for (int k = 0; k < 3; ++k) v[k] = (x[k] - (b[k] + 0.5) * h) / h;
    group_harmonics<GS, PM, 2, false>(lane, tb, sm.rec, v[0], v[1], v[2], side ? q : -q, buf);
    if (side == 0 && other) {
      __builtin_amdgcn_wave_barrier();
      for (int k = 0; k < 3; ++k) v[k] = (mv.rn[k] - (b_other[k] + 0.5) * h) / h;
      group_harmonics<GS, PM, 2, true>(lane, tb, sm.rec, v[0], v[1], v[2], q, buf);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    double *dst = ch.Ld + ch.ld_off[l] + (size_t)lin3(n, s[0], s[1], s[2]) * Cs;
#pragma unroll
    for (int j = 0; j < (PM + 1) * (PM + 1) / GS + 1; ++j) {
      int k = lane + j * GS;
      if (k < C) dst[k] = old[j] + buf[k];
    }
  }
}

// Bookkeeping of an accepted move by one workgroup: K += dk, H += R(dk),
// dipole, running energy, position and leaf bins (Sec. 3.4; the particle
// to cell map of Sec. 5.2). Returns nonzero on bin overflow.
template <int GS>
__device__ int accept_bookkeeping(const Chain &ch, const Tabs &tb, const Move &mv, double dE, Lds<GS> &sm) {
  constexpr int PM = PmaxOf<GS>::v;
  const int C = tb.C;
  const int t = threadIdx.x, g = t / GS, lane = t % GS;
  int *flag = sm.ints + 200;
  const double a = ch.a, q = mv.q;
  if (g < 2) {
    const double *r = g ? mv.rn : mv.r;
    group_harmonics<GS, PM, 1, false>(lane, tb, sm.rec, (r[0] - 0.5 * a) / a, (r[1] - 0.5 * a) / a,
                                      (r[2] - 0.5 * a) / a, 1.0, g ? sm.latN : sm.latO);
  }
  __syncthreads();
  for (int s = t; s < C; s += NT) {
    sm.dk[s] = q * (sm.latN[s] - sm.latO[s]);
    ch.K[s] += sm.dk[s];
  }
  __syncthreads();
  lattice_rows(tb, sm.dk, [&](int s, double v) { ch.H[s] += v; });
  if (t == 0) {
    int ovf = 0;
    for (int k = 0; k < 3; ++k) ch.dip[k] += q * (mv.rn[k] - mv.r[k]);
    ch.U[0] += dE;
    const int L = ch.L, n = 1 << (L - 1), B = ch.B;
    int k = mv.idx;
    int oldc = ch.leaf_of[k];
    int newc = lin3(n, mv.c1[L][0], mv.c1[L][1], mv.c1[L][2]);
    int sl = ch.slot_of[k];
    if (oldc == newc) {
      ch.bin_p[(size_t)oldc * B + sl] = make_double4(mv.rn[0], mv.rn[1], mv.rn[2], q);
    } else {
      int cnt = ch.bin_cnt[newc];
      if (cnt >= B) {
        ovf = 1;
      } else {
        int last = ch.bin_cnt[oldc] - 1;
        if (sl != last) {
          int moved = ch.bin_id[(size_t)oldc * B + last];
          ch.bin_id[(size_t)oldc * B + sl] = moved;
          ch.bin_p[(size_t)oldc * B + sl] = ch.bin_p[(size_t)oldc * B + last];
          ch.slot_of[moved] = sl;
        }
        ch.bin_cnt[oldc] = last;
        ch.bin_id[(size_t)newc * B + cnt] = k;
        ch.bin_p[(size_t)newc * B + cnt] = make_double4(mv.rn[0], mv.rn[1], mv.rn[2], q);
        ch.bin_cnt[newc] = cnt + 1;
        ch.slot_of[k] = cnt;
        ch.leaf_of[k] = newc;
      }
    }
    if (!ovf) {
      ch.px[k] = mv.rn[0];
      ch.py[k] = mv.rn[1];
      ch.pz[k] = mv.rn[2];
    }
    flag[0] = ovf;
  }
  __syncthreads();
  int ovf = flag[0];
  __syncthreads();
  return ovf;
}

}  // namespace fmmdev
