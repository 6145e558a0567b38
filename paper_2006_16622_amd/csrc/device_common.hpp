// device_common.hpp -- device-side data structures and building blocks of the
// multilevel Monte Carlo path: solid harmonics by a Cartesian recurrence,
// Philox4x64-10, exact-rounding wrap/locate, and workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmmdev {

// threads per workgroup: the batched run (one workgroup per chain) and the
// setup kernels use 512; the whole-GPU single chain and the single-call
// kernels use 256 (shorter barriers on the serial proposal path)
constexpr int WG_BATCH = 512;
constexpr int WG_SINGLE = 256;
constexpr int WG_SETUP = 512;
constexpr int MAXL = 8;       // levels (depth 7)
constexpr int NEAR = 27;      // leaf cells of a near region (Alg. 1)

// Constant tables shared by every chain of one degree p on one device.
struct Tabs {
  int p, C, Cs;                 // degree, coefficients, padded stride
  const double *rec;            // [3*Cs]: A_slot, B_slot (recurrence), c_m (diagonal)
  const double *wl2p;           // [Cs] weights of the real-layout L2P: 1, 2 (Re), -2 (Im)
  const double *wdot;           // [Cs] weights of the bilinear form E.H: 1, 2, 2
  const double *sgnc;           // [Cs] +1 for m >= 0 slots, -1 for m < 0 (conjugation)
  const int8_t *il_off;         // [8*189*3]
  const int16_t *il_id;         // [8*189] offset id in 0..315
  const double *m2l;            // [316][C in][Cs out]
  const float *m2l32;           // same in FP32 (mixed precision)
  const double *m2m;            // [8][C in][Cs out]
  int lat_w;                    // ELL width of the lattice operator
  int lat_lds;                  // nonzero: the run kernels keep it in LDS
  const int *lat_col;           // [lat_w][Cs] column of the w-th nonzero of row (output slot)
  const double *lat_val;        // [lat_w][Cs] its value (0 in padding)
  double self_const;            // 6 + 8/sqrt3 + 12/sqrt2
};

// Per-chain device state, carved out of the caller's workspace.
struct Chain {
  int N, d, L, B;               // charges, depth, levels (d+1), bin capacity
  int mixed;
  int free_space;               // free-space boundary conditions: no images, no lattice
  double a;                     // box side
  double scale;                 // factor applied to the staged positions (1; a volume move's s)
  double inv_h[MAXL + 2];       // n_l / a on level l (cells per unit length), one IEEE division
  double *px, *py, *pz, *pq;    // particles by id (wrapped positions)
  int *leaf_of, *slot_of;
  int *bin_cnt, *bin_id;        // [nleaf], [nleaf*B]
  double4 *bin_p;               // [nleaf*B] x, y, z, q
  double *Ld;                   // scaled local expansions, levels 2..L, cell-major, stride Cs
  double *Mp;                   // scaled multipoles, levels 1..L (setup)
  long long ld_off[MAXL + 2];   // offset (in doubles) of level l in Ld
  long long mp_off[MAXL + 2];
  double *K, *H;                // lattice moments (scaled by a) and H = R(K)
  double *dip;                  // [3]
  double *U;                    // [2]: running energy, setup energy
  int *status;                  // [4]: error code, overflow, singular count
  double *scratch;              // small scratch: [0] dE of the single-call propose
  double *mbox;                 // cross-workgroup mailbox (single-chain run)
  unsigned *sync;               // [4] sequence / done counters
  double *red;                  // partial sums of reductions
  double *part;                 // [512] per-workgroup partial sums of the whole-GPU run
  double *dscr;                 // chunk rows of the direct P2L setup (null without it)
  double *stage;                // raw host positions (3N) then charges (N)
};

// LDS layout of one workgroup of the Monte Carlo kernels. Besides scratch
// for the propose and accept phases it holds, for the whole launch, the
// constant tables the step needs (recurrence constants, L2P and bilinear
// weights, optionally the lattice operator) and the chain's small mutable
// state (K, H = R(K), dipole, running energy), written back at the end.
template <int GS, int NT>
struct Lds {
  static constexpr int NG = NT / GS;
  double *rec;                 // 3 Cs: recurrence constants
  float *rec32;                // 3 Cs: the same in FP32 (mixed precision evaluation)
  int *il32;                   // 8 * 189: interaction-list offsets per octant, one word each
  double **dstp;               // NG: destination rows of an accept block's groups
  double *wl2p, *wdot, *sgnc;  // Cs each
  double *H, *K;               // Cs each: chain state
  double *st;                  // 8: dipole[3], running energy, setup energy
  double *lat_val;             // W Cs (when resident)
  int *lat_col;                // W Cs (when resident)
  double *gbuf;                // NG Cs: one buffer per group
  double *latO, *latN, *dk;    // Cs each
  double *p2lg, *p2la;         // Cs each: P2L column constants g_j and alpha_j
  double *red;                 // NT
  double *vals;                // 32
  double4 *stash;              // 2: records kept by the proposal for the bookkeeping
  int *ints;                   // 384
  __device__ Lds(double *base, int Cs, int ellw) {
    rec = base;
    wl2p = rec + 3 * Cs;
    wdot = wl2p + Cs;
    sgnc = wdot + Cs;
    H = sgnc + Cs;
    K = H + Cs;
    st = K + Cs;
    lat_val = st + 8;
    gbuf = lat_val + (size_t)ellw * Cs;
    latO = gbuf + (size_t)NG * Cs;
    latN = latO + Cs;
    dk = latN + Cs;
    p2lg = dk + Cs;
    p2la = p2lg + Cs;
    red = p2la + Cs;
    vals = red + NT;
    stash = (double4 *)(vals + 32);
    ints = (int *)(stash + 2);
    lat_col = ints + 384;
    rec32 = (float *)(lat_col + (size_t)ellw * Cs);
    il32 = (int *)(rec32 + 3 * (size_t)Cs);
    dstp = (double **)(il32 + 8 * 189);
  }
  __host__ __device__ static size_t bytes(int Cs, int ellw) {
    return sizeof(double) * ((size_t)(NG + 14 + ellw) * Cs + 8 + NT + 32 + 8) + 4 * (384 + (size_t)ellw * Cs) +
           4 * 3 * (size_t)Cs + 4 * 8 * 189 + sizeof(double *) * NG;
  }
  // recurrence constants in the evaluation type
  template <typename R>
  __device__ const R *rec_of() const {
    if constexpr (sizeof(R) == 4)
      return rec32;
    else
      return rec;
  }
};

__device__ __forceinline__ int cslot(int n, int m) { return n * n + n + m; }

// the three signed byte offsets of an interaction-list entry, kept in LDS as
// one word (x in the low byte), so that an entry is a single LDS read
__device__ __forceinline__ int il_pack(const int8_t *o) {
  return (int)(uint8_t)o[0] | ((int)(uint8_t)o[1] << 8) | ((int)(uint8_t)o[2] << 16);
}
__device__ __forceinline__ void il_unpack(int w, int o[3]) {
  o[0] = (w << 24) >> 24;
  o[1] = (w << 16) >> 24;
  o[2] = (w << 8) >> 24;
}
// entry i of an interaction-list table: the packed LDS copy, or the byte
// table of the constant tables in global memory
__device__ __forceinline__ void il_entry(const int *il32, int i, int o[3]) { il_unpack(il32[i], o); }
__device__ __forceinline__ void il_entry(const int8_t *il, int i, int o[3]) {
  for (int k = 0; k < 3; ++k) o[k] = il[3 * i + k];
}

// Global-memory view of a workspace pointer. The chain's pointers reach the
// kernels through LDS, so the compiler no longer knows they address global
// memory and would use flat instructions, which also count against the LDS
// counter: every wait for an LDS result would then wait for all pending
// global stores too. Accesses through glb() are global instructions.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ gptr<T> glb(T *p) {
  return (gptr<T>)p;
}

// bin records (x, y, z, q) through the global view
typedef double dvec4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double4 ld_rec(const double4 *p, size_t i) {
  const dvec4 v = glb((const dvec4 *)p)[i];
  return make_double4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st_rec(double4 *p, size_t i, const double4 &r) {
  glb((dvec4 *)p)[i] = (dvec4){r.x, r.y, r.z, r.w};
}

// ------------------------------------------------------------------ rounding
// Wrap into [0, a): x - a floor(x/a), a result equal to a (or below 0 by
// rounding) becomes 0. FMA contraction is off in this function and in the
// displacement arithmetic below (plain operators under the pragma; the
// __d*_rn helpers are plain operators too and would be contracted): each
// operation rounds once, as IEEE double arithmetic without contraction does
// on the host.
__device__ __forceinline__ double wrap_coord(double x, double a) {
#pragma clang fp contract(off)
  double k = floor(x / a);
  double ak = a * k;
  double w = x - ak;
  if (w >= a) w = 0.0;
  if (w < 0.0) w = 0.0;
  return w;
}

// floor(x * (n/a)) clamped to [0, n-1]; a point on a face goes to the upper
// cell. inv = n/a is formed once per level by one IEEE division.
__device__ __forceinline__ int cell_coord(double x, double inv, int n) {
#pragma clang fp contract(off)
  int i = (int)floor(x * inv);
  return i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
}

// ------------------------------------------------------------------ Philox4x64-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11)
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    uint64_t y0 = hi1 ^ c[1] ^ k0, y2 = hi0 ^ c[3] ^ k1;
    c[0] = y0;
    c[1] = lo1;
    c[2] = y2;
    c[3] = lo0;
  }
}

// the two halves of the draw of Metropolis-Hastings step `step` of chain
// `chain`: counter (step, 0) gives idx and delta, counter (step, 1) gives u
__device__ __forceinline__ void mh_draw_move(uint64_t seed, uint64_t chain, uint64_t step, int64_t N, double D,
                                             int64_t &idx, double delta[3]) {
#pragma clang fp contract(off)
  uint64_t w[4] = {step, 0, 0, 0};
  philox4x64_10(w, seed, chain);
  idx = (int64_t)__umul64hi(w[0], (uint64_t)N);
  const double two53 = 1.0 / 9007199254740992.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double f = (double)(w[k + 1] >> 11) * two53;
    double two_f = 2.0 * f;
    double centred = two_f - 1.0;
    delta[k] = D * centred;
  }
}
__device__ __forceinline__ void mh_draw_u(uint64_t seed, uint64_t chain, uint64_t step, double &u) {
  uint64_t v[4] = {step, 1, 0, 0};
  philox4x64_10(v, seed, chain);
  const double two53 = 1.0 / 9007199254740992.0;
  u = (double)(v[0] >> 11) * two53;
}

// (idx, delta, u) of Metropolis-Hastings step `step` of chain `chain`
__device__ __forceinline__ void mh_draw(uint64_t seed, uint64_t chain, uint64_t step, int64_t N,
                                        double D, int64_t &idx, double delta[3], double &u) {
  mh_draw_move(seed, chain, step, N, D, idx, delta);
  mh_draw_u(seed, chain, step, u);
}

// ------------------------------------------------------------------ harmonics
// One group of GS lanes (GS > p) evaluates, for one point x (already divided
// by the cell size), the table of T_n^m(x) = |x|^n Y_n^m(x^), n <= p: lane m
// forms the diagonal T_m^m = c_m (x + i y)^m (the powers by a scan over the
// lanes) and runs the three-term recurrence in n down column m. Every lane
// of the group must call it. The result goes to the real-layout buffer
// buf (C doubles) as
//   KIND 0 (regular):         buf[n,m] = c Re T,         buf[n,-m] = c Im T
//   KIND 1 (conj. regular):   buf[n,m] = c Re T,         buf[n,-m] = -c Im T
//   KIND 2 (conj. irregular): buf[n,m] = c Re T / r^2n+1, buf[n,-m] = -c Im T / r^2n+1
// (KIND 1 is the P2M term q |s|^n Y_n^{-m}, KIND 2 the P2L term
// q |s|^-(n+1) Y_n^{-m} of Alg. L.2). With ACC the values are added.
// The loops are unrolled to PMAX so that the recurrence constants of the
// column are all loaded before the dependent arithmetic starts.
// rec layout: [0, Cs) A(n,m), [Cs, 2Cs) B(n,m) at slot(n,m); [2Cs, 2Cs+p] c_m.
// lane i of a group receives the value of lane i - O (lanes below O get
// zero with DPP, which scan_step turns into the unit factor, and their own
// value with the shuffle, which it discards); DPP row shifts when a group
// is one 16-lane row
template <int GS, int O>
__device__ __forceinline__ double shift_up(double v) {
  if constexpr (GS == 16) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, 0x110 + O, 0xf, 0xf, true);
    hi = __builtin_amdgcn_update_dpp(0, hi, 0x110 + O, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
  } else {
    return __shfl_up(v, O, GS);
  }
}

template <int GS, int O>
__device__ __forceinline__ float shift_up(float v) {
  if constexpr (GS == 16) {
    int b = __float_as_int(v);
    b = __builtin_amdgcn_update_dpp(0, b, 0x110 + O, 0xf, 0xf, true);
    return __int_as_float(b);
  } else {
    return __shfl_up(v, O, GS);
  }
}

template <int GS, int O, typename R>
__device__ __forceinline__ void scan_step(int lane, R &wr, R &wi, R &s, bool irregular) {
  if constexpr (O < GS) {
    R ur = shift_up<GS, O>(wr), ui = shift_up<GS, O>(wi);
    R us = irregular ? shift_up<GS, O>(s) : R(1);
    if constexpr (GS == 16) {
      // the DPP shift left zeros in the lanes below O: adding 1 to the real
      // part there makes their factor the unit (1 + 0i, exact), so every
      // lane multiplies and no result is selected (elsewhere + 0 is exact)
      const R one = lane < O ? R(1) : R(0);
      ur += one;
      R nr = wr * ur - wi * ui;
      R ni = wr * ui + wi * ur;
      wr = nr;
      wi = ni;
      if (irregular) s *= us + one;
    } else if (lane >= O) {
      R nr = wr * ur - wi * ui;
      R ni = wr * ui + wi * ur;
      wr = nr;
      wi = ni;
      if (irregular) s *= us;
    }
    scan_step<GS, 2 * O, R>(lane, wr, wi, s, irregular);
  }
}

__device__ __forceinline__ double sqrt_r(double v) { return sqrt(v); }
__device__ __forceinline__ float sqrt_r(float v) { return sqrtf(v); }

// R is the arithmetic type of the evaluation (double, or float in the mixed
// precision mode); the results are handed on as doubles. The core forms,
// in lane m, the column T_n^m for n = m .. p and passes each term
// c T_n^m (conjugated for KIND 1 and 2, divided by r^(2n+1) for KIND 2) to
// sink(j, n, re, im) with n = m + j. The recurrence runs unconditionally to
// the uniform bound p (rows beyond a lane's last row reuse a valid constant
// slot and are computed but not passed on) and its constants come through a
// restrict-qualified pointer, so their loads can be issued ahead of the
// dependent arithmetic; results leave through the sink only.
template <int GS, int PMAX, int KIND, typename R, bool ALL = false, typename Sink>
__device__ __forceinline__ void harmonics_core(int lane, const Tabs &tb, const R *__restrict__ rec, R x, R y, R z,
                                               R c, Sink &&sink) {
  const int p = tb.p, Cs = tb.Cs;
  const int m = lane;
  const R r2 = x * x + y * y + z * z;
  // (x + i y)^m and, for KIND 2, |x|^-(2m+1), by a multiplicative scan over the lanes
  R wr = m == 0 ? R(1) : x, wi = m == 0 ? R(0) : y;
  R inv_r2 = R(0), s = R(1);
  if (KIND == 2) {
    inv_r2 = R(1) / r2;
    s = m == 0 ? sqrt_r(inv_r2) : inv_r2;
  }
  scan_step<GS, 1, R>(lane, wr, wi, s, KIND == 2);
  if (m > p) return;
  const R cm = rec[2 * Cs + m];
  R tr = wr * cm, ti = wi * cm;
  R pr = R(0), pi = R(0);  // T_{n-2}
  const R im_sign = (KIND == 0) ? R(1) : R(-1);
#pragma unroll
  for (int j = 0; j <= PMAX; ++j) {
    if (j <= p) {  // uniform over the group
      if (j > 0) {
        const int n = m + j <= p ? m + j : p;  // a valid slot for rows beyond p
        const int sl = n * n + n + m;
        R a = rec[sl] * z, b = rec[Cs + sl] * r2;
        R nr = a * tr - b * pr;
        R ni = a * ti - b * pi;
        pr = tr;
        pi = ti;
        tr = nr;
        ti = ni;
        if (KIND == 2) s *= inv_r2;
      }
      if constexpr (ALL) {  // every row; the sink is told which are valid
        const R f = c * s;
        sink(j, m + j, (double)(f * tr), (double)(im_sign * f * ti), m + j <= p);
      } else if (m + j <= p) {
        const R f = c * s;
        sink(j, m + j, (double)(f * tr), (double)(im_sign * f * ti));
      }
    }
  }
}

// One group of GS lanes evaluates the table for one point into the
// real-layout buffer buf (C doubles): stored, or added with ACC. Each lane
// runs only its own rows (n <= p), loading the constants as it goes; for a
// single point this keeps the fewest registers live.
template <int GS, int PMAX, int KIND, bool ACC, typename R = double>
__device__ __forceinline__ void group_harmonics(int lane, const Tabs &tb, const R *__restrict__ rec, R x, R y, R z,
                                                R c, double *__restrict__ buf) {
  const int p = tb.p, Cs = tb.Cs;
  const int m = lane;
  const R r2 = x * x + y * y + z * z;
  R wr = m == 0 ? R(1) : x, wi = m == 0 ? R(0) : y;
  R inv_r2 = R(0), s = R(1);
  if (KIND == 2) {
    inv_r2 = R(1) / r2;
    s = m == 0 ? sqrt_r(inv_r2) : inv_r2;
  }
  scan_step<GS, 1, R>(lane, wr, wi, s, KIND == 2);
  if (m > p) return;
  const R cm = rec[2 * Cs + m];
  R tr = wr * cm, ti = wi * cm;
  R pr = R(0), pi = R(0);  // T_{n-2}
  const R im_sign = (KIND == 0) ? R(1) : R(-1);
#pragma unroll
  for (int j = 0; j <= PMAX; ++j) {
    const int n = m + j;
    if (n <= p) {
      if (j > 0) {
        const int sl = n * n + n + m;
        R a = rec[sl] * z, b = rec[Cs + sl] * r2;
        R nr = a * tr - b * pr;
        R ni = a * ti - b * pi;
        pr = tr;
        pi = ti;
        tr = nr;
        ti = ni;
        if (KIND == 2) s *= inv_r2;
      }
      const R f = c * s;
      const int sp = n * n + n + m;
      if (ACC)
        buf[sp] += (double)(f * tr);
      else
        buf[sp] = (double)(f * tr);
      if (m > 0) {
        const int sn = n * n + n - m;
        if (ACC)
          buf[sn] += (double)(im_sign * f * ti);
        else
          buf[sn] = (double)(im_sign * f * ti);
      }
    }
  }
}

// Column sums in registers: lane m holds sum c T_n^m for n = m + j in
// re[j], im[j]. Several points are added without touching memory; flush()
// then writes the column once. The additions are those of an accumulation
// in memory, in the same order.
template <int PMAX>
struct ColSum {
  double re[PMAX + 1], im[PMAX + 1];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int j = 0; j <= PMAX; ++j) re[j] = im[j] = 0.0;
  }
};

template <int GS, int PMAX, int KIND, typename R = double>
__device__ __forceinline__ void group_harmonics_sum(int lane, const Tabs &tb, const R *__restrict__ rec, R x, R y,
                                                    R z, R c, ColSum<PMAX> &acc) {
  harmonics_core<GS, PMAX, KIND, R>(lane, tb, rec, x, y, z, c, [&](int j, int, double re, double im) {
    acc.re[j] += re;
    acc.im[j] += im;
  });
}

// write (or add, with ACC) a group's column sums into the real-layout buffer
template <int PMAX, bool ACC, typename P>
__device__ __forceinline__ void flush_cols(int lane, const Tabs &tb, const ColSum<PMAX> &acc, P buf) {
  const int p = tb.p, m = lane;
  if (m > p) return;
#pragma unroll
  for (int j = 0; j <= PMAX; ++j) {
    const int n = m + j;
    if (n <= p) {
      const int sp = n * n + n + m;
      if (ACC)
        buf[sp] += acc.re[j];
      else
        buf[sp] = acc.re[j];
      if (m > 0) {
        const int sn = n * n + n - m;
        if (ACC)
          buf[sn] += acc.im[j];
        else
          buf[sn] = acc.im[j];
      }
    }
  }
}

// ------------------------------------------------------------------ P2L by columns
// The P2L term (KIND 2 above) summed over many points into one target, in
// a form with fewer operations per row, for the updates of an accepted move
// (Alg. L.2). With T_n^m = (x + i y)^m P_n (P real, P_m = c_m,
// P_n = A(n,m) z P_{n-1} - B(n,m) r^2 P_{n-2}), the term of row j (n = m + j)
// of column m is
//   c conj(T_n^m) / r^(2n+1) = alpha_j G S_j,  G = c conj(xi^m) / r,
//   xi = (x + i y) / r^2,  S_0 = 1,  S_1 = z / r^2,
//   S_j = (z / r^2) S_{j-1} + g_j S_{j-2} / r^2,
//   g_j = -B(n,m) / (A(n,m) A(n-1,m)),  alpha_j = c_m A(m+1,m) ... A(n,m),
// (S_j = P_n / (alpha_j r^(2j))). Both constants are tabulated once per
// workgroup; lane m keeps g_j in registers for a run of evaluations and sums
// G S_j over the points; alpha_j is applied once, when the sums are written
// out. Rows beyond p have g_j = 0 and are never
// written; neither are lanes beyond p.
__device__ __forceinline__ double rsqrt_nr(double v) {
  double y = __builtin_amdgcn_rsq(v);
#pragma unroll
  for (int i = 0; i < 2; ++i) {  // Newton steps for 1/sqrt(v)
    const double e = fma(-v * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}
__device__ __forceinline__ float rsqrt_nr(float v) {
  float y = __builtin_amdgcn_rsqf(v);
  const float e = fmaf(-v * y, y, 1.0f);
  return fmaf(0.5f * y, e, y);
}

template <int PMAX, typename R>
struct P2LCols {
  R g[PMAX + 1];  // g[j], j >= 2
};

// the constants of column m (one thread per column; rec: the recurrence
// constants in global memory): g_j and alpha_j at slot (m + j, m)
__device__ __forceinline__ void fill_p2l_cols(int m, const Tabs &tb, double *g, double *alpha) {
  const int p = tb.p, Cs = tb.Cs;
  const double *rec = tb.rec;
  if (m > p) return;
  double a = rec[2 * Cs + m];
  for (int n = m; n <= p; ++n) {
    const int s = n * n + n + m, s1 = (n - 1) * (n - 1) + (n - 1) + m;
    if (n > m) a *= rec[s];
    alpha[s] = a;
    g[s] = n >= m + 2 ? -rec[Cs + s] / (rec[s] * rec[s1]) : 0.0;
  }
}

template <int PMAX, typename R>
__device__ __forceinline__ void load_p2l_cols(int lane, const Tabs &tb, const double *g, P2LCols<PMAX, R> &cols) {
  const int p = tb.p, m = lane;
#pragma unroll
  for (int j = 0; j <= PMAX; ++j) {
    const int n = m + j;
    cols.g[j] = R(0);
    if (j >= 2 && n <= p) cols.g[j] = (R)g[n * n + n + m];
  }
}

// add the terms of K points (v[k] in cell units from the target's centre,
// charge c[k]) to the column sums; the K evaluations are interleaved row by
// row, each row's sum taking them in the order k = 0 .. K-1
template <int GS, int PMAX, typename R, int K>
__device__ __forceinline__ void p2l_sum(int lane, const P2LCols<PMAX, R> &cols, const R (&v)[K][3], const R (&c)[K],
                                        ColSum<PMAX> &acc) {
  R zz[K], ir2[K], gr[K], gi[K], s1[K], s2[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const R x = v[k][0], y = v[k][1], z = v[k][2];
    const R r2 = x * x + y * y + z * z;
    const R ir = rsqrt_nr(r2);
    ir2[k] = ir * ir;
    zz[k] = z * ir2[k];
    R wr = lane == 0 ? R(1) : x * ir2[k], wi = lane == 0 ? R(0) : y * ir2[k], unused = R(1);
    scan_step<GS, 1, R>(lane, wr, wi, unused, false);  // xi^m
    const R f = c[k] * ir;
    gr[k] = f * wr;
    gi[k] = -(f * wi);
    s2[k] = R(1);
    s1[k] = zz[k];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    acc.re[0] += (double)gr[k];
    acc.im[0] += (double)gi[k];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    acc.re[1] += (double)(gr[k] * s1[k]);
    acc.im[1] += (double)(gi[k] * s1[k]);
  }
#pragma unroll
  for (int j = 2; j <= PMAX; ++j) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const R sj = fma(cols.g[j], ir2[k] * s2[k], zz[k] * s1[k]);
      s2[k] = s1[k];
      s1[k] = sj;
      acc.re[j] += (double)(gr[k] * sj);
      acc.im[j] += (double)(gi[k] * sj);
    }
  }
}

// write a group's P2L column sums, times alpha_j, into the real-layout buffer.
// No store is branched on: a row beyond p (and every row of a lane beyond p)
// goes to a slot of the lane's own in `spare` (32 doubles, never read), and
// the imaginary part is written before the real one, so that for m = 0 the
// real part is the one that stays in the shared slot.
template <int PMAX, typename P>
__device__ __forceinline__ void flush_p2l(int lane, const Tabs &tb, const double *alpha, const ColSum<PMAX> &acc, P buf,
                                          double *spare) {
  const int p = tb.p, m = lane;
#pragma unroll
  for (int j = 0; j <= PMAX; ++j) {
    const int n = m + j;
    const bool valid = n <= p;
    const int sp = valid ? n * n + n + m : 0;
    const double a = alpha[sp];
    double *pi = valid && m > 0 ? &buf[n * n + n - m] : spare + (lane & 15);
    double *pr = valid ? &buf[sp] : spare + 16 + (lane & 15);
    *pi = a * acc.im[j];
    *pr = a * acc.re[j];
  }
}

// Butterfly all-reductions over aligned groups of W lanes (W = 16, 32, 64):
// step o combines each lane with lane ^ o, o = W/2 .. 1. The steps across
// 16-lane rows (32, 16) are shuffles; the steps inside a row are DPP row
// rotations by o, a single instruction. After the steps above o every value
// is unchanged under lane ^ o' for each o' > o inside the row, so the lane
// that a rotation by o reaches holds the same value as lane ^ o: the sums
// are those of the xor butterfly, bit for bit, in the same operand order.
template <int O>
__device__ __forceinline__ int row_ror(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x120 + O, 0xf, 0xf, true);
}
template <int O>
__device__ __forceinline__ double row_ror(double v) {
  const int lo = row_ror<O>(__double2loint(v)), hi = row_ror<O>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
template <int W, int O, int K>
__device__ __forceinline__ void sum_steps(double (&v)[K]) {
  if constexpr (O >= 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if constexpr (O >= 16)
        v[k] += __shfl_xor(v[k], O, W);
      else
        v[k] += row_ror<O>(v[k]);
    }
    sum_steps<W, O / 2, K>(v);
  }
}
// K values at once, their steps interleaved
template <int W, int K>
__device__ __forceinline__ void sum_allreduce(double (&v)[K]) {
  sum_steps<W, W / 2, K>(v);
}
template <int W, int O>
__device__ __forceinline__ unsigned or_steps(unsigned v) {
  if constexpr (O >= 1) {
    if constexpr (O >= 16)
      v |= (unsigned)__shfl_xor((int)v, O, W);
    else
      v |= (unsigned)row_ror<O>((int)v);
    return or_steps<W, O / 2>(v);
  } else {
    return v;
  }
}

// sum over the GS lanes of a group (lanes of one wavefront)
template <int GS>
__device__ __forceinline__ double group_sum(double v) {
  double a[1] = {v};
  sum_allreduce<GS, 1>(a);
  return a[0];
}

// deterministic workgroup sum of four values at once: a butterfly inside
// each wavefront, then the NT/64 wave totals in order; red: 16 doubles of LDS
template <int NT>
__device__ __forceinline__ void wg_sum4(double v[4], double *red) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double w[4] = {v[0], v[1], v[2], v[3]};
  sum_allreduce<64, 4>(w);
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = w[k];
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) red[4 * wv + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[4 * w + k];
    v[k] = s;
  }
  __syncthreads();
}

// deterministic workgroup sum (fixed tree); red: NT doubles of LDS
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double *red) {
  int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// widest ELL row of the lattice operator for the degrees a kernel variant
// serves (the tables are padded to it with zero entries)
__host__ __device__ constexpr int ell_width(int pm) { return pm <= 8 ? 10 : pm <= 12 ? 21 : pm <= 15 ? 36 : 78; }

// y[s] = sum_k R[s][k] x[k] over the padded ELL layout, width W known at
// compile time, so that all of a row's loads are issued before its sums;
// the even and odd entries are summed apart and then added, the order of
// lattice_rows below (padding entries add +0)
template <int NT, int W, typename PV, typename PC, typename F>
__device__ __forceinline__ void lattice_rows_w(const Tabs &tb, PV val, PC col, const double *x, F &&use) {
  for (int s = threadIdx.x; s < tb.C; s += NT) {
    double a[W];
    int c[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      a[w] = val[(size_t)w * tb.Cs + s];
      c[w] = col[(size_t)w * tb.Cs + s];
    }
    double v0 = 0.0, v1 = 0.0;
#pragma unroll
    for (int w = 0; w + 1 < W; w += 2) {
      v0 += a[w] * x[c[w]];
      v1 += a[w + 1] * x[c[w + 1]];
    }
    if (W % 2) v0 += a[W - 1] * x[c[W - 1]];
    use(s, v0 + v1);
  }
}

// y[s] = sum_k R[s][k] x[k] over the ELL layout of the lattice operator for
// the output slots s = t, t + NT, ... of the calling thread, handed to `use`
template <int NT, typename PV, typename PC, typename F>
__device__ __forceinline__ void lattice_rows(const Tabs &tb, PV val, PC col, const double *x, F &&use) {
  for (int s = threadIdx.x; s < tb.C; s += NT) {
    double v0 = 0.0, v1 = 0.0;
    int w = 0;
    for (; w + 1 < tb.lat_w; w += 2) {
      double a0 = val[(size_t)w * tb.Cs + s], a1 = val[(size_t)(w + 1) * tb.Cs + s];
      int c0 = col[(size_t)w * tb.Cs + s], c1 = col[(size_t)(w + 1) * tb.Cs + s];
      v0 += a0 * x[c0];
      v1 += a1 * x[c1];
    }
    if (w < tb.lat_w) v0 += val[(size_t)w * tb.Cs + s] * x[col[(size_t)w * tb.Cs + s]];
    use(s, v0 + v1);
  }
}

}  // namespace fmmdev
