// setup_kernels.hpp -- the O(N) initialisation of the expansions (Sec. 3.2,
// FMM-pass variant without L2L, and Sec. 3.4 periodic moments): wrap and bin
// the charges, P2M on the leaves, M2M upwards, M2L over the interaction
// lists on levels 2..L, the lattice term, and the total energy.
#pragma once

#include "device_common.hpp"
#include "mp_step.hpp"

namespace fmmdev {

__global__ void k_fill_i32(int *p, int v, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double *p, double v, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Every setup kernel serves several chains at once: blockIdx.y is the
// chain, the chain descriptors are an array in device memory, and blocks
// beyond a chain's own size return at once. One chain is a batch of one.

// clear the bin counts, the status words and the run's sequence counters
__global__ void k_setup_clear(const Chain *chains) {
  const Chain &ch = chains[blockIdx.y];
  const long long nleaf = 1LL << (3 * ch.d);
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nleaf) ch.bin_cnt[i] = 0;
  if (blockIdx.x == 0) {
    if (threadIdx.x < 8) ch.status[threadIdx.x] = 0;
    for (int k = threadIdx.x; k < 512; k += blockDim.x) ch.sync[k] = 0u;
  }
}

// copy the current positions and charges into the staging area (re-setup
// from the device-resident state)
__global__ void k_restage(const Chain *chains) {
  const Chain &ch = chains[blockIdx.y];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ch.N) return;
  ch.stage[3 * i + 0] = ch.px[i];
  ch.stage[3 * i + 1] = ch.py[i];
  ch.stage[3 * i + 2] = ch.pz[i];
  ch.stage[3 * ch.N + i] = ch.pq[i];
}

// scale (by ch.scale: 1, or the factor of a volume move; a product by 1 is
// exact) and wrap the staged positions, locate leaf cells, count bin
// occupancy
__global__ void k_stage(const Chain *chains) {
  const Chain &ch = chains[blockIdx.y];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ch.N) return;
  double x = wrap_coord(ch.stage[3 * i + 0] * ch.scale, ch.a);
  double y = wrap_coord(ch.stage[3 * i + 1] * ch.scale, ch.a);
  double z = wrap_coord(ch.stage[3 * i + 2] * ch.scale, ch.a);
  double q = ch.stage[3 * ch.N + i];
  ch.px[i] = x;
  ch.py[i] = y;
  ch.pz[i] = z;
  ch.pq[i] = q;
  int n = 1 << (ch.L - 1);
  const double inv = ch.inv_h[ch.L];
  int c = lin3(n, cell_coord(x, inv, n), cell_coord(y, inv, n), cell_coord(z, inv, n));
  ch.leaf_of[i] = c;
  int s = atomicAdd(&ch.bin_cnt[c], 1);
  if (s < ch.B)
    ch.bin_id[(size_t)c * ch.B + s] = i;
  else
    atomicMax(&ch.status[1], 1);
}

// deterministic bin order (ascending particle id), packed particle records
__global__ void k_bin_finalize(const Chain *chains) {
  const Chain &ch = chains[blockIdx.y];
  const int nleaf = 1 << (3 * ch.d);
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nleaf) return;
  int cnt = ch.bin_cnt[c];
  if (cnt > ch.B) cnt = ch.B;
  int *ids = ch.bin_id + (size_t)c * ch.B;
  for (int i = 1; i < cnt; ++i) {
    int v = ids[i], j = i - 1;
    while (j >= 0 && ids[j] > v) {
      ids[j + 1] = ids[j];
      --j;
    }
    ids[j + 1] = v;
  }
  for (int j = 0; j < cnt; ++j) {
    int id = ids[j];
    ch.bin_p[(size_t)c * ch.B + j] = make_double4(ch.px[id], ch.py[id], ch.pz[id], ch.pq[id]);
    ch.slot_of[id] = j;
  }
}

// P2M on the leaves, Eq. (multipole_expansion_coefficients), scaled by the
// leaf size: M^_n^m = sum q (|s|/h)^n Y_n^{-m}; one lane group per leaf
template <int GS, int PM>
__global__ void __launch_bounds__(WG_SETUP) k_p2m_leaf(const Chain *chains, Tabs tb) {
  constexpr int NG = WG_SETUP / GS;
  extern __shared__ double lds[];
  const Chain &ch = chains[blockIdx.y];
  const int nleaf = 1 << (3 * ch.d);
  const int g = threadIdx.x / GS, lane = threadIdx.x % GS, Cs = tb.Cs;
  double *buf = lds + (size_t)g * Cs;
  int c = blockIdx.x * NG + g;
  if (c >= nleaf) return;
  const int n = 1 << (ch.L - 1);
  const double h = ch.a / n;
  int cx = c % n, cy = (c / n) % n, cz = c / (n * n);
  for (int s = lane; s < Cs; s += GS) buf[s] = 0.0;
  __builtin_amdgcn_wave_barrier();
  int cnt = ch.bin_cnt[c];
  ColSum<PM> cs;
  cs.zero();
  for (int j = 0; j < cnt; ++j) {
    double4 pj = ch.bin_p[(size_t)c * ch.B + j];
    group_harmonics_sum<GS, PM, 1>(lane, tb, tb.rec, (pj.x - (cx + 0.5) * h) / h, (pj.y - (cy + 0.5) * h) / h,
                                   (pj.z - (cz + 0.5) * h) / h, pj.w, cs);
  }
  flush_cols<PM, false>(lane, tb, cs, buf);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  double *dst = ch.Mp + ch.mp_off[ch.L] + (size_t)c * Cs;
  for (int s = lane; s < Cs; s += GS) dst[s] = buf[s];
}

// M2M from level l+1 to level l (one workgroup per parent cell); chains
// whose finest level is l or coarser take no part
__global__ void k_m2m(const Chain *chains, Tabs tb, int l) {
  const Chain &ch = chains[blockIdx.y];
  if (l >= ch.L) return;
  const int n = 1 << (l - 1), nc = 2 * n, C = tb.C, Cs = tb.Cs;
  int pc = blockIdx.x;
  if (pc >= n * n * n) return;
  int px = pc % n, py = (pc / n) % n, pz = pc / (n * n);
  const double *child = ch.Mp + ch.mp_off[l + 1];
  double *dst = ch.Mp + ch.mp_off[l] + (size_t)pc * Cs;
  for (int j = threadIdx.x; j < Cs; j += blockDim.x) {
    double acc = 0.0;
    if (j < C) {
      for (int oc = 0; oc < 8; ++oc) {
        int cl = lin3(nc, 2 * px + (oc & 1), 2 * py + ((oc >> 1) & 1), 2 * pz + ((oc >> 2) & 1));
        const double *m = child + (size_t)cl * Cs;
        const double *op = tb.m2m + (size_t)oc * C * Cs + j;
        for (int s = 0; s < C; ++s) acc += op[(size_t)s * Cs] * m[s];
      }
    }
    dst[j] = acc;
  }
}

// ------------------------------------------------------------------ M2L
// L^_a = sum over the 189 offsets o of IL(octant of a) of T_o M^_{(a+o) mod n}
// (the FMM initialisation without L2L, Sec. 3.2). The operators T_o do not
// depend on the level (coefficients are scaled by the cell size), so every
// target cell of one octant, on any level of any chain, multiplies the same
// 189 matrices: a batched GEMM on the matrix cores. A tile is up to
// M2L_TT targets of one octant of one chain; a workgroup computes TO output
// coefficients of its tile, so each operator element it stages serves the
// tile's targets. The four wavefronts each own (TO / 32) x (M2L_TT / 32)
// 16 x 16 accumulator blocks; inputs are staged through LDS in chunks of
// 16, double-buffered, the multipoles gathered per target.
// In FP32 the matrix cores accumulate one offset's product (at most Cs
// terms per output) and each offset's partial sum is added into an FP64
// accumulator, so the rounding of the 189-offset sum is FP64's.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row within the 16 x 16 block of accumulator element v of lane `lane`
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int M2L_NT = 256;  // threads of the M2L kernel
constexpr int M2L_TT = 64;   // targets per tile (128 measured slower: fewer workgroups)
constexpr int M2L_KC = 16;   // inputs per staged chunk

// target t of an octant's list (levels 2, 3, ... in turn, 8^(l-2) targets
// on level l, each level's targets in x-fastest order): its level and cell
__device__ __forceinline__ int m2l_target(int t, int oc, int c[3]) {
  int l = 2, base = 0, cnt = 1;
  while (t >= base + cnt) {
    base += cnt;
    cnt <<= 3;
    ++l;
  }
  const int i = t - base, sh = l - 2, half = 1 << sh;
  c[0] = 2 * (i & (half - 1)) + (oc & 1);
  c[1] = 2 * ((i >> sh) & (half - 1)) + ((oc >> 1) & 1);
  c[2] = 2 * (i >> (2 * sh)) + (oc >> 2);
  return l;
}

template <typename T, int TO>
__global__ void __launch_bounds__(M2L_NT) k_m2l(const Chain *chains, Tabs tb, const int4 *tiles, const T *ops) {
  using MF = Mfma<T>;
  constexpr int RB = TO / 32;  // row blocks of a wavefront
  __shared__ T As[2][M2L_KC][TO];
  __shared__ T Bs[2][M2L_KC][M2L_TT];
  const int4 tl = tiles[blockIdx.x];
  const Chain &ch = chains[tl.x];
  const int oc = tl.y, first = tl.z, count = tl.w;
  const int j0 = blockIdx.y * TO;
  const int C = tb.C, Cs = tb.Cs;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  constexpr int CB = M2L_TT / 32;  // column blocks of a wavefront
  constexpr int BR = M2L_KC * M2L_TT / M2L_NT;  // inputs per thread and chunk
  const int ro = (w >> 1) * (TO / 2), co = (w & 1) * (M2L_TT / 2);
  // loader roles: A rows t/16 of the chunk, 4 outputs at (t%16)*4 + 64 r;
  // B target t % M2L_TT, inputs BR (t / M2L_TT) .. + BR - 1 of the chunk
  const int arow = t >> 4, acol = (t & 15) * 4;
  const int bt = t % M2L_TT, brow = (t / M2L_TT) * BR;
  const bool bvalid = bt < count;
  int bc[3] = {0, 0, 0}, bn = 1;
  const double *bsrc = nullptr;
  if (bvalid) {
    const int l = m2l_target(first + bt, oc, bc);
    bn = 1 << (l - 1);
    bsrc = ch.Mp + ch.mp_off[l];
  }
  constexpr int AR = (TO + 63) / 64;
  const int nq = (C + M2L_KC - 1) / M2L_KC;
  const int total = 189 * nq;
  T ra[AR][4], rb[BR];
  auto fetch = [&](int it) {
    const int k = it / nq, s0 = (it - k * nq) * M2L_KC;
    const int id = tb.il_id[oc * 189 + k];
    const int s = s0 + arow;
#pragma unroll
    for (int r = 0; r < AR; ++r) {
      const int col = acol + 64 * r;
      const bool ok = s < C && col < TO && j0 + col < Cs;
      const T *pa = ops + ((size_t)id * C + (ok ? s : 0)) * Cs + j0 + (ok ? col : 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) ra[r][e] = ok ? pa[e] : (T)0;
    }
    const int8_t *o = tb.il_off + (oc * 189 + k) * 3;
    const int bx = bc[0] + o[0], by = bc[1] + o[1], bz = bc[2] + o[2];
    const bool inside = bx >= 0 && bx < bn && by >= 0 && by < bn && bz >= 0 && bz < bn;
    if (bvalid && (inside || !ch.free_space)) {  // free space: no images
      const int x = imod(bx, bn), y = imod(by, bn), z = imod(bz, bn);
      const double *pb = bsrc + (size_t)lin3(bn, x, y, z) * Cs + s0 + brow;
#pragma unroll
      for (int e = 0; e < BR; ++e) rb[e] = (T)pb[e];
    } else {
#pragma unroll
      for (int e = 0; e < BR; ++e) rb[e] = (T)0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int r = 0; r < AR; ++r) {
      const int col = acol + 64 * r;
      if (col < TO)
#pragma unroll
        for (int e = 0; e < 4; ++e) As[buf][arow][col + e] = ra[r][e];
    }
#pragma unroll
    for (int e = 0; e < BR; ++e) Bs[buf][brow + e][bt] = rb[e];
  };
  typename MF::acc_t acc[RB][CB];
  constexpr bool split = sizeof(T) == 4;
  double accd[split ? RB : 1][CB][4];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = (typename MF::acc_t){0, 0, 0, 0};
  if constexpr (split)
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < CB; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) accd[i][j][v] = 0.0;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int it = 0; it < total; ++it) {
    const int buf = it & 1;
    if (it + 1 < total) fetch(it + 1);
#pragma unroll
    for (int k4 = 0; k4 < M2L_KC; k4 += 4) {
      const int kr = k4 + (lane >> 4);
      T b[CB];
#pragma unroll
      for (int j = 0; j < CB; ++j) b[j] = Bs[buf][kr][co + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const T a = As[buf][kr][ro + 16 * i + (lane & 15)];
#pragma unroll
        for (int j = 0; j < CB; ++j) acc[i][j] = MF::mma(a, b[j], acc[i][j]);
      }
    }
    if constexpr (split) {
      if ((it + 1) % nq == 0) {  // the last chunk of an offset: fold into FP64
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) accd[i][j][v] += (double)acc[i][j][v];
            acc[i][j] = (typename MF::acc_t){0, 0, 0, 0};
          }
      }
    }
    if (it + 1 < total) stash(buf ^ 1);
    __syncthreads();
  }
  // store: lane holds, per block, target co + 16 j + lane%16 and rows MF::row
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int tt = co + 16 * j + (lane & 15);
    if (tt >= count) continue;
    int c[3];
    const int l = m2l_target(first + tt, oc, c);
    const int n = 1 << (l - 1);
    double *dst = ch.Ld + ch.ld_off[l] + (size_t)lin3(n, c[0], c[1], c[2]) * Cs;
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = j0 + ro + 16 * i + MF::row(lane, v);
        double val;
        if constexpr (split)
          val = accd[i][j][v];
        else
          val = acc[i][j][v];
        if (r < Cs) dst[r] = val;
      }
  }
}

// Direct P2L initialisation, Alg. L.3, ordered by target: the relation
// "beta lies in IL(alpha)" is symmetric (with the image offset negated), so
// the local expansion of cell beta on level l is the sum, over the 189 cells
// alpha of IL(beta) (images included), of the P2L of every charge of alpha
// at the centre of beta. The items of a target are the pairs (offset k,
// leaf j below alpha), 189 * 8^(L-l) of them; they are cut into chunks of
// P2L_CHUNK items, and one workgroup forms one chunk: its lane groups take
// the items in turn, sum their charges' terms in registers, and the groups'
// sums are added in a fixed order. A target with one chunk is written to
// its row directly; otherwise each chunk goes to the chain's scratch rows,
// and k_p2l_reduce adds the chunks in order.
constexpr int P2L_CHUNK = 1024;
__host__ __device__ inline long long p2l_items(int L, int l) { return 189LL << (3 * (L - l)); }
__host__ __device__ inline int p2l_chunks(int L, int l) {
  return (int)((p2l_items(L, l) + P2L_CHUNK - 1) / P2L_CHUNK);
}

template <int GS, int PM>
__global__ void __launch_bounds__(WG_SETUP) k_p2l_direct(const Chain *chains, Tabs tb, int l) {
  constexpr int NG = WG_SETUP / GS;
  extern __shared__ double lds[];
  const Chain &ch = chains[blockIdx.y];
  if (l > ch.L) return;
  const int n = 1 << (l - 1), sh = ch.L - l, m = 1 << sh, nL = 1 << (ch.L - 1);
  const int nch = p2l_chunks(ch.L, l);
  const long long ntarget = 1LL << (3 * (l - 1));
  if ((long long)blockIdx.x >= ntarget * nch) return;
  const int target = blockIdx.x / nch, chunk = blockIdx.x % nch;
  const int g = threadIdx.x / GS, lane = threadIdx.x % GS, Cs = tb.Cs, C = tb.C;
  const double a = ch.a, h = a / n;
  const int c[3] = {target % n, (target / n) % n, target / (n * n)};
  const int oc = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2);
  const long long it0 = (long long)chunk * P2L_CHUNK;
  const long long it1 = it0 + P2L_CHUNK < p2l_items(ch.L, l) ? it0 + P2L_CHUNK : p2l_items(ch.L, l);
  ColSum<PM> cs;
  cs.zero();
  for (long long it = it0 + g; it < it1; it += NG) {
    const int k = (int)(it >> (3 * sh)), j = (int)(it & ((1LL << (3 * sh)) - 1));
    const int8_t *o = tb.il_off + (oc * 189 + k) * 3;
    const int b[3] = {c[0] + o[0], c[1] + o[1], c[2] + o[2]};
    if (ch.free_space && (b[0] < 0 || b[0] >= n || b[1] < 0 || b[1] >= n || b[2] < 0 || b[2] >= n)) continue;
    int leaf[3];
    double shift[3];
    for (int d = 0; d < 3; ++d) {
      const int s = imod(b[d], n);
      shift[d] = ifloordiv(b[d], n) * a;
      leaf[d] = s * m;
    }
    leaf[0] += j % m;
    leaf[1] += (j / m) % m;
    leaf[2] += j / (m * m);
    const int lf = lin3(nL, leaf[0], leaf[1], leaf[2]);
    const int cnt = ch.bin_cnt[lf];
    for (int t = 0; t < cnt; ++t) {
      const double4 pj = ch.bin_p[(size_t)lf * ch.B + t];
      group_harmonics_sum<GS, PM, 2>(lane, tb, tb.rec, (pj.x + shift[0] - (c[0] + 0.5) * h) / h,
                                     (pj.y + shift[1] - (c[1] + 0.5) * h) / h,
                                     (pj.z + shift[2] - (c[2] + 0.5) * h) / h, pj.w, cs);
    }
  }
  double *buf = lds + (size_t)g * Cs;
  for (int s = lane; s < Cs; s += GS) buf[s] = 0.0;
  __builtin_amdgcn_wave_barrier();
  flush_cols<PM, false>(lane, tb, cs, buf);
  __syncthreads();
  double *dst = nch == 1 ? ch.Ld + ch.ld_off[l] + (size_t)target * Cs
                         : ch.dscr + ((size_t)target * nch + chunk) * Cs;
  for (int s = threadIdx.x; s < C; s += WG_SETUP) {
    double v = 0.0;
    for (int gg = 0; gg < NG; ++gg) v += lds[(size_t)gg * Cs + s];
    dst[s] = v;
  }
}

// the chunks of each target of level l added in order into its row
__global__ void k_p2l_reduce(const Chain *chains, Tabs tb, int l) {
  const Chain &ch = chains[blockIdx.y];
  if (l > ch.L) return;
  const int nch = p2l_chunks(ch.L, l);
  const long long ntarget = 1LL << (3 * (l - 1));
  if (nch == 1 || (long long)blockIdx.x >= ntarget) return;
  const int target = blockIdx.x, Cs = tb.Cs;
  double *row = ch.Ld + ch.ld_off[l] + (size_t)target * Cs;
  const double *src = ch.dscr + (size_t)target * nch * Cs;
  for (int s = threadIdx.x; s < tb.C; s += blockDim.x) {
    double v = 0.0;
    for (int k = 0; k < nch; ++k) v += src[(size_t)k * Cs + s];
    row[s] = v;
  }
}

// K = level-1 multipole (about the box centre, scaled by a); H = R(K);
// dipole D = sum q r (one workgroup per chain)
__global__ void k_lattice_init(const Chain *chains, Tabs tb) {
  const Chain &ch = chains[blockIdx.y];
  __shared__ double red[WG_SETUP];
  const int C = tb.C, t = threadIdx.x;
  const double *M1 = ch.Mp + ch.mp_off[1];
  for (int s = t; s < C; s += WG_SETUP) ch.K[s] = M1[s];
  __syncthreads();
  lattice_rows<WG_SETUP>(tb, tb.lat_val, tb.lat_col, M1, [&](int s, double v) { ch.H[s] = v; });
  double d[3] = {0, 0, 0};
  for (int i = t; i < ch.N; i += WG_SETUP) {
    d[0] += ch.pq[i] * ch.px[i];
    d[1] += ch.pq[i] * ch.py[i];
    d[2] += ch.pq[i] * ch.pz[i];
  }
  for (int k = 0; k < 3; ++k) {
    double v = wg_sum<WG_SETUP>(d[k], red);
    if (t == 0) ch.dip[k] = v;
  }
}

// per-particle potential phi_i = sum_l Psi^D_l(r_i) + near(r_i) (excluding
// the particle itself, images included); block partial sums of
// 1/2 q_i phi_i written to ch.red[block]. In the multipole-based variant
// (MP) the far part is the sum over levels of the multipoles of the
// interaction list of the particle's cell, evaluated at r_i (Sec. 3.3).
template <int GS, int PM, bool MP = false>
__global__ void __launch_bounds__(WG_SETUP) k_energy(const Chain *chains, Tabs tb) {
  constexpr int NG = WG_SETUP / GS;
  extern __shared__ double lds[];
  __shared__ double red[WG_SETUP];
  const Chain &ch = chains[blockIdx.y];
  if ((long long)blockIdx.x * NG >= ch.N) return;
  const int g = threadIdx.x / GS, lane = threadIdx.x % GS, Cs = tb.Cs, C = tb.C;
  double *buf = lds + (size_t)g * Cs;
  int i = blockIdx.x * NG + g;
  double contrib = 0.0;
  if (i < ch.N) {
    const double a = ch.a;
    double r[3] = {ch.px[i], ch.py[i], ch.pz[i]};
    double phi = 0.0;
    if constexpr (MP) {
      double far = 0.0;
      for (int l = 2; l <= ch.L; ++l) {
        const int n = 1 << (l - 1);
        int c[3];
        for (int k = 0; k < 3; ++k) c[k] = cell_coord(r[k], ch.inv_h[l], n);
        for (int k = 0; k < 189; ++k) far += m2p_cell<GS, PM>(ch, tb, tb.rec, tb.il_off, l, c, r, k, lane);
      }
      phi += group_sum<GS>(far);
    }
    for (int l = 2; l <= ch.L && !MP; ++l) {
      int n = 1 << (l - 1);
      double h = a / n;
      int c[3];
      for (int k = 0; k < 3; ++k) c[k] = cell_coord(r[k], ch.inv_h[l], n);
      group_harmonics<GS, PM, 0, false>(lane, tb, tb.rec, (r[0] - (c[0] + 0.5) * h) / h,
                                                   (r[1] - (c[1] + 0.5) * h) / h,
                                                   (r[2] - (c[2] + 0.5) * h) / h, 1.0, buf);
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      const double *src = ch.Ld + ch.ld_off[l] + (size_t)lin3(n, c[0], c[1], c[2]) * Cs;
      double acc = 0.0;
      for (int s = lane; s < C; s += GS) acc += tb.wl2p[s] * src[s] * buf[s];
      phi += group_sum<GS>(acc) / h;
      __builtin_amdgcn_wave_barrier();
    }
    const int n = 1 << (ch.L - 1);
    int c[3];
    for (int k = 0; k < 3; ++k) c[k] = cell_coord(r[k], ch.inv_h[ch.L], n);
    double dn = 0.0;
    for (int e = lane; e < 27; e += GS) {
      int b[3] = {c[0] + e % 3 - 1, c[1] + (e / 3) % 3 - 1, c[2] + e / 9 - 1};
      int s = lin3(n, imod(b[0], n), imod(b[1], n), imod(b[2], n));
      double sh[3] = {ifloordiv(b[0], n) * a, ifloordiv(b[1], n) * a, ifloordiv(b[2], n) * a};
      bool zero = ifloordiv(b[0], n) == 0 && ifloordiv(b[1], n) == 0 && ifloordiv(b[2], n) == 0;
      int cnt = (ch.free_space && !zero) ? 0 : ch.bin_cnt[s];  // free space: no images
      for (int j = 0; j < cnt; ++j) {
        if (zero && ch.bin_id[(size_t)s * ch.B + j] == i) continue;
        double4 pj = ch.bin_p[(size_t)s * ch.B + j];
        double dx = r[0] - (pj.x + sh[0]), dy = r[1] - (pj.y + sh[1]), dz = r[2] - (pj.z + sh[2]);
        dn += pj.w / sqrt(dx * dx + dy * dy + dz * dz);
      }
    }
    phi += group_sum<GS>(dn);
    if (lane == 0) contrib = 0.5 * ch.pq[i] * phi;
  }
  double v = wg_sum<WG_SETUP>(contrib, red);
  if (threadIdx.x == 0) ch.red[blockIdx.x] = v;
}

// total energy: the block partials of k_energy in order, the far lattice
// 1/2 E.H (real weighted form, scaled by 1/a) and the tin-foil term
// -(2 pi / 3V) |D|^2 (Sec. 3.4). The result goes to scratch[8]; mode 1 also
// sets the running energy, mode 2 both the running and the setup energy.
template <int GS>
__global__ void k_energy_final(const Chain *chains, Tabs tb, int mode) {
#pragma clang fp contract(off)
  const Chain &ch = chains[blockIdx.y];
  if (threadIdx.x != 0) return;
  constexpr int NG = WG_SETUP / GS;
  const int nb = (ch.N + NG - 1) / NG;
  double u = 0.0;
  for (int b = 0; b < nb; ++b) u += ch.red[b];
  if (!ch.free_space) {  // far lattice and tin-foil terms (Sec. 3.4)
    double eh = 0.0;
    for (int s = 0; s < tb.C; ++s) eh += tb.wdot[s] * ch.K[s] * ch.H[s];
    const double a = ch.a;
    u += 0.5 * eh / a;
    const double d2 = ch.dip[0] * ch.dip[0] + ch.dip[1] * ch.dip[1] + ch.dip[2] * ch.dip[2];
    u += -2.0 * M_PI / (3.0 * a * a * a) * d2;
  }
  ch.scratch[8] = u;
  if (mode >= 1) ch.U[0] = u;
  if (mode >= 2) ch.U[1] = u;
}

}  // namespace fmmdev
