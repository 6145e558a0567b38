// setup_kernels.hpp -- the O(N) initialisation of the expansions (Sec. 3.2,
// FMM-pass variant without L2L, and Sec. 3.4 periodic moments): wrap and bin
// the charges, P2M on the leaves, M2M upwards, M2L over the interaction
// lists on levels 2..L, the lattice term, and the total energy.
#pragma once

#include "device_common.hpp"
#include "mc_step.hpp"

namespace fmmdev {

__global__ void k_fill_i32(int *p, int v, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double *p, double v, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// wrap positions, locate leaf cells, count bin occupancy
__global__ void k_stage(Chain ch) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ch.N) return;
  double x = wrap_coord(ch.stage[3 * i + 0], ch.a);
  double y = wrap_coord(ch.stage[3 * i + 1], ch.a);
  double z = wrap_coord(ch.stage[3 * i + 2], ch.a);
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
__global__ void k_bin_finalize(Chain ch, int nleaf) {
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
// leaf size: M^_n^m = sum q (|s|/h)^n Y_n^{-m}
template <int GS, int PM>
__global__ void k_p2m_leaf(Chain ch, Tabs tb, int nleaf) {
  constexpr int NG = WG_SETUP / GS;
  extern __shared__ double lds[];
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
  for (int j = 0; j < cnt; ++j) {
    double4 pj = ch.bin_p[(size_t)c * ch.B + j];
    group_harmonics<GS, PM, 1, true>(lane, tb, tb.rec, (pj.x - (cx + 0.5) * h) / h,
                                                (pj.y - (cy + 0.5) * h) / h, (pj.z - (cz + 0.5) * h) / h,
                                                pj.w, buf);
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  double *dst = ch.Mp + ch.mp_off[ch.L] + (size_t)c * Cs;
  for (int s = lane; s < Cs; s += GS) dst[s] = buf[s];
}

// M2M from level l+1 to level l (one workgroup per parent cell)
__global__ void k_m2m(Chain ch, Tabs tb, int l) {
  const int n = 1 << (l - 1), nc = 2 * n, C = tb.C, Cs = tb.Cs;
  int pc = blockIdx.x;
  int px = pc % n, py = (pc / n) % n, pz = pc / (n * n);
  const double *child = ch.Mp + ch.mp_off[l + 1];
  double *dst = ch.Mp + ch.mp_off[l] + (size_t)pc * Cs;
  for (int j = threadIdx.x; j < Cs; j += WG_SETUP) {
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

// M2L on level l: for each target cell a (octant oc), L^_a = sum over the 189
// offsets o of IL(oc) of T_o M^_{(a+o) mod n}; a batched GEMM over the target
// cells of one octant, tiled 64 (outputs) x 64 (cells) x 16 (inputs).
constexpr int M2L_NT = 256;  // threads of the M2L tile kernel (16 x 16, 4 x 4 outputs each)

__global__ void __launch_bounds__(M2L_NT) k_m2l_f64(Chain ch, Tabs tb, int l) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  __shared__ int src[64];
  const int n = 1 << (l - 1), half = n >> 1 ? n >> 1 : 1;
  const int C = tb.C, Cs = tb.Cs;
  const int oc = blockIdx.z, j0 = blockIdx.y * 64, p0 = blockIdx.x * 64;
  const int ntgt = half * half * half;
  const int t = threadIdx.x, tj = t % 16, tc = t / 16;
  const int ox = oc & 1, oy = (oc >> 1) & 1, oz = (oc >> 2) & 1;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[i][k] = 0.0;
  const double *M = ch.Mp + ch.mp_off[l];
  for (int k189 = 0; k189 < 189; ++k189) {
    const int8_t *o = tb.il_off + (oc * 189 + k189) * 3;
    const double *op = tb.m2l + (size_t)tb.il_id[oc * 189 + k189] * C * Cs;
    __syncthreads();
    if (t < 64) {
      int pl = p0 + t;
      int s = -1;
      if (pl < ntgt) {
        int Px = pl % half, Py = (pl / half) % half, Pz = pl / (half * half);
        int ax = 2 * Px + ox + o[0], ay = 2 * Py + oy + o[1], az = 2 * Pz + oz + o[2];
        s = lin3(n, imod(ax, n), imod(ay, n), imod(az, n));
      }
      src[t] = s;
    }
    __syncthreads();
    for (int k0 = 0; k0 < C; k0 += 16) {
      for (int e = t; e < 16 * 64; e += M2L_NT) {
        int kk = e / 64, jj = e % 64;
        int k = k0 + kk, j = j0 + jj;
        As[kk][jj] = (k < C && j < C) ? op[(size_t)k * Cs + j] : 0.0;
        int cc = e / 16, k2 = e % 16;
        int s = src[cc];
        Bs[k2][cc] = (s >= 0 && k0 + k2 < C) ? M[(size_t)s * Cs + k0 + k2] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        double av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = As[kk][tj + 16 * i];
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[i] = Bs[kk][tc + 16 * i];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[i][k] += av[i] * bv[k];
      }
      __syncthreads();
    }
  }
  double *Ld = ch.Ld + ch.ld_off[l];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int pl = p0 + tc + 16 * k;
    if (pl >= ntgt) continue;
    int Px = pl % half, Py = (pl / half) % half, Pz = pl / (half * half);
    int cell = lin3(n, 2 * Px + ox, 2 * Py + oy, 2 * Pz + oz);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int j = j0 + tj + 16 * i;
      if (j < C) Ld[(size_t)cell * Cs + j] = acc[i][k];
    }
  }
}

// K = level-1 multipole (about the box centre, scaled by a); H = R(K);
// dipole D = sum q r (one workgroup)
__global__ void k_lattice_init(Chain ch, Tabs tb) {
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
// 1/2 q_i phi_i written to ch.red[block]
template <int GS, int PM>
__global__ void k_energy(Chain ch, Tabs tb) {
  constexpr int NG = WG_SETUP / GS;
  extern __shared__ double lds[];
  __shared__ double red[WG_SETUP];
  const int g = threadIdx.x / GS, lane = threadIdx.x % GS, Cs = tb.Cs, C = tb.C;
  double *buf = lds + (size_t)g * Cs;
  int i = blockIdx.x * NG + g;
  double contrib = 0.0;
  if (i < ch.N) {
    const double a = ch.a;
    double r[3] = {ch.px[i], ch.py[i], ch.pz[i]};
    double phi = 0.0;
    for (int l = 2; l <= ch.L; ++l) {
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
      int cnt = ch.bin_cnt[s];
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

}  // namespace fmmdev
