// fmm_mc.hip -- host side and C ABI of the MI355X library for Metropolis-
// Hastings Monte Carlo of point charges with the multilevel local-expansion
// method (Saunders, Grant & Mueller, arXiv:2006.16622). See include/fmm_mc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/fmm_mc.h"
#include "device_common.hpp"
#include "host_ops.hpp"
#include "mc_step.hpp"
#include "run_kernels.hpp"
#include "setup_kernels.hpp"

using namespace fmmdev;

namespace {

constexpr int PMAX = 24;
constexpr int LEVELS_MAX = 7;

int pad_cs(int C) { return (C + 15) / 16 * 16; }
int group_size(int p) { return p + 1 <= 16 ? 16 : 32; }

// Kernel variants: (lanes per group, largest degree of the unrolled
// harmonic recurrence); the smallest that holds p is used.
int variant_of(int p) { return p <= 8 ? 0 : p <= 12 ? 1 : p <= 15 ? 2 : 3; }

template <typename F>
void with_variant(int v, F &&f) {
  using I16 = std::integral_constant<int, 16>;
  using I32 = std::integral_constant<int, 32>;
  switch (v) {
    case 0: f(I16{}, std::integral_constant<int, 8>{}); break;
    case 1: f(I16{}, std::integral_constant<int, 12>{}); break;
    case 2: f(I16{}, std::integral_constant<int, 15>{}); break;
    default: f(I32{}, std::integral_constant<int, 24>{}); break;
  }
}

template <class T>
struct TypeTag {
  using type = T;
};

// run-kernel variants: the lane-group variant of p and the evaluation type
// (FP32 in the mixed-precision mode)
template <typename F>
void with_run_variant(int p, bool mixed, F &&f) {
  with_variant(variant_of(p), [&](auto gs, auto pm) {
    if (mixed)
      f(gs, pm, TypeTag<float>{});
    else
      f(gs, pm, TypeTag<double>{});
  });
}

struct DevTables {
  int device = -1, p = -1;
  Tabs tabs{};
  std::vector<void *> allocs;
};

std::mutex g_mu;
std::vector<DevTables *> g_tables;

// choices of the autotuner, per (device, p, depth, precision)
struct TuneEntry {
  int device, p, levels;
  uint32_t mixed;
  int m2l_rows, helpers;
};
std::vector<TuneEntry> g_tune;

#define HIPCHK(x)                                  \
  do {                                             \
    hipError_t e_ = (x);                           \
    if (e_ != hipSuccess) return FMM_MC_EDEVICE;   \
  } while (0)

template <typename T>
int upload(DevTables *dt, const std::vector<T> &v, const T **out) {
  void *p = nullptr;
  size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
  HIPCHK(hipMalloc(&p, bytes));
  dt->allocs.push_back(p);
  if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = (const T *)p;
  return 0;
}

// Build the constant tables of degree p on the current device.
int build_tables(int p, DevTables **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  for (auto *t : g_tables)
    if (t->device == dev && t->p == p) {
      *out = t;
      return 0;
    }
  auto *dt = new DevTables();
  dt->device = dev;
  dt->p = p;
  const int C = (p + 1) * (p + 1), Cs = pad_cs(C);
  Tabs &tb = dt->tabs;
  tb.p = p;
  tb.C = C;
  tb.Cs = Cs;
  // recurrence constants: A(n,m) = (2n-1)/sqrt(n^2-m^2), B(n,m) =
  // sqrt(((n-1)^2-m^2)/(n^2-m^2)) at slot(n,m)
  std::vector<double> rec(3 * Cs, 0.0), wl2p(Cs, 0.0), wdot(Cs, 0.0), sgnc(Cs, 0.0);
  for (int n = 0; n <= p; ++n)
    for (int m = 0; m < n; ++m) {
      int s = fmmhost::slot(n, m);
      rec[s] = (2.0 * n - 1.0) / std::sqrt(double(n * n - m * m));
      rec[Cs + s] = std::sqrt(double((n - 1) * (n - 1) - m * m) / double(n * n - m * m));
    }
  // c_m = prod_{i<=m} sqrt((2i-1)/(2i)): T_m^m = c_m (x + i y)^m
  rec[2 * Cs] = 1.0;
  for (int m = 1; m <= p; ++m) rec[2 * Cs + m] = rec[2 * Cs + m - 1] * std::sqrt((2.0 * m - 1.0) / (2.0 * m));
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) {
      int s = fmmhost::slot(n, m);
      wl2p[s] = m == 0 ? 1.0 : (m > 0 ? 2.0 : -2.0);
      wdot[s] = m == 0 ? 1.0 : 2.0;
      sgnc[s] = m < 0 ? -1.0 : 1.0;
    }
  fmmhost::ILTables il = fmmhost::build_il();
  // level-independent M2L operators of the 316 distinct offsets
  std::vector<double> m2l((size_t)316 * C * Cs, 0.0), tmp((size_t)C * C);
  std::vector<float> m2l32((size_t)316 * C * Cs, 0.0f);
  for (int id = 0; id < 316; ++id) {
    int o[3] = {il.distinct[3 * id], il.distinct[3 * id + 1], il.distinct[3 * id + 2]};
    fmmhost::m2l_operator(p, o, tmp.data());
    for (int s = 0; s < C; ++s)
      for (int j = 0; j < C; ++j) {
        double v = tmp[(size_t)s * C + j];
        m2l[((size_t)id * C + s) * Cs + j] = v;
        m2l32[((size_t)id * C + s) * Cs + j] = (float)v;
      }
  }
  std::vector<double> m2m((size_t)8 * C * Cs, 0.0);
  for (int oc = 0; oc < 8; ++oc) {
    fmmhost::m2m_operator(p, oc, tmp.data());
    for (int s = 0; s < C; ++s)
      for (int j = 0; j < C; ++j) m2m[((size_t)oc * C + s) * Cs + j] = tmp[(size_t)s * C + j];
  }
  std::vector<double> lat((size_t)C * C);
  fmmhost::lattice_operator(p, lat.data());
  // ELL layout (column-major by row) of the sparse lattice operator, padded
  // with zero entries (column 0) to the width the kernel variant unrolls
  int W = 1;
  for (int j = 0; j < C; ++j) {
    int nz = 0;
    for (int s = 0; s < C; ++s) nz += lat[(size_t)j * C + s] != 0.0;
    W = std::max(W, nz);
  }
  // (the variants with groups of 16 lanes, whose whole-GPU proposal unrolls it)
  const int pmv[3] = {8, 12, 15};
  if (variant_of(p) < 3) W = std::max(W, ell_width(pmv[variant_of(p)]));
  std::vector<int> ecol((size_t)W * Cs, 0);
  std::vector<double> eval((size_t)W * Cs, 0.0);
  for (int j = 0; j < C; ++j) {
    int w = 0;
    for (int s = 0; s < C; ++s) {
      double v = lat[(size_t)j * C + s];
      if (v != 0.0) {
        ecol[(size_t)w * Cs + j] = s;
        eval[(size_t)w * Cs + j] = v;
        ++w;
      }
    }
  }
  tb.lat_w = W;
  tb.lat_lds = (size_t)W * Cs * 12 <= 48 * 1024 ? 1 : 0;
  int rc = 0;
  rc |= upload(dt, rec, &tb.rec);
  rc |= upload(dt, wl2p, &tb.wl2p);
  rc |= upload(dt, wdot, &tb.wdot);
  rc |= upload(dt, sgnc, &tb.sgnc);
  rc |= upload(dt, il.off, &tb.il_off);
  rc |= upload(dt, il.off_id, &tb.il_id);
  rc |= upload(dt, m2l, &tb.m2l);
  rc |= upload(dt, m2l32, &tb.m2l32);
  rc |= upload(dt, m2m, &tb.m2m);
  rc |= upload(dt, ecol, &tb.lat_col);
  rc |= upload(dt, eval, &tb.lat_val);
  tb.self_const = 6.0 + 8.0 / std::sqrt(3.0) + 12.0 / std::sqrt(2.0);
  if (rc) {
    for (void *a : dt->allocs) (void)hipFree(a);
    delete dt;
    return FMM_MC_EDEVICE;
  }
  g_tables.push_back(dt);
  *out = dt;
  return 0;
}

// ------------------------------------------------------------------ layout
struct Layout {
  size_t off[32];
  size_t total;
  int B;
};

enum {
  O_PX, O_PY, O_PZ, O_PQ, O_LEAF, O_SLOT, O_BCNT, O_BID, O_BP, O_LD, O_MP, O_K, O_H,
  O_DIP, O_U, O_STATUS, O_SCRATCH, O_MBOX, O_SYNC, O_RED, O_PART, O_STAGE, O_STATS, O_CHAIN, O_TILES, O_DSCR,
  O_END
};

int bin_capacity(int64_t n, int levels) {
  double nleaf = std::pow(8.0, levels);
  double mean = double(n) / nleaf;
  int want = (int)std::ceil(3.0 * mean + 16.0);
  int B = 16;
  while (B < want) B *= 2;
  return B;
}

// M2L tiles of one chain: per octant, its targets on levels 2..levels+1
// ((8^levels - 1)/7 of them) in runs of M2L_TT
long long m2l_octant_targets(int levels) { return ((1LL << (3 * levels)) - 1) / 7; }
int m2l_tiles(int levels) { return 8 * (int)((m2l_octant_targets(levels) + M2L_TT - 1) / M2L_TT); }

void append_m2l_tiles(std::vector<int4> &out, int chain, int levels) {
  const long long T = m2l_octant_targets(levels);
  for (int oc = 0; oc < 8; ++oc)
    for (long long f = 0; f < T; f += M2L_TT)
      out.push_back(make_int4(chain, oc, (int)f, (int)std::min<long long>(M2L_TT, T - f)));
}

// chunk rows the direct P2L setup needs: the largest level below the leaves
long long direct_rows(int levels) {
  const int L = levels + 1;
  long long rows = 0;
  for (int l = 2; l < L; ++l)
    if (p2l_chunks(L, l) > 1) rows = std::max(rows, (1LL << (3 * (l - 1))) * p2l_chunks(L, l));
  return rows;
}

void make_layout(int64_t n, int levels, int p, uint32_t flags, Layout &ly) {
  const int C = (p + 1) * (p + 1), Cs = pad_cs(C), L = levels + 1;
  const int64_t nleaf = 1LL << (3 * levels);
  int64_t ncell_ld = 0, ncell_mp = 0;
  for (int l = 1; l <= L; ++l) {
    int64_t c = 1LL << (3 * (l - 1));
    ncell_mp += c;
    if (l >= 2) ncell_ld += c;
  }
  ly.B = bin_capacity(n, levels);
  size_t sz[O_END];
  sz[O_PX] = sz[O_PY] = sz[O_PZ] = sz[O_PQ] = 8 * n;
  sz[O_LEAF] = sz[O_SLOT] = 4 * n;
  sz[O_BCNT] = 4 * nleaf;
  sz[O_BID] = 4 * nleaf * ly.B;
  sz[O_BP] = 32 * nleaf * ly.B;
  sz[O_LD] = 8 * ncell_ld * Cs;
  sz[O_MP] = 8 * ncell_mp * Cs;
  sz[O_K] = sz[O_H] = 8 * Cs;
  sz[O_DIP] = 8 * 4;
  sz[O_U] = 8 * 4;
  sz[O_STATUS] = 4 * 8;
  sz[O_SCRATCH] = 8 * 64;
  sz[O_MBOX] = 8 * 64;
  sz[O_SYNC] = 4 * 512;
  const int NG = WG_SETUP / group_size(p);
  sz[O_RED] = 8 * ((n + NG - 1) / NG + 64);
  sz[O_PART] = 8 * 512;
  sz[O_STAGE] = 8 * 4 * n;
  sz[O_STATS] = 8 * 64;
  sz[O_CHAIN] = sizeof(Chain);
  sz[O_TILES] = sizeof(int4) * (size_t)m2l_tiles(levels);
  sz[O_DSCR] = (flags & FMM_MC_DIRECT_SETUP) ? 8 * (size_t)direct_rows(levels) * Cs : 0;
  size_t o = 0;
  for (int i = 0; i < O_END; ++i) {
    ly.off[i] = o;
    o += (sz[i] + 255) / 256 * 256;
  }
  ly.total = o;
}

}  // namespace

struct fmm_mc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t n = 0;
  int levels = 0, p = 0, C = 0, Cs = 0, GS = 16;
  uint32_t flags = 0;
  double box = 1.0;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  Layout ly{};
  Chain ch{};
  Chain *d_chain = nullptr;
  DevTables *tables = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
  int4 *d_tiles = nullptr;            // this chain's M2L tile list (workspace)
  int ntiles = 0;
  hipStream_t cap_stream = nullptr;   // private stream for graph capture
  hipGraph_t graph = nullptr;         // captured re-setup
  hipGraphExec_t gexec = nullptr;
  int m2l_rows = 0;                   // tuned M2L output rows per workgroup (0: 96)
  int helpers = 0;                    // tuned helper workgroups of the whole-GPU run (0: all blocks)
  double last_ms[4] = {0, 0, 0, 0};
  bool ready = false;
  // a volume move can be undone while the staging area still holds the
  // positions before it (until any other call changes the state)
  bool undo_ok = false;
  double box_prev = 1.0;
  // buffers of the run entry points, allocated at setup (host_stats) or on
  // the first run of many chains led by this handle (grown when a run has
  // more chains than any before): launch arguments and per-chain results
  double *host_stats = nullptr;       // pinned, RUN_NSTAT doubles: results of a one-chain run
  char *run_dev = nullptr;            // device: descriptors, first steps, ids, step sizes, results
  size_t run_dev_cap = 0;
  char *run_host = nullptr;           // pinned staging of the same
  size_t run_host_cap = 0;
};

namespace {

// dynamic LDS of the Monte Carlo kernels with workgroups of nt threads
size_t smem_bytes(int GS, const Tabs &tb, int nt) {
  int w = tb.lat_lds ? tb.lat_w : 0;
  if (nt == WG_BATCH) return GS == 16 ? Lds<16, WG_BATCH>::bytes(tb.Cs, w) : Lds<32, WG_BATCH>::bytes(tb.Cs, w);
  return GS == 16 ? Lds<16, WG_SINGLE>::bytes(tb.Cs, w) : Lds<32, WG_SINGLE>::bytes(tb.Cs, w);
}

int grid_for(long long n, int bs) { return (int)((n + bs - 1) / bs); }

// One setup pass over a batch of chains of the same degree (a single chain
// is a batch of one): optional restage from the device positions, clear,
// wrap and bin, P2M, M2M, M2L (all levels and chains in one launch), the
// lattice moments and the total energy. Only kernels: the sequence can be
// captured into a graph. e1/e2, if given, bracket the M2L launch.
struct SetupLaunch {
  hipStream_t st = nullptr;
  const Chain *chains = nullptr;  // device array
  int nchains = 0;
  long long max_n = 0;
  int max_levels = 0;
  const int4 *tiles = nullptr;
  int ntiles = 0;
  int p = 0, GS = 16, C = 0, Cs = 0;
  const Tabs *tb = nullptr;
  bool restage = false;
  bool fp32_m2l = false;
  bool multipole = false;  // the multipole-based variant: no M2L
  bool direct = false;     // direct P2L (Alg. L.3) in place of M2L
  int m2l_rows = 0;  // 96 or 192 (0: 96)
  int energy_mode = 2;
  hipEvent_t e1 = nullptr, e2 = nullptr;
};

void launch_m2l(const SetupLaunch &S) {
  const Tabs &tb = *S.tb;
  const bool narrow = S.m2l_rows ? S.m2l_rows == 96 : true;
  const int TO = narrow ? 96 : 192;
  dim3 mg(S.ntiles, (S.C + TO - 1) / TO);
  hipStream_t st = S.st;
  if (S.fp32_m2l) {
    if (narrow)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_m2l<float, 96>), mg, dim3(M2L_NT), 0, st, S.chains, tb, S.tiles, tb.m2l32);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_m2l<float, 192>), mg, dim3(M2L_NT), 0, st, S.chains, tb, S.tiles, tb.m2l32);
  } else {
    if (narrow)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_m2l<double, 96>), mg, dim3(M2L_NT), 0, st, S.chains, tb, S.tiles, tb.m2l);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_m2l<double, 192>), mg, dim3(M2L_NT), 0, st, S.chains, tb, S.tiles, tb.m2l);
  }
}

int enqueue_setup(const SetupLaunch &S) {
  const Tabs &tb = *S.tb;
  hipStream_t st = S.st;
  constexpr int NT = WG_SETUP;
  const int NG = NT / S.GS;
  const int nc = S.nchains;
  const long long max_nleaf = 1LL << (3 * S.max_levels);
  const size_t shm = (size_t)NG * S.Cs * sizeof(double);
  if (S.restage) hipLaunchKernelGGL(k_restage, dim3(grid_for(S.max_n, NT), nc), dim3(NT), 0, st, S.chains);
  hipLaunchKernelGGL(k_setup_clear, dim3(grid_for(max_nleaf, NT), nc), dim3(NT), 0, st, S.chains);
  hipLaunchKernelGGL(k_stage, dim3(grid_for(S.max_n, NT), nc), dim3(NT), 0, st, S.chains);
  hipLaunchKernelGGL(k_bin_finalize, dim3(grid_for(max_nleaf, NT), nc), dim3(NT), 0, st, S.chains);
  with_variant(variant_of(S.p), [&](auto gs, auto pm) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_p2m_leaf<decltype(gs)::value, decltype(pm)::value>),
                       dim3(grid_for(max_nleaf, NG), nc), dim3(NT), shm, st, S.chains, tb);
  });
  for (int l = S.max_levels; l >= 1; --l)
    hipLaunchKernelGGL(k_m2m, dim3(1 << (3 * (l - 1)), nc), dim3(256), 0, st, S.chains, tb, l);
  if (S.e1) HIPCHK(hipEventRecord(S.e1, st));
  if (S.direct) {
    for (int l = 2; l <= S.max_levels + 1; ++l) {
      const long long nt = 1LL << (3 * (l - 1));
      const int nch = p2l_chunks(S.max_levels + 1, l);  // the most chunks any chain of the batch has
      with_variant(variant_of(S.p), [&](auto gs, auto pm) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_p2l_direct<decltype(gs)::value, decltype(pm)::value>),
                           dim3((unsigned)(nt * nch), nc), dim3(NT), shm, st, S.chains, tb, l);
      });
      if (nch > 1) hipLaunchKernelGGL(k_p2l_reduce, dim3((unsigned)nt, nc), dim3(256), 0, st, S.chains, tb, l);
    }
  } else if (!S.multipole) {
    launch_m2l(S);
  }
  if (S.e2) HIPCHK(hipEventRecord(S.e2, st));
  hipLaunchKernelGGL(k_lattice_init, dim3(1, nc), dim3(NT), 0, st, S.chains, tb);
  with_variant(variant_of(S.p), [&](auto gs, auto pm) {
    if (S.multipole)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_energy<decltype(gs)::value, decltype(pm)::value, true>),
                         dim3(grid_for(S.max_n, NG), nc), dim3(NT), shm, st, S.chains, tb);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_energy<decltype(gs)::value, decltype(pm)::value>),
                         dim3(grid_for(S.max_n, NG), nc), dim3(NT), shm, st, S.chains, tb);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_energy_final<decltype(gs)::value>), dim3(1, nc), dim3(64), 0, st,
                       S.chains, tb, S.energy_mode);
  });
  HIPCHK(hipGetLastError());
  return 0;
}

SetupLaunch single_launch(fmm_mc_ctx *h) {
  SetupLaunch S;
  S.st = h->stream;
  S.chains = h->d_chain;
  S.nchains = 1;
  S.max_n = h->n;
  S.max_levels = h->levels;
  S.tiles = h->d_tiles;
  S.ntiles = h->ntiles;
  S.p = h->p;
  S.GS = h->GS;
  S.C = h->C;
  S.Cs = h->Cs;
  S.tb = &h->tables->tabs;
  S.fp32_m2l = (h->flags & FMM_MC_MIXED) != 0;
  S.multipole = (h->flags & FMM_MC_MULTIPOLE) != 0;
  S.direct = (h->flags & FMM_MC_DIRECT_SETUP) != 0;
  S.m2l_rows = h->m2l_rows;
  return S;
}

// status words of a chain after a setup: overflow of a leaf bin
int setup_status(fmm_mc_ctx *h) {
  int status[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(status, h->ch.status, sizeof(status), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return status[1] ? FMM_MC_EOVERFLOW : 0;
}

// a fresh evaluation of the total energy of the current state
int compute_energy(fmm_mc_ctx *h, double *U) {
  const Tabs &tb = h->tables->tabs;
  constexpr int NT = WG_SETUP;
  const int NG = NT / h->GS;
  const size_t shm = (size_t)NG * h->Cs * sizeof(double);
  const bool mp = (h->flags & FMM_MC_MULTIPOLE) != 0;
  with_variant(variant_of(h->p), [&](auto gs, auto pm) {
    if (mp)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_energy<decltype(gs)::value, decltype(pm)::value, true>),
                         dim3(grid_for(h->n, NG), 1), dim3(NT), shm, h->stream, h->d_chain, tb);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_energy<decltype(gs)::value, decltype(pm)::value>),
                         dim3(grid_for(h->n, NG), 1), dim3(NT), shm, h->stream, h->d_chain, tb);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_energy_final<decltype(gs)::value>), dim3(1, 1), dim3(64), 0, h->stream,
                       h->d_chain, tb, 0);
  });
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(U, h->ch.scratch + 8, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return 0;
}

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

bool in_box(const double *v, double a) {
  return v[0] >= 0.0 && v[0] < a && v[1] >= 0.0 && v[1] < a && v[2] >= 0.0 && v[2] < a;
}

}  // namespace

// Device and pinned host buffers of a run of many chains (one workgroup
// each), kept by the handle of the run's first chain: the chain
// descriptors, first steps and ids of a launch's slots, the step sizes of
// the run's chains and the per-slot results. Allocated on the first such
// run and grown only when a run has more chains than any before, so that
// repeated runs allocate nothing.
static constexpr size_t round256(size_t b) { return (b + 255) / 256 * 256; }
static constexpr size_t run_area_bytes(size_t n_chains) {
  return round256(sizeof(Chain) * n_chains) + round256(sizeof(int64_t) * n_chains) +
         round256(sizeof(int) * n_chains) + round256(sizeof(double) * n_chains) +
         round256(sizeof(double) * RUN_NSTAT * n_chains);
}
struct RunArea {
  size_t o_desc, o_first, o_id, o_step, o_stats, bytes;
  RunArea(int n_chains) {
    o_desc = 0;
    o_first = o_desc + round256(sizeof(Chain) * n_chains);
    o_id = o_first + round256(sizeof(int64_t) * n_chains);
    o_step = o_id + round256(sizeof(int) * n_chains);
    o_stats = o_step + round256(sizeof(double) * n_chains);
    bytes = o_stats + round256(sizeof(double) * RUN_NSTAT * n_chains);
  }
};

// ---- fixed memory of fmm_mc_run_noalloc (callers that cannot allocate).
// The argument and result block of a run of many chains lives in this
// array instead of the first handle's buffers. Each GPU holds its own copy
// of it for the life of the process; its address on a device is looked up
// once, at the first setup on that device, and only that address is used
// from the host. Every call on one GPU uses the same array (and the same
// host staging, under a lock), so calls that overlap on one GPU race.
static constexpr size_t NOALLOC_SCRATCH_BYTES = 1u << 20;
static_assert(run_area_bytes(FMM_MC_NOALLOC_MAX_CHAINS) <= NOALLOC_SCRATCH_BYTES, "scratch too small");
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

// host side: the device address of `scratch` per device, and one pinned
// staging block of the same layout plus the run's host bookkeeping
// (allocated at the first setup in the process, under g_mu)
static constexpr int MAX_DEVICES = 64;
static void *g_scratch_dev[MAX_DEVICES] = {};
static std::mutex g_noalloc_mu;  // held for the whole of a fmm_mc_run_noalloc call
static char *g_noalloc_host = nullptr;
static constexpr size_t noalloc_work_bytes(size_t n) {
  return sizeof(int64_t) * n + sizeof(double) * RUN_NSTAT * n + sizeof(double) * n + sizeof(int) * n;
}
static constexpr size_t NOALLOC_HOST_BYTES = NOALLOC_SCRATCH_BYTES + noalloc_work_bytes(FMM_MC_NOALLOC_MAX_CHAINS);

// at setup, with the chain's device current: look up the address of
// `scratch` on it, and allocate the host staging once per process.
// Failures are left for fmm_mc_run_noalloc to report.
static void noalloc_prepare(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_dev[dev] = ptr;
  }
  if (!g_noalloc_host && hipHostMalloc((void **)&g_noalloc_host, NOALLOC_HOST_BYTES, hipHostMallocDefault) != hipSuccess)
    g_noalloc_host = nullptr;
}

extern "C" {

int fmm_mc_workspace_bytes(int64_t n, int levels, int p, uint32_t flags, size_t *bytes) {
  if (!bytes || n < 2 || levels < 1 || levels > LEVELS_MAX || p < 0 || p > PMAX) return FMM_MC_EINVAL;
  Layout ly;
  make_layout(n, levels, p, flags, ly);
  *bytes = ly.total;
  return FMM_MC_OK;
}

// Validate the inputs, carve the workspace, upload the staged charges, the
// chain descriptor and its M2L tile list; the setup kernels are not run.
static int create_chain(fmm_mc_t *out, void *dev_ws, size_t ws_bytes, void *hip_stream, int64_t n,
                        const double *pos, const double *q, double box, int levels, int p, uint32_t flags) {
  if (!out || !dev_ws || !pos || !q) return FMM_MC_EINVAL;
  if (n < 2 || n > (int64_t)1 << 30 || levels < 1 || levels > LEVELS_MAX || p < 0 || p > PMAX)
    return FMM_MC_EINVAL;
  if (!(box > 0.0) || !std::isfinite(box)) return FMM_MC_EINVAL;
  if (((uintptr_t)dev_ws) % 256) return FMM_MC_EINVAL;
  if ((flags & ~(FMM_MC_MIXED | FMM_MC_MULTIPOLE | FMM_MC_DIRECT_SETUP | FMM_MC_FREE_SPACE)) ||
      ((flags & FMM_MC_MULTIPOLE) && (flags & (FMM_MC_MIXED | FMM_MC_DIRECT_SETUP))))
    return FMM_MC_EINVAL;
  double qs = 0.0, qa = 0.0;
  const bool free_space = (flags & FMM_MC_FREE_SPACE) != 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!finite3(pos + 3 * i) || !std::isfinite(q[i])) return FMM_MC_EINVAL;
    if (free_space && !in_box(pos + 3 * i, box)) return FMM_MC_EINVAL;
    qs += q[i];
    qa += std::fabs(q[i]);
  }
  if (std::fabs(qs) > 1e-12 * qa) return FMM_MC_ENONNEUTRAL;
  Layout ly;
  make_layout(n, levels, p, flags, ly);
  if (ws_bytes < ly.total) return FMM_MC_ENOMEM;
  auto *h = new (std::nothrow) fmm_mc_ctx();
  if (!h) return FMM_MC_ENOMEM;
  int rc = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    rc = build_tables(p, &h->tables);
  }
  if (rc) {
    delete h;
    return rc;
  }
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return FMM_MC_EDEVICE;
  }
  noalloc_prepare(h->device);
  h->stream = (hipStream_t)hip_stream;
  h->n = n;
  h->levels = levels;
  h->p = p;
  h->C = (p + 1) * (p + 1);
  h->Cs = pad_cs(h->C);
  h->GS = group_size(p);
  h->flags = flags;
  h->box = box;
  h->ws = (char *)dev_ws;
  h->ws_bytes = ws_bytes;
  h->ly = ly;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &e : g_tune)
      if (e.device == h->device && e.p == p && e.levels == levels && e.mixed == flags) {
        h->m2l_rows = e.m2l_rows;
        h->helpers = e.helpers;
      }
  }
  Chain &ch = h->ch;
  char *w = h->ws;
  ch.N = (int)n;
  ch.d = levels;
  ch.L = levels + 1;
  ch.B = ly.B;
  ch.mixed = (flags & FMM_MC_MIXED) ? 1 : 0;
  ch.free_space = (flags & FMM_MC_FREE_SPACE) ? 1 : 0;
  ch.a = box;
  ch.scale = 1.0;
  for (int l = 0; l <= MAXL + 1; ++l) ch.inv_h[l] = double(1LL << (l > 0 ? l - 1 : 0)) / box;
  ch.px = (double *)(w + ly.off[O_PX]);
  ch.py = (double *)(w + ly.off[O_PY]);
  ch.pz = (double *)(w + ly.off[O_PZ]);
  ch.pq = (double *)(w + ly.off[O_PQ]);
  ch.leaf_of = (int *)(w + ly.off[O_LEAF]);
  ch.slot_of = (int *)(w + ly.off[O_SLOT]);
  ch.bin_cnt = (int *)(w + ly.off[O_BCNT]);
  ch.bin_id = (int *)(w + ly.off[O_BID]);
  ch.bin_p = (double4 *)(w + ly.off[O_BP]);
  ch.Ld = (double *)(w + ly.off[O_LD]);
  ch.Mp = (double *)(w + ly.off[O_MP]);
  long long o_ld = 0, o_mp = 0;
  for (int l = 0; l <= MAXL + 1; ++l) {
    ch.ld_off[l] = 0;
    ch.mp_off[l] = 0;
  }
  for (int l = 1; l <= ch.L; ++l) {
    long long c = 1LL << (3 * (l - 1));
    ch.mp_off[l] = o_mp;
    o_mp += c * h->Cs;
    if (l >= 2) {
      ch.ld_off[l] = o_ld;
      o_ld += c * h->Cs;
    }
  }
  ch.K = (double *)(w + ly.off[O_K]);
  ch.H = (double *)(w + ly.off[O_H]);
  ch.dip = (double *)(w + ly.off[O_DIP]);
  ch.U = (double *)(w + ly.off[O_U]);
  ch.status = (int *)(w + ly.off[O_STATUS]);
  ch.scratch = (double *)(w + ly.off[O_SCRATCH]);
  ch.mbox = (double *)(w + ly.off[O_MBOX]);
  ch.sync = (unsigned *)(w + ly.off[O_SYNC]);
  ch.red = (double *)(w + ly.off[O_RED]);
  ch.part = (double *)(w + ly.off[O_PART]);
  ch.dscr = (flags & FMM_MC_DIRECT_SETUP) ? (double *)(w + ly.off[O_DSCR]) : nullptr;
  ch.stage = (double *)(w + ly.off[O_STAGE]);
  h->d_chain = (Chain *)(w + ly.off[O_CHAIN]);
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess ||
      hipEventCreate(&h->ev2) != hipSuccess ||
      hipHostMalloc((void **)&h->host_stats, sizeof(double) * RUN_NSTAT, hipHostMallocDefault) != hipSuccess) {
    fmm_mc_destroy(h);
    return FMM_MC_EDEVICE;
  }
  std::vector<double> stage(4 * n);
  std::memcpy(stage.data(), pos, sizeof(double) * 3 * n);
  std::memcpy(stage.data() + 3 * n, q, sizeof(double) * n);
  if (hipMemcpyAsync(ch.stage, stage.data(), sizeof(double) * 4 * n, hipMemcpyHostToDevice, h->stream) !=
          hipSuccess ||
      hipMemcpyAsync(h->d_chain, &ch, sizeof(Chain), hipMemcpyHostToDevice, h->stream) != hipSuccess) {
    fmm_mc_destroy(h);
    return FMM_MC_EDEVICE;
  }
  std::vector<int4> tiles;
  append_m2l_tiles(tiles, 0, levels);
  h->d_tiles = (int4 *)(w + ly.off[O_TILES]);
  h->ntiles = (int)tiles.size();
  if (hipMemcpyAsync(h->d_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, h->stream) !=
          hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    fmm_mc_destroy(h);
    return FMM_MC_EDEVICE;
  }
  *out = h;
  return FMM_MC_OK;
}

int fmm_mc_setup(fmm_mc_t *out, void *dev_ws, size_t ws_bytes, void *hip_stream, int64_t n,
                 const double *pos, const double *q, double box, int levels, int p, uint32_t flags) {
  fmm_mc_t h = nullptr;
  int rc = create_chain(&h, dev_ws, ws_bytes, hip_stream, n, pos, q, box, levels, p, flags);
  if (rc) return rc;
  SetupLaunch S = single_launch(h);
  S.energy_mode = 2;
  S.e1 = h->ev1;
  S.e2 = h->ev2;
  rc = enqueue_setup(S);
  if (!rc) rc = setup_status(h);
  if (!rc) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, h->ev1, h->ev2) == hipSuccess) h->last_ms[1] = ms;
  }
  if (rc) {
    fmm_mc_destroy(h);
    return rc;
  }
  h->ready = true;
  *out = h;
  return FMM_MC_OK;
}

int fmm_mc_setup_batch(fmm_mc_t *out, int n_chains, void *const *dev_ws, const size_t *ws_bytes,
                       void *hip_stream, const int64_t *n, const double *const *pos, const double *const *q,
                       const double *box, const int *levels, int p, uint32_t flags) {
  if (!out || n_chains < 1 || !dev_ws || !ws_bytes || !n || !pos || !q || !box || !levels) return FMM_MC_EINVAL;
  std::vector<fmm_mc_t> hs(n_chains, nullptr);
  auto fail = [&](int rc) {
    for (auto *h : hs)
      if (h) fmm_mc_destroy(h);
    return rc;
  };
  std::vector<Chain> descs(n_chains);
  std::vector<int4> tiles;
  long long max_n = 0;
  int max_levels = 0;
  for (int c = 0; c < n_chains; ++c) {
    int rc = create_chain(&hs[c], dev_ws[c], ws_bytes[c], hip_stream, n[c], pos[c], q[c], box[c], levels[c], p,
                          flags);
    if (rc) return fail(rc);
    descs[c] = hs[c]->ch;
    append_m2l_tiles(tiles, c, levels[c]);
    max_n = std::max<long long>(max_n, n[c]);
    max_levels = std::max(max_levels, levels[c]);
  }
  fmm_mc_t h0 = hs[0];
  hipStream_t st = h0->stream;
  Chain *d_descs = nullptr;
  int4 *d_tiles = nullptr;
  if (hipMallocAsync((void **)&d_descs, sizeof(Chain) * n_chains, st) != hipSuccess ||
      hipMallocAsync((void **)&d_tiles, sizeof(int4) * tiles.size(), st) != hipSuccess)
    return fail(FMM_MC_EDEVICE);
  int rc = 0;
  if (hipMemcpyAsync(d_descs, descs.data(), sizeof(Chain) * n_chains, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(d_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, st) != hipSuccess)
    rc = FMM_MC_EDEVICE;
  if (!rc) {
    SetupLaunch S = single_launch(h0);
    S.chains = d_descs;
    S.nchains = n_chains;
    S.max_n = max_n;
    S.max_levels = max_levels;
    S.tiles = d_tiles;
    S.ntiles = (int)tiles.size();
    S.energy_mode = 2;
    S.e1 = h0->ev1;
    S.e2 = h0->ev2;
    rc = enqueue_setup(S);
  }
  (void)hipFreeAsync(d_descs, st);
  (void)hipFreeAsync(d_tiles, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = FMM_MC_EDEVICE;
  for (int c = 0; c < n_chains && !rc; ++c) rc = setup_status(hs[c]);
  if (rc) return fail(rc);
  float ms = 0;
  if (hipEventElapsedTime(&ms, h0->ev1, h0->ev2) == hipSuccess) h0->last_ms[1] = ms;
  for (int c = 0; c < n_chains; ++c) {
    hs[c]->ready = true;
    out[c] = hs[c];
  }
  return FMM_MC_OK;
}

// Re-setup from the device-resident positions: the setup pass, captured
// once into a graph on a private stream and replayed on the chain's stream.
// The running energy becomes the fresh total energy; the setup energy stays.
int fmm_mc_resetup(fmm_mc_t h) {
  if (!h || !h->ready) return FMM_MC_ESTATE;
  h->undo_ok = false;
  if (!h->gexec) {
    if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    SetupLaunch S = single_launch(h);
    S.st = h->cap_stream;
    S.restage = true;
    S.energy_mode = 1;
    S.fp32_m2l = false;  // the re-setup is FP64 in every mode
    HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_setup(S);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (rc || e != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return rc ? rc : FMM_MC_EDEVICE;
    }
    h->graph = g;
    if (hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0) != hipSuccess) {
      h->gexec = nullptr;
      return FMM_MC_EDEVICE;
    }
  }
  HIPCHK(hipGraphLaunch(h->gexec, h->stream));
  return setup_status(h);
}

// the box side of a chain, in its host and device descriptors
static int set_box(fmm_mc_t h, double box, double scale) {
  h->box = box;
  h->ch.a = box;
  h->ch.scale = scale;
  for (int l = 0; l <= MAXL + 1; ++l) h->ch.inv_h[l] = double(1LL << (l > 0 ? l - 1 : 0)) / box;
  HIPCHK(hipMemcpyAsync(h->d_chain, &h->ch, sizeof(Chain), hipMemcpyHostToDevice, h->stream));
  return 0;
}

// the setup pass from the staging area as it is (no restage): positions
// times ch.scale, wrapped into the current box
static int setup_from_stage(fmm_mc_t h) {
  SetupLaunch S = single_launch(h);
  S.restage = false;
  S.energy_mode = 2;
  S.fp32_m2l = false;  // FP64 in every mode, as every re-setup
  int rc = enqueue_setup(S);
  if (!rc) rc = setup_status(h);
  return rc;
}

int fmm_mc_rescale(fmm_mc_t h, double new_box, double *dE) {
  if (!h || !h->ready) return FMM_MC_ESTATE;
  if (!dE || !(new_box > 0.0) || !std::isfinite(new_box)) return FMM_MC_EINVAL;
  // a fresh setup of the current state (positions -> staging area ->
  // expansions) and its energy
  int rc = fmm_mc_resetup(h);
  if (rc) return rc;
  double U0 = 0.0, U1 = 0.0;
  rc = fmm_mc_running_energy(h, &U0);
  if (rc) return rc;
  // the scaled state, set up from the same staging area
  const double old_box = h->box;
  rc = set_box(h, new_box, new_box / old_box);
  if (!rc) rc = setup_from_stage(h);
  // later re-setups stage the (scaled) positions as they are
  if (!rc) rc = set_box(h, new_box, 1.0);
  if (!rc) rc = fmm_mc_running_energy(h, &U1);
  if (rc) return rc;
  *dE = U1 - U0;
  h->box_prev = old_box;
  h->undo_ok = true;
  return FMM_MC_OK;
}

int fmm_mc_rescale_undo(fmm_mc_t h) {
  if (!h || !h->ready || !h->undo_ok) return FMM_MC_ESTATE;
  h->undo_ok = false;
  // the staging area still holds the positions before the volume move
  int rc = set_box(h, h->box_prev, 1.0);
  if (!rc) rc = setup_from_stage(h);
  return rc;
}

int fmm_mc_propose(fmm_mc_t h, int64_t idx, const double *new_pos, double *dE) {
  if (!h || !h->ready) return FMM_MC_ESTATE;
  if (!new_pos || !dE || !finite3(new_pos)) return FMM_MC_EINVAL;
  if (idx < 0 || idx >= h->n) return FMM_MC_ERANGE;
  const Tabs &tb = h->tables->tabs;
  const size_t shm = smem_bytes(h->GS, h->tables->tabs, WG_SINGLE);
  if (h->flags & FMM_MC_MULTIPOLE)
    with_variant(variant_of(h->p), [&](auto gs, auto pm) {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_propose_one<decltype(gs)::value, decltype(pm)::value, double, true>),
                         dim3(1), dim3(WG_SINGLE), shm, h->stream, h->ch, tb, idx, new_pos[0], new_pos[1],
                         new_pos[2]);
    });
  else
    with_run_variant(h->p, h->flags & FMM_MC_MIXED, [&](auto gs, auto pm, auto rt) {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_propose_one<decltype(gs)::value, decltype(pm)::value,
                                                       typename decltype(rt)::type>), dim3(1),
                         dim3(WG_SINGLE), shm, h->stream, h->ch, tb, idx, new_pos[0], new_pos[1], new_pos[2]);
    });
  HIPCHK(hipGetLastError());
  double r[2];
  HIPCHK(hipMemcpyAsync(r, h->ch.scratch, sizeof(r), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  *dE = r[0];
  if (r[1] != 0.0) return FMM_MC_ESINGULAR;
  return FMM_MC_OK;
}

int fmm_mc_accept(fmm_mc_t h, int64_t idx, const double *new_pos, const double *dE_in, double *dE_out) {
  if (!h || !h->ready) return FMM_MC_ESTATE;
  h->undo_ok = false;
  if (!new_pos || !finite3(new_pos)) return FMM_MC_EINVAL;
  if ((h->flags & FMM_MC_FREE_SPACE) && !in_box(new_pos, h->box)) return FMM_MC_EINVAL;
  if (idx < 0 || idx >= h->n) return FMM_MC_ERANGE;
  double dE = 0.0;
  if (dE_in) {
    dE = *dE_in;
  } else {
    int rc = fmm_mc_propose(h, idx, new_pos, &dE);
    if (rc) return rc;
  }
  const Tabs &tb = h->tables->tabs;
  constexpr int NT = WG_SINGLE;
  const size_t shm = smem_bytes(h->GS, h->tables->tabs, NT);
  const int NG = NT / h->GS;
  const int nb = accept_blocks(h->ch.L, NG);
  if (h->flags & FMM_MC_MULTIPOLE)
    with_variant(variant_of(h->p), [&](auto gs, auto pm) {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_accept_book<decltype(gs)::value, decltype(pm)::value, true>), dim3(1),
                         dim3(NT), shm, h->stream, h->ch, tb, idx, new_pos[0], new_pos[1], new_pos[2], dE);
    });
  else
    with_run_variant(h->p, h->flags & FMM_MC_MIXED, [&](auto gs, auto pm, auto rt) {
      constexpr int G_ = decltype(gs)::value, P_ = decltype(pm)::value;
      using R_ = typename decltype(rt)::type;
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_accept_blocks<G_, P_, R_>), dim3(nb), dim3(NT), shm, h->stream, h->ch,
                         tb, idx, new_pos[0], new_pos[1], new_pos[2]);
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_accept_book<G_, P_>), dim3(1), dim3(NT), shm, h->stream, h->ch, tb, idx,
                         new_pos[0], new_pos[1], new_pos[2], dE);
    });
  HIPCHK(hipGetLastError());
  int status = 0;
  HIPCHK(hipMemcpyAsync(&status, h->ch.status, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (dE_out) *dE_out = dE;
  return status ? status : FMM_MC_OK;
}

static int ensure_run_area(fmm_mc_ctx *h, size_t bytes) {
  if (h->run_dev_cap < bytes) {
    if (h->run_dev) {
      HIPCHK(hipStreamSynchronize(h->stream));
      HIPCHK(hipFree(h->run_dev));
      h->run_dev = nullptr;
      h->run_dev_cap = 0;
    }
    HIPCHK(hipMalloc((void **)&h->run_dev, bytes));
    h->run_dev_cap = bytes;
  }
  if (h->run_host_cap < bytes) {
    if (h->run_host) {
      HIPCHK(hipStreamSynchronize(h->stream));
      HIPCHK(hipHostFree(h->run_host));
      h->run_host = nullptr;
      h->run_host_cap = 0;
    }
    HIPCHK(hipHostMalloc((void **)&h->run_host, bytes, hipHostMallocDefault));
    h->run_host_cap = bytes;
  }
  return 0;
}

// Where a run keeps its arguments and results. The default (dev == null)
// is the first chain's buffers above; fmm_mc_run_noalloc hands in its own.
struct RunMem {
  char *dev = nullptr;   // device block laid out as RunArea
  char *host = nullptr;  // host staging of the same layout
  char *work = nullptr;  // noalloc_work_bytes(n_chains) of host bookkeeping
};

// shared driver of fmm_mc_run, fmm_mc_run_noalloc and fmm_mc_replay. With
// resetup_every > 0 a chain stops after that many accepts, is re-set up
// (its captured setup graph, FP64) and continues where it stopped, until
// every chain has done `steps` steps; the chains still running are
// relaunched together. A run of one chain on the whole GPU passes its
// arguments by value and takes its results from the chain's workspace; a
// run of many copies its slots' arguments in once and the results out once
// per launch.
static int run_chains(fmm_mc_t *chains, int n_chains, int64_t steps, uint64_t seed, int64_t t0, double beta,
                      const double *steps_h, int mode, int64_t resetup_every, const int64_t *l_idx,
                      const double *l_pos, const double *l_u, int64_t *tr_idx, double *tr_pos, double *tr_dE,
                      uint8_t *tr_acc, int32_t *tr_leaf, fmm_mc_stats *stats, const RunMem *mem = nullptr) {
  fmm_mc_t h0 = chains[0];
  for (int c = 0; c < n_chains; ++c) {
    if (!chains[c] || !chains[c]->ready) return FMM_MC_ESTATE;
    if (chains[c]->p != h0->p || chains[c]->device != h0->device || chains[c]->stream != h0->stream ||
        chains[c]->flags != h0->flags)
      return FMM_MC_ESTATE;
  }
  for (int c = 0; c < n_chains; ++c) chains[c]->undo_ok = false;
  const bool mixed = (h0->flags & FMM_MC_MIXED) != 0;
  const bool mp = (h0->flags & FMM_MC_MULTIPOLE) != 0;
  hipStream_t st = h0->stream;
  const Tabs &tb = h0->tables->tabs;
  const int GS = h0->GS;
  const bool single = (n_chains == 1 && mode != 1);
  // many chains with 16-lane groups run the whole-GPU chain's workgroup-0
  // loop, one workgroup per chain (k_run_chains); the others k_run_batched
  const bool lead = !single && !mp && GS == 16;
  const int NT = single || lead ? WG_SINGLE : WG_BATCH;
  size_t shm = smem_bytes(GS, tb, NT);
  const RunArea ra(n_chains);
  char *dev = nullptr, *host = nullptr;
  if (!single) {
    if (mem) {
      dev = mem->dev;
      host = mem->host;
    } else {
      int r = ensure_run_area(h0, ra.bytes);
      if (r) return r;
      dev = h0->run_dev;
      host = h0->run_host;
    }
  }
  double *d_stats = single ? (double *)(h0->ws + h0->ly.off[O_STATS]) : (double *)(dev + ra.o_stats);
  double *h_stats = single ? h0->host_stats : (double *)(host + ra.o_stats);
  RunParams rp{};
  rp.steps = steps;
  rp.t0 = t0;
  rp.seed = seed;
  rp.beta = beta;
  rp.max_step = single ? nullptr : (const double *)(dev + ra.o_step);
  rp.max_step0 = steps_h[0];
  rp.first = single ? nullptr : (const int64_t *)(dev + ra.o_first);
  rp.chain_id = single ? nullptr : (const int *)(dev + ra.o_id);
  rp.acc_limit = resetup_every > 0 ? resetup_every : 0;
  rp.list_idx = l_idx;
  rp.list_pos = l_pos;
  rp.list_u = l_u;
  rp.tr_idx = tr_idx;
  rp.tr_pos = tr_pos;
  rp.tr_dE = tr_dE;
  rp.tr_acc = tr_acc;
  rp.tr_leaf = tr_leaf;
  rp.stats = d_stats;
  if (!single && steps_h != (const double *)(host + ra.o_step))
    std::memcpy(host + ra.o_step, steps_h, sizeof(double) * n_chains);
  int G = 1;
  if (single && mp) {
    // workgroup 0 proposes and accepts, the others (one per CU at most)
    // share the far-field items of each proposal
    const int NG = NT / GS;
    int ncu = 0, per = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h0->device));
    G = (mp_items(h0->ch.L) + NG - 1) / NG + 1;
    if (h0->helpers > 0) G = std::min(G, h0->helpers + 1);
    G = std::max(1, std::min(G, std::min(ncu, 448)));
    hipError_t oe = hipSuccess;
    with_variant(variant_of(h0->p), [&](auto gs, auto pm) {
      oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, k_run_single_mp<decltype(gs)::value, decltype(pm)::value>, NT, shm);
    });
    HIPCHK(oe);
    if (per < 1) return FMM_MC_EDEVICE;
  } else if (single) {
    // workgroup 0 proposes, the others (one per CU at most) hold the accept
    // blocks; the busiest helper's speculative rows must fit its LDS
    const int NG = NT / GS;
    const int nblk = accept_blocks(h0->ch.L, NG);
    int ncu = 0, maxlds = 0, per = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h0->device));
    HIPCHK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, h0->device));
    // the kernel's own (static) LDS comes out of the same budget
    hipFuncAttributes fa{};
    hipError_t ae = hipSuccess;
    with_run_variant(h0->p, mixed, [&](auto gs, auto pm, auto rt) {
      ae = hipFuncGetAttributes(
          &fa, (const void *)k_run_single<decltype(gs)::value, decltype(pm)::value, typename decltype(rt)::type>);
    });
    HIPCHK(ae);
    maxlds -= (int)fa.sharedSizeBytes;
    auto kmax_of = [&](int g) { return g < 2 ? 1 : (nblk + g - 2) / (g - 1); };
    auto shm_of = [&](int g) { return smem_bytes(GS, tb, NT) + (g < 2 ? 0 : spec_extra_bytes(kmax_of(g), NG, h0->Cs)); };
    G = nblk + 1;
    if (h0->helpers > 0) G = std::min(G, h0->helpers + 1);
    G = std::max(1, std::min(G, ncu));
    while (G < ncu && G < nblk + 1 && (kmax_of(G) > SPEC_MAX || shm_of(G) > (size_t)maxlds)) ++G;
    if (kmax_of(G) > SPEC_MAX || shm_of(G) > (size_t)maxlds) return FMM_MC_EDEVICE;
    shm = shm_of(G);
    hipError_t oe = hipSuccess;
    with_run_variant(h0->p, mixed, [&](auto gs, auto pm, auto rt) {
      oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, k_run_single<decltype(gs)::value, decltype(pm)::value, typename decltype(rt)::type>, NT, shm);
    });
    HIPCHK(oe);
    if (per < 1) return FMM_MC_EDEVICE;
  }
  // per chain of the run: steps done, accumulated counters, final energy,
  // and the chains of a launch's slots
  std::vector<char> own;
  char *work = mem ? mem->work : nullptr;
  if (!work) {
    own.resize(noalloc_work_bytes(n_chains));
    work = own.data();
  }
  int64_t *done = (int64_t *)work;
  double *acc = (double *)(done + n_chains);
  double *energy = acc + RUN_NSTAT * n_chains;
  int *ids = (int *)(energy + n_chains);
  std::memset(work, 0, noalloc_work_bytes(n_chains));
  double kernel_ms = 0.0;
  int rc = FMM_MC_OK;
  while (rc == FMM_MC_OK) {
    int na = 0;
    for (int c = 0; c < n_chains; ++c)
      if (done[c] < steps) ids[na++] = c;
    if (na == 0) break;
    if (single) {
      rp.first0 = done[0];
      hipLaunchKernelGGL(k_fill_i32, dim3(2), dim3(NT), 0, st, (int *)h0->ch.sync, 0, 512);
    } else {
      Chain *hd = (Chain *)(host + ra.o_desc);
      int64_t *hf = (int64_t *)(host + ra.o_first);
      int *hi = (int *)(host + ra.o_id);
      for (int k = 0; k < na; ++k) {
        hd[k] = chains[ids[k]]->ch;
        hf[k] = done[ids[k]];
        hi[k] = ids[k];
      }
      // descriptors, first steps, ids and step sizes lie before the results
      HIPCHK(hipMemcpyAsync(dev, host, ra.o_stats, hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipEventRecord(h0->ev0, st));
    if (single) {
      Chain chv = h0->ch;
      void *args[] = {&chv, (void *)&tb, &rp};
      hipError_t e = hipSuccess;
      if (mp)
        with_variant(variant_of(h0->p), [&](auto gs, auto pm) {
          e = hipLaunchCooperativeKernel((const void *)k_run_single_mp<decltype(gs)::value, decltype(pm)::value>,
                                         dim3(G), dim3(NT), args, shm, st);
        });
      else
        with_run_variant(h0->p, mixed, [&](auto gs, auto pm, auto rt) {
          e = hipLaunchCooperativeKernel(
              (const void *)k_run_single<decltype(gs)::value, decltype(pm)::value, typename decltype(rt)::type>,
              dim3(G), dim3(NT), args, shm, st);
        });
      HIPCHK(e);
    } else {
      const Chain *d_chains = (const Chain *)(dev + ra.o_desc);
      if (mp) {
        with_variant(variant_of(h0->p), [&](auto gs, auto pm) {
          hipLaunchKernelGGL(HIP_KERNEL_NAME(k_run_batched<decltype(gs)::value, decltype(pm)::value, double, true>),
                             dim3(na), dim3(NT), shm, st, d_chains, tb, rp);
        });
      } else {
        with_run_variant(h0->p, mixed, [&](auto gs, auto pm, auto rt) {
          constexpr int gsv = decltype(gs)::value;
          if constexpr (gsv == 16)  // lead
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_run_chains<gsv, decltype(pm)::value, typename decltype(rt)::type>),
                               dim3(na), dim3(NT), shm, st, d_chains, tb, rp);
          else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_run_batched<gsv, decltype(pm)::value, typename decltype(rt)::type>),
                               dim3(na), dim3(NT), shm, st, d_chains, tb, rp);
        });
      }
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(h0->ev1, st));
    HIPCHK(hipMemcpyAsync(h_stats, d_stats, sizeof(double) * RUN_NSTAT * na, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, h0->ev0, h0->ev1));
    kernel_ms += ms;
    for (int k = 0; k < na; ++k) {
      const int c = ids[k];
      const double *v = &h_stats[RUN_NSTAT * k];
      for (int j = 0; j < 8; ++j)
        if (j != 4) acc[RUN_NSTAT * c + j] += v[j];
      done[c] += (int64_t)v[0];
      energy[c] = v[8];
      if ((int)v[4] != 0) {
        acc[RUN_NSTAT * c + 4] = v[4];
        rc = (int)v[4];
      } else if (v[0] < 1.0) {
        rc = FMM_MC_ESTATE;  // a launch that made no step would be relaunched for ever
      }
    }
    if (rc != FMM_MC_OK) break;
    // chains that stopped at the accept limit with steps left: re-setup
    for (int k = 0; k < na && rc == FMM_MC_OK; ++k) {
      const int c = ids[k];
      if (done[c] < steps) {
        int r = fmm_mc_resetup(chains[c]);
        if (r) rc = r;
      }
    }
  }
  h0->last_ms[0] = kernel_ms;
  if (stats)
    for (int c = 0; c < n_chains; ++c) {
      const double *v = &acc[RUN_NSTAT * c];
      stats[c].proposed = (int64_t)v[0];
      stats[c].accepted = (int64_t)v[1];
      stats[c].singular = (int64_t)v[2];
      stats[c].dE_sum = v[3];
      stats[c].energy = energy[c];
      stats[c].status = (int32_t)v[4];
      stats[c].t_propose_us = v[5];
      stats[c].t_accept_us = v[6];
      stats[c].t_wait_us = v[7];
    }
  return rc;
}

int fmm_mc_run(fmm_mc_t *chains, int n_chains, int64_t steps, uint64_t seed, const fmm_mc_run_opts *opts,
               fmm_mc_stats *stats) {
  if (!chains || n_chains < 1 || steps < 0 || !opts) return FMM_MC_EINVAL;
  if (!(opts->beta >= 0.0) || !std::isfinite(opts->beta)) return FMM_MC_EINVAL;
  std::vector<double> st(n_chains);
  for (int c = 0; c < n_chains; ++c) {
    st[c] = opts->chain_max_step ? opts->chain_max_step[c] : opts->max_step;
    if (!(st[c] >= 0.0) || !std::isfinite(st[c])) return FMM_MC_EINVAL;
  }
  if (steps == 0) return FMM_MC_OK;
  if (opts->resetup_every < 0) return FMM_MC_EINVAL;
  return run_chains(chains, n_chains, steps, seed, opts->t0, opts->beta, st.data(), opts->mode, opts->resetup_every,
                    nullptr, nullptr, nullptr, opts->trace_idx, opts->trace_newpos, opts->trace_dE, opts->trace_acc,
                    nullptr, stats);
}

int fmm_mc_run_noalloc(fmm_mc_t *chains, int n_chains, int64_t steps, uint64_t seed, const fmm_mc_run_opts *opts,
                       fmm_mc_stats *stats) {
  if (n_chains > FMM_MC_NOALLOC_MAX_CHAINS) return FMM_MC_ENOMEM;
  if (!chains || n_chains < 1 || steps < 0 || !opts) return FMM_MC_EINVAL;
  if (!(opts->beta >= 0.0) || !std::isfinite(opts->beta)) return FMM_MC_EINVAL;
  // a re-setup captures and instantiates a graph on its first use
  if (opts->resetup_every != 0) return FMM_MC_EINVAL;
  if (!chains[0] || !chains[0]->ready) return FMM_MC_ESTATE;
  const int dev = chains[0]->device;
  if (dev < 0 || dev >= MAX_DEVICES) return FMM_MC_EDEVICE;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  RunMem mem;
  {
    std::lock_guard<std::mutex> lk2(g_mu);
    mem.dev = (char *)g_scratch_dev[dev];
  }
  mem.host = g_noalloc_host;
  if (!mem.dev || !mem.host) return FMM_MC_EDEVICE;
  mem.work = mem.host + NOALLOC_SCRATCH_BYTES;
  // the step sizes go straight to their place in the staging block
  const RunArea ra(n_chains);
  double *st = (double *)(mem.host + ra.o_step);
  for (int c = 0; c < n_chains; ++c) {
    st[c] = opts->chain_max_step ? opts->chain_max_step[c] : opts->max_step;
    if (!(st[c] >= 0.0) || !std::isfinite(st[c])) return FMM_MC_EINVAL;
  }
  if (steps == 0) return FMM_MC_OK;
  return run_chains(chains, n_chains, steps, seed, opts->t0, opts->beta, st, opts->mode, 0, nullptr, nullptr,
                    nullptr, opts->trace_idx, opts->trace_newpos, opts->trace_dE, opts->trace_acc, nullptr, stats,
                    &mem);
}

int fmm_mc_replay(fmm_mc_t h, int64_t m, const int64_t *idx, const double *new_pos, const double *u, double beta,
                  double *dE, uint8_t *acc, int32_t *leaf) {
  if (!h || !h->ready) return FMM_MC_ESTATE;
  if (m < 0 || (m > 0 && (!idx || !new_pos || !u))) return FMM_MC_EINVAL;
  if (m == 0) return FMM_MC_OK;
  for (int64_t i = 0; i < m; ++i) {
    if (idx[i] < 0 || idx[i] >= h->n) return FMM_MC_ERANGE;
    if (!finite3(new_pos + 3 * i) || !std::isfinite(u[i])) return FMM_MC_EINVAL;
  }
  // the fixed lists in and the per-step results out, in stream-ordered
  // device memory of this call (the replay is the test path)
  double *d_dE = nullptr, *d_lpos = nullptr, *d_lu = nullptr;
  int64_t *d_lidx = nullptr;
  uint8_t *d_acc = nullptr;
  int32_t *d_leaf = nullptr;
  HIPCHK(hipMallocAsync((void **)&d_dE, sizeof(double) * m, h->stream));
  HIPCHK(hipMallocAsync((void **)&d_acc, m, h->stream));
  HIPCHK(hipMallocAsync((void **)&d_leaf, sizeof(int32_t) * m, h->stream));
  HIPCHK(hipMallocAsync((void **)&d_lidx, sizeof(int64_t) * m, h->stream));
  HIPCHK(hipMallocAsync((void **)&d_lpos, sizeof(double) * 3 * m, h->stream));
  HIPCHK(hipMallocAsync((void **)&d_lu, sizeof(double) * m, h->stream));
  int rc = FMM_MC_OK;
  if (hipMemcpyAsync(d_lidx, idx, sizeof(int64_t) * m, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipMemcpyAsync(d_lpos, new_pos, sizeof(double) * 3 * m, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipMemcpyAsync(d_lu, u, sizeof(double) * m, hipMemcpyHostToDevice, h->stream) != hipSuccess)
    rc = FMM_MC_EDEVICE;
  double zero = 0.0;
  fmm_mc_t hs[1] = {h};
  if (rc == FMM_MC_OK)
    rc = run_chains(hs, 1, m, 0, 0, beta, &zero, 0, 0, d_lidx, d_lpos, d_lu, nullptr, nullptr, d_dE, d_acc, d_leaf,
                    nullptr);
  if (rc == FMM_MC_OK) {
    if (dE && hipMemcpyAsync(dE, d_dE, sizeof(double) * m, hipMemcpyDeviceToHost, h->stream) != hipSuccess)
      rc = FMM_MC_EDEVICE;
    if (acc && hipMemcpyAsync(acc, d_acc, m, hipMemcpyDeviceToHost, h->stream) != hipSuccess) rc = FMM_MC_EDEVICE;
    if (leaf && hipMemcpyAsync(leaf, d_leaf, sizeof(int32_t) * m, hipMemcpyDeviceToHost, h->stream) != hipSuccess)
      rc = FMM_MC_EDEVICE;
  }
  (void)hipFreeAsync(d_dE, h->stream);
  (void)hipFreeAsync(d_acc, h->stream);
  (void)hipFreeAsync(d_leaf, h->stream);
  (void)hipFreeAsync(d_lidx, h->stream);
  (void)hipFreeAsync(d_lpos, h->stream);
  (void)hipFreeAsync(d_lu, h->stream);
  HIPCHK(hipStreamSynchronize(h->stream));
  return rc;
}

int fmm_mc_energy(fmm_mc_t h, double *U) {
  if (!h || !h->ready) return FMM_MC_ESTATE;
  if (!U) return FMM_MC_EINVAL;
  return compute_energy(h, U);
}

int fmm_mc_running_energy(fmm_mc_t h, double *U) {
  if (!h || !h->ready) return FMM_MC_ESTATE;
  if (!U) return FMM_MC_EINVAL;
  HIPCHK(hipMemcpyAsync(U, h->ch.U, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return FMM_MC_OK;
}

int fmm_mc_get_positions(fmm_mc_t h, double *pos) {
  if (!h || !h->ready) return FMM_MC_ESTATE;
  if (!pos) return FMM_MC_EINVAL;
  std::vector<double> b(3 * h->n);
  HIPCHK(hipMemcpyAsync(b.data(), h->ch.px, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(b.data() + h->n, h->ch.py, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(b.data() + 2 * h->n, h->ch.pz, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int64_t i = 0; i < h->n; ++i) {
    pos[3 * i] = b[i];
    pos[3 * i + 1] = b[h->n + i];
    pos[3 * i + 2] = b[2 * h->n + i];
  }
  return FMM_MC_OK;
}

// a level of the scaled expansions ch.X + off, unscaled (by h^-(n+1) for
// local expansions, h^n for multipoles) into the host layout
static int dump_level(fmm_mc_t h, const double *base, int level, bool multipole, double *out) {
  const long long nc = 1LL << (3 * (level - 1));
  std::vector<double> b((size_t)nc * h->Cs);
  HIPCHK(hipMemcpyAsync(b.data(), base, sizeof(double) * b.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  const double hcell = h->box / double(1 << (level - 1));
  for (long long c = 0; c < nc; ++c)
    for (int n = 0; n <= h->p; ++n) {
      const double sc = multipole ? std::pow(hcell, n) : std::pow(hcell, -(n + 1));
      for (int m = -n; m <= n; ++m) {
        int s = n * n + n + m;
        out[(size_t)c * h->C + s] = b[(size_t)c * h->Cs + s] * sc;
      }
    }
  return FMM_MC_OK;
}

int fmm_mc_dump_multipoles(fmm_mc_t h, int level, double *out) {
  if (!h || !h->ready) return FMM_MC_ESTATE;
  if (!out || level < 1 || level > h->ch.L) return FMM_MC_EINVAL;
  return dump_level(h, h->ch.Mp + h->ch.mp_off[level], level, true, out);
}

int fmm_mc_dump_locals(fmm_mc_t h, int level, double *out) {
  if (!h || !h->ready || (h->flags & FMM_MC_MULTIPOLE)) return FMM_MC_ESTATE;
  if (!out || level < 2 || level > h->ch.L) return FMM_MC_EINVAL;
  return dump_level(h, h->ch.Ld + h->ch.ld_off[level], level, false, out);
}

int fmm_mc_last_timing(fmm_mc_t h, double *out, int nout) {
  if (!h || !out || nout < 1) return FMM_MC_EINVAL;
  for (int i = 0; i < nout && i < 4; ++i) out[i] = h->last_ms[i];
  return FMM_MC_OK;
}

// a chain descriptor whose pointers are moved from one workspace to another
extern "C++" {
template <typename T>
static T *rebase(T *p, const char *from, char *to) {
  return p ? (T *)(to + ((const char *)p - from)) : nullptr;
}

static Chain rebase_chain(const Chain &c, const char *from, char *to) {
  Chain r = c;
  r.px = rebase(c.px, from, to);
  r.py = rebase(c.py, from, to);
  r.pz = rebase(c.pz, from, to);
  r.pq = rebase(c.pq, from, to);
  r.leaf_of = rebase(c.leaf_of, from, to);
  r.slot_of = rebase(c.slot_of, from, to);
  r.bin_cnt = rebase(c.bin_cnt, from, to);
  r.bin_id = rebase(c.bin_id, from, to);
  r.bin_p = rebase(c.bin_p, from, to);
  r.Ld = rebase(c.Ld, from, to);
  r.Mp = rebase(c.Mp, from, to);
  r.K = rebase(c.K, from, to);
  r.H = rebase(c.H, from, to);
  r.dip = rebase(c.dip, from, to);
  r.U = rebase(c.U, from, to);
  r.status = rebase(c.status, from, to);
  r.scratch = rebase(c.scratch, from, to);
  r.mbox = rebase(c.mbox, from, to);
  r.sync = rebase(c.sync, from, to);
  r.red = rebase(c.red, from, to);
  r.part = rebase(c.part, from, to);
  r.dscr = rebase(c.dscr, from, to);
  r.stage = rebase(c.stage, from, to);
  return r;
}
}  // extern "C++"

int fmm_mc_autotune(fmm_mc_t h, int64_t steps, double beta, double max_step, fmm_mc_tuning *out) {
  if (!h || !h->ready) return FMM_MC_ESTATE;
  if (steps < 0 || !(beta >= 0.0) || !std::isfinite(beta) || !(max_step >= 0.0) || !std::isfinite(max_step))
    return FMM_MC_EINVAL;
  if (steps == 0) steps = 1000;
  const size_t bytes = h->ly.total;
  char *tmp = nullptr;
  HIPCHK(hipMalloc((void **)&tmp, bytes));
  // a shadow context on a clone of the workspace (tables and events shared)
  fmm_mc_ctx sh = *h;
  sh.ws = tmp;
  sh.graph = nullptr;
  sh.gexec = nullptr;
  sh.cap_stream = nullptr;
  sh.ch = rebase_chain(h->ch, h->ws, tmp);
  sh.d_chain = (Chain *)(tmp + h->ly.off[O_CHAIN]);
  sh.d_tiles = (int4 *)(tmp + h->ly.off[O_TILES]);
  auto clone = [&]() {
    return hipMemcpyAsync(tmp, h->ws, bytes, hipMemcpyDeviceToDevice, h->stream) == hipSuccess &&
           hipMemcpyAsync(sh.d_chain, &sh.ch, sizeof(Chain), hipMemcpyHostToDevice, h->stream) == hipSuccess;
  };
  fmm_mc_tuning t{};
  int rc = clone() ? 0 : FMM_MC_EDEVICE;
  // (a) M2L output rows per workgroup, timed on the clone (3 launches each)
  const int rows[2] = {96, 192};
  const bool mp = (h->flags & FMM_MC_MULTIPOLE) != 0;
  const bool no_m2l = mp || (h->flags & FMM_MC_DIRECT_SETUP);  // no M2L pass to tune
  double best = 1e300;
  t.m2l_rows = no_m2l ? 96 : 192;
  for (int k = 0; k < 2 && !rc && !no_m2l; ++k) {
    SetupLaunch S = single_launch(&sh);
    S.m2l_rows = rows[k];
    launch_m2l(S);
    if (hipEventRecord(h->ev1, h->stream) != hipSuccess) rc = FMM_MC_EDEVICE;
    for (int r = 0; r < 3; ++r) launch_m2l(S);
    float ms = 0;
    if (rc || hipEventRecord(h->ev2, h->stream) != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess ||
        hipEventElapsedTime(&ms, h->ev1, h->ev2) != hipSuccess)
      rc = FMM_MC_EDEVICE;
    t.m2l_ms[k] = ms / 3.0;
    if (!rc && t.m2l_ms[k] < best) {
      best = t.m2l_ms[k];
      t.m2l_rows = rows[k];
    }
  }
  // (b) helper workgroups of the whole-GPU run: `steps` MH steps of each
  // candidate from the same cloned state, in two interleaved passes (the
  // faster of the two counts); a smaller count than all blocks is taken
  // only if it is more than 2 % faster
  // units of helper work: accept blocks, or groups of far-field items in
  // the multipole-based variant
  const int NGs = WG_SINGLE / h->GS;
  const int nblk = mp ? (mp_items(h->ch.L) + NGs - 1) / NGs : accept_blocks(h->ch.L, NGs);
  const int div[8] = {1, 2, 3, 4, 6, 8, 12, 16};
  for (int k = 0; k < 8; ++k) {
    const int cand = (nblk + div[k] - 1) / div[k];
    bool seen = false;
    for (int j = 0; j < t.n_helper_candidates; ++j) seen = seen || t.helper_candidates[j] == cand;
    if (seen || cand < 1) continue;
    const int j = t.n_helper_candidates++;
    t.helper_candidates[j] = cand;
    t.step_us[j] = 1e300;
  }
  for (int pass = 0; pass < 2 && !rc; ++pass)
    for (int j = 0; j < t.n_helper_candidates && !rc; ++j) {
      if (!clone()) {
        rc = FMM_MC_EDEVICE;
        break;
      }
      sh.helpers = t.helper_candidates[j];
      fmm_mc_t arr[1] = {&sh};
      rc = run_chains(arr, 1, steps, 0x5eedULL, 0, beta, &max_step, 2, 0, nullptr, nullptr, nullptr, nullptr,
                      nullptr, nullptr, nullptr, nullptr, nullptr);
      t.step_us[j] = std::min(t.step_us[j], sh.last_ms[0] * 1e3 / (double)steps);
    }
  t.helpers = nblk;
  best = t.step_us[0];  // candidate 0 is all blocks
  for (int j = 1; j < t.n_helper_candidates; ++j)
    if (t.step_us[j] < 0.98 * t.step_us[0] && t.step_us[j] < best) {
      best = t.step_us[j];
      t.helpers = t.helper_candidates[j];
    }
  (void)hipStreamSynchronize(h->stream);
  (void)hipFree(tmp);
  if (rc) return rc;
  h->m2l_rows = t.m2l_rows;
  h->helpers = t.helpers;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    const uint32_t mixed = h->flags;
    bool found = false;
    for (auto &e : g_tune)
      if (e.device == h->device && e.p == h->p && e.levels == h->levels && e.mixed == mixed) {
        e.m2l_rows = t.m2l_rows;
        e.helpers = t.helpers;
        found = true;
      }
    if (!found) g_tune.push_back({h->device, h->p, h->levels, mixed, t.m2l_rows, t.helpers});
  }
  if (out) *out = t;
  return FMM_MC_OK;
}

int fmm_mc_set_helpers(fmm_mc_t h, int helpers) {
  if (!h || helpers < 0) return FMM_MC_EINVAL;
  h->helpers = helpers;
  return FMM_MC_OK;
}

int fmm_mc_destroy(fmm_mc_t h) {
  if (!h) return FMM_MC_EINVAL;
  // nothing of this handle may still be in flight when its objects go
  (void)hipStreamSynchronize(h->stream);
  if (h->cap_stream) (void)hipStreamSynchronize(h->cap_stream);
  if (h->run_dev) (void)hipFree(h->run_dev);
  if (h->run_host) (void)hipHostFree(h->run_host);
  if (h->host_stats) (void)hipHostFree(h->host_stats);
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  if (h->ev2) (void)hipEventDestroy(h->ev2);
  delete h;
  return FMM_MC_OK;
}

int fmm_mc_release_tables(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  for (size_t i = 0; i < g_tables.size();) {
    if (g_tables[i]->device == dev) {
      for (void *a : g_tables[i]->allocs) (void)hipFree(a);
      delete g_tables[i];
      g_tables.erase(g_tables.begin() + i);
    } else {
      ++i;
    }
  }
  return FMM_MC_OK;
}

const char *fmm_mc_strerror(int code) {
  switch (code) {
    case FMM_MC_OK: return "ok";
    case FMM_MC_EINVAL: return "invalid argument";
    case FMM_MC_ERANGE: return "particle index out of range";
    case FMM_MC_ENONNEUTRAL: return "charges do not sum to zero";
    case FMM_MC_ESINGULAR: return "new position coincides with another charge";
    case FMM_MC_ENOMEM: return "workspace too small";
    case FMM_MC_EDEVICE: return "HIP call failed";
    case FMM_MC_EOVERFLOW: return "leaf cell capacity exceeded";
    case FMM_MC_ESTATE: return "handle not ready or chains inconsistent";
    default: return "unknown error";
  }
}

// Host-only diagnostic: the constant operators as the library builds them
// (no device needed). kind 0: M2L operator of IL offset (o[0],o[1],o[2]),
// element [in s][out j]; kind 1: M2M operator of child octant o[0]; kind 2:
// lattice operator, element [out j][in s]. out: (p+1)^4 doubles, host.
int fmm_mc_host_operator(int kind, int p, const int *o, double *out) {
  if (!out || p < 0 || p > PMAX) return FMM_MC_EINVAL;
  if (kind == 0) {
    if (!o) return FMM_MC_EINVAL;
    fmmhost::m2l_operator(p, o, out);
  } else if (kind == 1) {
    if (!o || o[0] < 0 || o[0] > 7) return FMM_MC_EINVAL;
    fmmhost::m2m_operator(p, o[0], out);
  } else if (kind == 2) {
    fmmhost::lattice_operator(p, out);
  } else {
    return FMM_MC_EINVAL;
  }
  return FMM_MC_OK;
}

}  // extern "C"
