// mp_step.hpp -- the per-step device work of the multipole-based variant
// (Sec. 3.3): the far field of a proposal as the multipole expansions of the
// interaction lists of both cells on every level, evaluated at the charge
// (Alg. M.1), and the accept as the update of one multipole expansion per
// level and side (Alg. M.2). The near field, the self-image correction, the
// far lattice and the tin-foil term are those of the local variant
// (Sec. 3.4, propose_wg without its local expansions).
#pragma once

#include "mc_step.hpp"

namespace fmmdev {

// far-field items of one move: level 2..L, old or new side, IL offset
__host__ __device__ inline int mp_items(int L) { return 378 * (L - 1); }

// M2P, Eq. (multipole_expansion), of the stored multipole of the cell whose
// image b = c + IL offset k of cell c on level l lies in the interaction
// list, at the point x. Lane m of the group forms column m of the
// conjugated irregular harmonics at the scaled displacement (x - R_b)/h and
// multiplies each term with the matching scaled coefficient M^ (real
// layout: Re at slot (n, m), Im at slot (n, -m)), so that the group sum of
// the returned lane values is Re sum M_n^m I_n^m = Phi_b(x - R_b), with the
// weights 1 (m = 0) and 2 (m > 0) of the real form and 1/h of the scaling.
template <int GS, int PM, typename IL>
__device__ __forceinline__ double m2p_cell(const Chain &ch, const Tabs &tb, const double *rec, const IL *il,
                                           int l, const int c[3], const double x[3], int k, int lane) {
  const int n = 1 << (l - 1);
  const double h = ch.a / n;
  const int oc = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2);
  int o[3];
  il_entry(il, oc * 189 + k, o);
  const int b[3] = {c[0] + o[0], c[1] + o[1], c[2] + o[2]};
  // free space: cells outside the box hold nothing (uniform over the group)
  if (ch.free_space && (b[0] < 0 || b[0] >= n || b[1] < 0 || b[1] >= n || b[2] < 0 || b[2] >= n)) return 0.0;
  double v[3];
  for (int d = 0; d < 3; ++d) v[d] = (x[d] - (b[d] + 0.5) * h) / h;
  const auto src =
      glb(ch.Mp) + ch.mp_off[l] + (size_t)lin3(n, pmod(b[0], n), pmod(b[1], n), pmod(b[2], n)) * tb.Cs;
  const int p = tb.p, m = lane;
  // the coefficients of column m, requested before the recurrence starts
  double mre[PM + 1], mim[PM + 1];
#pragma unroll
  for (int j = 0; j <= PM; ++j) {
    const int nn = m + j;
    const bool in = m <= p && nn <= p;
    mre[j] = in ? src[nn * nn + nn + m] : 0.0;
    mim[j] = in && m > 0 ? src[nn * nn + nn - m] : 0.0;
  }
  double acc = 0.0;
  harmonics_core<GS, PM, 2, double>(lane, tb, rec, v[0], v[1], v[2], 1.0,
                                    [&](int j, int, double re, double im) { acc += mre[j] * re + mim[j] * im; });
  return (m == 0 ? acc : 2.0 * acc) / h;
}

// item i of the far field of move mv, with the sign of its side
// (+ at r' over IL(a'_l), - at r over IL(a_l)), as lane values
template <int GS, int PM>
__device__ __forceinline__ double m2p_item(const Chain &ch, const Tabs &tb, const double *rec, const int *il32,
                                           const Move &mv, int item, int lane) {
  const int l = 2 + item / 378, rem = item % 378, side = rem / 189, k = rem % 189;
  const double v = m2p_cell<GS, PM>(ch, tb, rec, il32, l, side ? mv.c1[l] : mv.c0[l], side ? mv.rn : mv.r, k, lane);
  return side ? v : -v;
}

// lane partial sums of the far-field items first + g, first + g + stride,
// ... of move mv, for group g of the calling workgroup (items in a fixed
// order per group)
template <int GS, int PM>
__device__ __forceinline__ double m2p_far_part(const Chain &ch, const Tabs &tb, const double *rec,
                                               const int *il32, const Move &mv, int first, int stride) {
  const int g = threadIdx.x / GS, lane = threadIdx.x % GS;
  const int ni = mp_items(ch.L);
  double acc = 0.0;
  for (int i = first + g; i < ni; i += stride) acc += m2p_item<GS, PM>(ch, tb, rec, il32, mv, i, lane);
  return acc;
}

// Energy change of move mv in the multipole-based variant, by one whole
// workgroup: the terms of propose_wg without local expansions, plus
// q [Phi_far(r') - Phi_far(r)] over all far-field items (Alg. M.1), the
// groups' partial sums added by a fixed tree.
template <int GS, int PM, int NT, typename Spare>
__device__ ProposeOut propose_mp_wg(const Chain &ch, const Tabs &tb, const Move &mv, Lds<GS, NT> &sm,
                                    Spare &&spare) {
  constexpr int NG = NT / GS;
  ProposeOut po = propose_wg<GS, PM, double, false>(ch, tb, mv, sm, spare);
  double far = m2p_far_part<GS, PM>(ch, tb, sm.rec, sm.il32, mv, 0, NG);
  far = wg_sum<NT>(far, sm.red);
  po.dE += mv.q * far;
  return po;
}

// The multipole part of an accepted move (Alg. M.2): on every level the
// charge leaves the multipole of its old cell (-q at r) and joins that of
// its new cell (+q at r'). Group g takes level 2 + g / 2 and side g % 2 (and
// further levels in steps of NG / 2); when both cells of a level coincide
// the old-side group adds both terms (in the order old, new) and the
// new-side group does nothing, so no row has two writers. The sums stay in
// registers until the row is updated once.
template <int GS, int PM, int NT>
__device__ void accept_mp_wg(const Chain &ch, const Tabs &tb, const Move &mv, const double *rec) {
  constexpr int NG = NT / GS;
  const int g = threadIdx.x / GS, lane = threadIdx.x % GS;
  const double a = ch.a, q = mv.q;
  for (int it = g; it < 2 * (ch.L - 1); it += NG) {
    const int l = 2 + it / 2, side = it % 2, n = 1 << (l - 1);
    const double h = a / n;
    const int *c0 = mv.c0[l], *c1 = mv.c1[l];
    const bool same = c0[0] == c1[0] && c0[1] == c1[1] && c0[2] == c1[2];
    if (side == 1 && same) continue;
    const int *c = side ? c1 : c0;
    const double *x = side ? mv.rn : mv.r;
    ColSum<PM> cs;
    cs.zero();
    group_harmonics_sum<GS, PM, 1>(lane, tb, rec, (x[0] - (c[0] + 0.5) * h) / h, (x[1] - (c[1] + 0.5) * h) / h,
                                   (x[2] - (c[2] + 0.5) * h) / h, side ? q : -q, cs);
    if (same)
      group_harmonics_sum<GS, PM, 1>(lane, tb, rec, (mv.rn[0] - (c[0] + 0.5) * h) / h,
                                     (mv.rn[1] - (c[1] + 0.5) * h) / h, (mv.rn[2] - (c[2] + 0.5) * h) / h, q, cs);
    const auto row = glb(ch.Mp) + ch.mp_off[l] + (size_t)lin3(n, c[0], c[1], c[2]) * tb.Cs;
    flush_cols<PM, true>(lane, tb, cs, row);
  }
}

}  // namespace fmmdev
