// host_ops.hpp -- host-side construction of the constant operators of the
// multilevel method: interaction-list offset tables, the level-independent
// (cell-size scaled) M2M and M2L operators, and the periodic lattice
// operator. All in FP64 on the CPU, once per degree p; the device only
// applies them.
//
// Harmonic conventions (those of the paper, Sec. 3.2):
//   Y_n^m = sqrt((n-|m|)!/(n+|m|)!) P_n^|m|(cos th) e^{i m phi}, no
//   Condon-Shortley phase; T_n^m(x) := |x|^n Y_n^m(x^) is a homogeneous
//   harmonic polynomial computed by the Cartesian recurrence
//     T_0^0 = 1,  T_m^m = sqrt((2m-1)/(2m)) (x + i y) T_{m-1}^{m-1},
//     T_n^m = [(2n-1) z T_{n-1}^m - sqrt((n-1)^2-m^2) |x|^2 T_{n-2}^m] / sqrt(n^2-m^2).
//   With N_n^m = sqrt((n-|m|)!(n+|m|)!), the scaled regular / irregular
//   solid harmonics R_n^m = T_n^m / N_n^m and I_n^m = N_n^m T_n^m / |x|^{2n+1}
//   satisfy 1/|x-s| = sum R_n^{-m}(s) I_n^m(x) (|s| < |x|) and the shift
//   identities
//     R_n^m(x+y) = sum_{k,l} i^{|l|+|m-l|-|m|} R_k^l(x) R_{n-k}^{m-l}(y)
//     I_n^m(t+u) = sum_{k,l} (-1)^k i^{|m-l|-|m|-|l|} R_k^l(u) I_{n+k}^{m-l}(t), |u| < |t|.
//   Multipole M_n^m = sum q |s|^n Y_n^{-m}(s^) (Eq. multipole_expansion_coefficients),
//   local L_n^m with Psi = sum L_n^m |x|^n Y_n^m (Eq. local_expansion).
//
// Storage. Coefficients of a real potential satisfy c_n^{-m} = conj(c_n^m);
// a vector of (p+1)^2 reals holds, at slot n*n+n+m, Re c_n^m for m >= 0 and
// Im c_n^{|m|} for m < 0. On a level of cell size h the library stores the
// dimensionless scaled coefficients  M^_n = M_n / h^n  and  L^_n = L_n h^{n+1},
// so every translation operator below is the same on every level.
#pragma once

#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>

namespace fmmhost {

using cd = std::complex<double>;

inline int slot(int n, int m) { return n * n + n + m; }

inline double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= double(i);
  return f;
}

inline double Nnm(int n, int m) {
  static std::vector<double> tab;
  if (tab.empty()) {
    tab.resize(171);
    tab[0] = 1.0;
    for (int i = 1; i <= 170; ++i) tab[i] = tab[i - 1] * double(i);
  }
  int am = m < 0 ? -m : m;
  return std::sqrt(tab[n - am] * tab[n + am]);
}

inline cd ipow(int k) {
  int r = ((k % 4) + 4) % 4;
  static const cd v[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
  return v[r];
}

// T_n^m(x,y,z) for n <= P, all m, complex, index slot(n,m)
inline void solid_T(int P, double x, double y, double z, std::vector<cd> &T) {
  T.assign((P + 1) * (P + 1), cd(0, 0));
  double r2 = x * x + y * y + z * z;
  cd w(x, y), diag(1.0, 0.0);
  for (int m = 0; m <= P; ++m) {
    if (m > 0) diag *= w * std::sqrt((2.0 * m - 1.0) / (2.0 * m));
    cd tm2(0, 0), tm1 = diag;
    T[slot(m, m)] = tm1;
    for (int n = m + 1; n <= P; ++n) {
      double A = (2.0 * n - 1.0) / std::sqrt(double(n * n - m * m));
      double B = std::sqrt(double((n - 1) * (n - 1) - m * m) / double(n * n - m * m));
      cd t = A * z * tm1 - B * r2 * tm2;
      T[slot(n, m)] = t;
      tm2 = tm1;
      tm1 = t;
    }
    for (int n = m; n <= P; ++n) T[slot(n, -m)] = std::conj(T[slot(n, m)]);
  }
}

inline void solid_R(int P, double x, double y, double z, std::vector<cd> &R) {
  solid_T(P, x, y, z, R);
  for (int n = 0; n <= P; ++n)
    for (int m = -n; m <= n; ++m) R[slot(n, m)] /= Nnm(n, m);
}

inline void solid_I(int P, double x, double y, double z, std::vector<cd> &I) {
  solid_T(P, x, y, z, I);
  double r = std::sqrt(x * x + y * y + z * z);
  for (int n = 0; n <= P; ++n)
    for (int m = -n; m <= n; ++m) I[slot(n, m)] *= Nnm(n, m) / std::pow(r, 2 * n + 1);
}

// the complex coefficients (at most two) of the real-layout basis vector e_s
struct BasisEntry {
  int n, m;
  cd v;
};

inline int basis_entries(int s, BasisEntry *e) {
  int n = 0;
  while ((n + 1) * (n + 1) <= s) ++n;
  int m = s - n * n - n;
  if (m == 0) {
    e[0] = {n, 0, cd(1, 0)};
    return 1;
  }
  if (m > 0) {
    e[0] = {n, m, cd(1, 0)};
    e[1] = {n, -m, cd(1, 0)};
    return 2;
  }
  e[0] = {n, -m, cd(0, 1)};
  e[1] = {n, m, cd(0, -1)};
  return 2;
}

// real layout of a conjugate-symmetric complex vector
inline void to_real(int p, const std::vector<cd> &c, double *out) {
  for (int n = 0; n <= p; ++n) {
    out[slot(n, 0)] = c[slot(n, 0)].real();
    for (int m = 1; m <= n; ++m) {
      out[slot(n, m)] = c[slot(n, m)].real();
      out[slot(n, -m)] = c[slot(n, m)].imag();
    }
  }
}

// ---------------------------------------------------------------------------
// interaction list: for a cell of octant c (c_k = coordinate & 1), the 189
// offsets o with -2-c_k <= o_k <= 3-c_k and max |o_k| >= 2 (children of the
// parent's 27-cell neighbourhood minus the cell's own 27-cell neighbourhood,
// Sec. 3.1); all 316 distinct offsets are numbered for the operator table.
struct ILTables {
  std::vector<int8_t> off;      // 8 * 189 * 3
  std::vector<int16_t> off_id;  // 8 * 189 -> index into distinct
  std::vector<int8_t> distinct; // 316 * 3
};

inline ILTables build_il() {
  ILTables t;
  t.off.resize(8 * 189 * 3);
  t.off_id.resize(8 * 189);
  std::vector<int> ids(7 * 7 * 7, -1);
  for (int oc = 0; oc < 8; ++oc) {
    int c[3] = {oc & 1, (oc >> 1) & 1, (oc >> 2) & 1};
    int cnt = 0;
    for (int oz = -2 - c[2]; oz <= 3 - c[2]; ++oz)
      for (int oy = -2 - c[1]; oy <= 3 - c[1]; ++oy)
        for (int ox = -2 - c[0]; ox <= 3 - c[0]; ++ox) {
          int mx = std::abs(ox);
          if (std::abs(oy) > mx) mx = std::abs(oy);
          if (std::abs(oz) > mx) mx = std::abs(oz);
          if (mx < 2) continue;
          int key = (ox + 3) + 7 * ((oy + 3) + 7 * (oz + 3));
          if (ids[key] < 0) {
            ids[key] = int(t.distinct.size() / 3);
            t.distinct.push_back(int8_t(ox));
            t.distinct.push_back(int8_t(oy));
            t.distinct.push_back(int8_t(oz));
          }
          t.off[(oc * 189 + cnt) * 3 + 0] = int8_t(ox);
          t.off[(oc * 189 + cnt) * 3 + 1] = int8_t(oy);
          t.off[(oc * 189 + cnt) * 3 + 2] = int8_t(oz);
          t.off_id[oc * 189 + cnt] = int16_t(ids[key]);
          ++cnt;
        }
  }
  return t;
}

// ---------------------------------------------------------------------------
// M2L, scaled: target centre minus source centre t = -o (in cells).
//   L~_k^l = sum_{n,m} M~_n^m (-1)^k i^{|m-l|-|m|-|l|} I_{n+k}^{m-l}(t)
// with M~ = M / N, L~ = N L; in scaled form the operator is the same on
// every level. Out: real C x C matrix, element [in s][out j] (k-major).
inline void m2l_operator(int p, const int o[3], double *Tkj) {
  int C = (p + 1) * (p + 1), P2 = 2 * p;
  std::vector<cd> Ivec, Lc(C);
  solid_I(P2, -double(o[0]), -double(o[1]), -double(o[2]), Ivec);
  std::vector<double> col(C);
  BasisEntry be[2];
  for (int s = 0; s < C; ++s) {
    int ne = basis_entries(s, be);
    for (int k = 0; k <= p; ++k)
      for (int l = -k; l <= k; ++l) {
        cd acc(0, 0);
        double sg = (k % 2 == 0) ? 1.0 : -1.0;
        for (int e = 0; e < ne; ++e) {
          int n = be[e].n, m = be[e].m;
          acc += be[e].v / Nnm(n, m) * sg * ipow(std::abs(m - l) - std::abs(m) - std::abs(l)) *
                 Ivec[slot(n + k, m - l)];
        }
        Lc[slot(k, l)] = acc / Nnm(k, l);
      }
    to_real(p, Lc, col.data());
    for (int j = 0; j < C; ++j) Tkj[size_t(s) * C + j] = col[j];
  }
}

// M2M, scaled: child of octant oc (child centre - parent centre = d h_parent,
// d_k = oc_k/2 - 1/4):
//   M~P_n^m = sum_{k,l} i^{|l|+|l-m|-|m|} M~C_k^l R_{n-k}^{l-m}(c_C - c_P)
// Out: real C x C, element [in s][out j].
inline void m2m_operator(int p, int oc, double *Tkj) {
  int C = (p + 1) * (p + 1);
  double d[3] = {0.5 * (oc & 1) - 0.25, 0.5 * ((oc >> 1) & 1) - 0.25, 0.5 * ((oc >> 2) & 1) - 0.25};
  std::vector<cd> R, Mp(C);
  solid_R(p, d[0], d[1], d[2], R);
  std::vector<double> col(C);
  BasisEntry be[2];
  for (int s = 0; s < C; ++s) {
    int ne = basis_entries(s, be);
    for (int n = 0; n <= p; ++n)
      for (int m = -n; m <= n; ++m) {
        cd acc(0, 0);
        for (int e = 0; e < ne; ++e) {
          int k = be[e].n, l = be[e].m;
          if (k > n || std::abs(l - m) > n - k) continue;
          // child coefficients are scaled by the child size h/2: M~ = M^ (h/2)^k / N
          acc += ipow(std::abs(l) + std::abs(l - m) - std::abs(m)) * be[e].v / Nnm(k, l) *
                 std::pow(0.5, k) * R[slot(n - k, l - m)];
        }
        Mp[slot(n, m)] = acc * Nnm(n, m);
      }
    to_real(p, Mp, col.data());
    for (int j = 0; j < C; ++j) Tkj[size_t(s) * C + j] = col[j];
  }
}

// ---------------------------------------------------------------------------
// Far-image lattice sums of the unit cube, Z_L^mu = sum_{max|nu_k|>=2}
// T_L^mu(nu) / |nu|^{2L+1}, by the incomplete-gamma split of 1/|nu|^{2L+1} at
// t = eta:
//   sum' T(v)/|v|^{2L+1} = Gamma(L+1/2)^{-1} [ sum'_v T(v) Gamma(L+1/2, eta v^2)/|v|^{2L+1}
//                        + pi^{L-1/2} (-i)^L sum'_k T(k) exp(-pi^2 k^2/eta)/k^2 ]
// minus the 26 images with max|nu_k| = 1. Degrees L <= 2 are zero (neutral
// cell; inversion; cube-order summation leaves no L = 2 term by cubic
// symmetry); odd L and mu not divisible by 4 vanish by the cube's inversion
// and four-fold symmetry and are set to exactly zero.
inline double upper_gamma_half_int(int L, double x) {
  double g = std::sqrt(M_PI) * std::erfc(std::sqrt(x));
  double s = 0.5;
  for (int i = 0; i < L; ++i) {
    g = s * g + std::pow(x, s) * std::exp(-x);
    s += 1.0;
  }
  return g;
}

inline void lattice_sums(int Lmax, std::vector<cd> &Z) {
  int C = (Lmax + 1) * (Lmax + 1);
  const double eta = 2.5;
  const int cut = 10;
  std::vector<cd> real(C, 0.0), recip(C, 0.0), nearv(C, 0.0), T;
  for (int x = -cut; x <= cut; ++x)
    for (int y = -cut; y <= cut; ++y)
      for (int z = -cut; z <= cut; ++z) {
        if (!x && !y && !z) continue;
        int r2i = x * x + y * y + z * z;
        if (r2i > cut * cut) continue;
        double r2 = double(r2i), r = std::sqrt(r2);
        solid_T(Lmax, x, y, z, T);
        bool nearshell = std::abs(x) <= 1 && std::abs(y) <= 1 && std::abs(z) <= 1;
        for (int L = 3; L <= Lmax; ++L) {
          double gr = upper_gamma_half_int(L, eta * r2) / std::pow(r, 2 * L + 1);
          double gk = std::exp(-M_PI * M_PI * r2 / eta) / r2;
          double gn = 1.0 / std::pow(r, 2 * L + 1);
          for (int mu = -L; mu <= L; ++mu) {
            cd t = T[slot(L, mu)];
            real[slot(L, mu)] += t * gr;
            recip[slot(L, mu)] += t * gk;
            if (nearshell) nearv[slot(L, mu)] += t * gn;
          }
        }
      }
  Z.assign(C, cd(0, 0));
  for (int L = 4; L <= Lmax; L += 2) {
    double g = std::tgamma(L + 0.5);
    cd pref = std::pow(M_PI, L - 0.5) * ipow(-L);
    for (int mu = -L; mu <= L; ++mu) {
      if (((mu % 4) + 4) % 4 != 0) continue;
      cd full = (real[slot(L, mu)] + pref * recip[slot(L, mu)]) / g;
      cd v = full - nearv[slot(L, mu)];
      Z[slot(L, mu)] = cd(v.real(), 0.0);  // real by the cube's mirror symmetries
    }
  }
}

// Lattice operator, scaled by the box size: the far images of the box are
// M2L sources at centre offsets nu (target minus source = -nu), so it is the
// M2L operator with I_{n+k}^{m-l}(t) replaced by its lattice sum
// sum_far I(-nu) = N (-1)^{n+k} Z_{n+k}^{m-l}. Out: dense real C x C,
// element [out j][in s] (row-major by output).
inline void lattice_operator(int p, double *Rjs) {
  int C = (p + 1) * (p + 1), P2 = 2 * p;
  std::vector<cd> Z, Lc(C);
  lattice_sums(P2, Z);
  std::vector<double> col(C);
  BasisEntry be[2];
  for (int s = 0; s < C; ++s) {
    int ne = basis_entries(s, be);
    for (int k = 0; k <= p; ++k)
      for (int l = -k; l <= k; ++l) {
        cd acc(0, 0);
        double sg = (k % 2 == 0) ? 1.0 : -1.0;
        for (int e = 0; e < ne; ++e) {
          int n = be[e].n, m = be[e].m, Lt = n + k;
          cd Isum = Nnm(Lt, m - l) * ((Lt % 2 == 0) ? 1.0 : -1.0) * Z[slot(Lt, m - l)];
          acc += be[e].v / Nnm(n, m) * sg * ipow(std::abs(m - l) - std::abs(m) - std::abs(l)) * Isum;
        }
        Lc[slot(k, l)] = acc / Nnm(k, l);
      }
    to_real(p, Lc, col.data());
    for (int j = 0; j < C; ++j) Rjs[size_t(j) * C + s] = col[j];
  }
}

}  // namespace fmmhost
