/*
 * fmm_oracle.c -- plain, slow, CPU FP64 oracle of the multilevel
 * local-expansion method for Metropolis-Hastings Monte Carlo of point charges
 * in a periodic cube (Saunders, Grant & Mueller, arXiv:2006.16622, "A new
 * algorithm for electrostatic interactions in Monte Carlo simulations of
 * charged particles").
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check of the entry
 * module and the cpu_baseline leg of the benchmark may load this library. It
 * shares no code, header, table or constant with the GPU library; the two
 * meet only through the seeded input generators.
 *
 * Everything here follows the paper's text in its own order and notation:
 *   Y_n^m(th,ph) = sqrt((n-|m|)!/(n+|m|)!) P_n^{|m|}(cos th) e^{i m ph}
 *                  (no Condon-Shortley phase, so Y_n^{-m} = conj(Y_n^m);
 *                  the normalisation for which Eq. (local_expansion),
 *                  Eq. (multipole_expansion_coefficients) and Alg. L.2 use
 *                  Y_n^{-m} in the coefficients)
 *   multipole  M_n^m = sum_i q_i rho_i^n Y_n^{-m}          Eq. (multipole_expansion_coefficients)
 *   local      L_n^m = sum_i q_i rho_i^{-(n+1)} Y_n^{-m}   Alg. L.2, Alg. L.3
 *   Psi(dr)    = sum L_n^m rho^n Y_n^m                     Eq. (local_expansion)
 * A coefficient (n,m) lives at index n*n+n+m of a complex array of (p+1)^2
 * entries (m = -n..n, full storage: nothing is folded by symmetry).
 *
 * Translations (M2M, M2L, L2L) are the Greengard-Rokhlin translation
 * theorems the paper defers to for the FMM (Sec. 3.1); the periodic lattice
 * operator, whose defining reference is not available, is built as the M2L
 * operator summed over all image boxes outside the 27-box extended domain,
 * in cube (shell) order.
 *
 * Compile with gcc -O2, no fast-math, -ffp-contract=off: the wrap, cell
 * location, displacement and accept decision must round exactly as IEEE
 * double without contraction. With -fopenmp the cells of the M2L setup are
 * shared out over threads; each cell's sum is formed by one thread in the
 * same order, so every result is the same for any thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define IDX(n, m) ((n) * (n) + (n) + (m))

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */

/* n! for 0 <= n <= 170, tabulated on first use */
static double fact_tab[171];
static int fact_ready = 0;
static double fact(int n) {
  if (!fact_ready) {
    fact_tab[0] = 1.0;
    for (int i = 1; i <= 170; ++i) fact_tab[i] = fact_tab[i - 1] * (double)i;
    fact_ready = 1;
  }
  return fact_tab[n];
}

/* i^k for any integer k */
static cplx ipow(int k) {
  int r = ((k % 4) + 4) % 4;
  if (r == 0) return 1.0;
  if (r == 1) return I;
  if (r == 2) return -1.0;
  return -I;
}

/* A_n^m = (-1)^n / sqrt((n-m)!(n+m)!)  (Greengard-Rokhlin) */
static double Acoef(int n, int m) {
  double s = (n % 2 == 0) ? 1.0 : -1.0;
  return s / sqrt(fact(n - m) * fact(n + m));
}

/* spherical coordinates (r, theta, phi) of a vector: the function
 * "spherical" of Sec. 3.2 */
static void spherical(const double v[3], double *r, double *th, double *ph) {
  *r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  if (*r == 0.0) {
    *th = 0.0;
    *ph = 0.0;
    return;
  }
  double c = v[2] / *r;
  if (c > 1.0) c = 1.0;
  if (c < -1.0) c = -1.0;
  *th = acos(c);
  *ph = atan2(v[1], v[0]);
}

/* Y_n^m(th, ph) for 0 <= n <= nmax, -n <= m <= n, written to Y[IDX(n,m)].
 * Associated Legendre functions without Condon-Shortley phase from the
 * three-term recurrence in n:
 *   P_m^m = (2m-1)!! sin^m,  P_{m+1}^m = (2m+1) cos P_m^m,
 *   (n-m) P_n^m = (2n-1) cos P_{n-1}^m - (n+m-1) P_{n-2}^m. */
void orc_ylm(int nmax, double th, double ph, double *Yout) {
  cplx *Y = (cplx *)Yout;
  double x = cos(th), s = sin(th);
  int C = (nmax + 1) * (nmax + 1);
  double *P = (double *)calloc((size_t)C, sizeof(double));
  double pmm = 1.0;
  for (int m = 0; m <= nmax; ++m) {
    if (m > 0) pmm *= (2.0 * m - 1.0) * s;
    P[IDX(m, m)] = pmm;
    if (m + 1 <= nmax) P[IDX(m + 1, m)] = x * (2.0 * m + 1.0) * pmm;
    for (int n = m + 2; n <= nmax; ++n)
      P[IDX(n, m)] = ((2.0 * n - 1.0) * x * P[IDX(n - 1, m)] -
                      (n + m - 1.0) * P[IDX(n - 2, m)]) / (double)(n - m);
  }
  for (int n = 0; n <= nmax; ++n) {
    for (int m = 0; m <= n; ++m) {
      double nrm = sqrt(fact(n - m) / fact(n + m));
      cplx v = nrm * P[IDX(n, m)] * cexp(I * (double)m * ph);
      Y[IDX(n, m)] = v;
      Y[IDX(n, -m)] = conj(v);
    }
  }
  free(P);
}

/* ------------------------------------------------------------------ */
/* expansion operators                                                  */
/* ------------------------------------------------------------------ */

/* P2M, Eq. (multipole_expansion_coefficients): M_n^m += q rho^n Y_n^{-m}(s-c) */
void orc_p2m(int p, double q, const double *s, const double *c, double *Mout) {
  cplx *M = (cplx *)Mout;
  double v[3] = {s[0] - c[0], s[1] - c[1], s[2] - c[2]}, r, th, ph;
  spherical(v, &r, &th, &ph);
  cplx *Y = (cplx *)malloc(sizeof(cplx) * (p + 1) * (p + 1));
  orc_ylm(p, th, ph, (double *)Y);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) M[IDX(n, m)] += q * pow(r, n) * Y[IDX(n, -m)];
  free(Y);
}

/* the "E" moments of the periodic modification (Sec. 3.4):
 * E_n^m += q rho^n Y_n^{m}(s-c) */
void orc_p2e(int p, double q, const double *s, const double *c, double *Eout) {
  cplx *E = (cplx *)Eout;
  double v[3] = {s[0] - c[0], s[1] - c[1], s[2] - c[2]}, r, th, ph;
  spherical(v, &r, &th, &ph);
  cplx *Y = (cplx *)malloc(sizeof(cplx) * (p + 1) * (p + 1));
  orc_ylm(p, th, ph, (double *)Y);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) E[IDX(n, m)] += q * pow(r, n) * Y[IDX(n, m)];
  free(Y);
}

/* P2L, the update of Alg. L.2 / L.3: L_n^m += q rho^{-(n+1)} Y_n^{-m}(s-c) */
void orc_p2l(int p, double q, const double *s, const double *c, double *Lout) {
  cplx *L = (cplx *)Lout;
  double v[3] = {s[0] - c[0], s[1] - c[1], s[2] - c[2]}, r, th, ph;
  spherical(v, &r, &th, &ph);
  cplx *Y = (cplx *)malloc(sizeof(cplx) * (p + 1) * (p + 1));
  orc_ylm(p, th, ph, (double *)Y);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m)
      L[IDX(n, m)] += q * pow(r, -(n + 1)) * Y[IDX(n, -m)];
  free(Y);
}

/* L2P, Eq. (local_expansion): Psi(x-c) = sum L_n^m rho^n Y_n^m */
double orc_l2p(int p, const double *Lin, const double *x, const double *c) {
  const cplx *L = (const cplx *)Lin;
  double v[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]}, r, th, ph;
  spherical(v, &r, &th, &ph);
  cplx *Y = (cplx *)malloc(sizeof(cplx) * (p + 1) * (p + 1));
  orc_ylm(p, th, ph, (double *)Y);
  cplx acc = 0.0;
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) acc += L[IDX(n, m)] * pow(r, n) * Y[IDX(n, m)];
  free(Y);
  return creal(acc);
}

/* M2P, Eq. (multipole_expansion): Phi(x-c) = sum M_n^m rho^{-(n+1)} Y_n^m */
double orc_m2p(int p, const double *Min, const double *x, const double *c) {
  const cplx *M = (const cplx *)Min;
  double v[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]}, r, th, ph;
  spherical(v, &r, &th, &ph);
  cplx *Y = (cplx *)malloc(sizeof(cplx) * (p + 1) * (p + 1));
  orc_ylm(p, th, ph, (double *)Y);
  cplx acc = 0.0;
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) acc += M[IDX(n, m)] * pow(r, -(n + 1)) * Y[IDX(n, m)];
  free(Y);
  return creal(acc);
}

/* M2M (Greengard-Rokhlin): a multipole expansion O about centre Q is
 * re-expanded about the origin; d = Q - (new centre). Result added to M. */
void orc_m2m(int p, const double *Oin, const double *d, double *Mout) {
  const cplx *O = (const cplx *)Oin;
  cplx *M = (cplx *)Mout;
  double rho, al, be;
  spherical(d, &rho, &al, &be);
  cplx *Y = (cplx *)malloc(sizeof(cplx) * (p + 1) * (p + 1));
  orc_ylm(p, al, be, (double *)Y);
  for (int j = 0; j <= p; ++j)
    for (int k = -j; k <= j; ++k) {
      cplx s = 0.0;
      for (int n = 0; n <= j; ++n)
        for (int m = -n; m <= n; ++m) {
          if (abs(k - m) > j - n) continue;
          s += O[IDX(j - n, k - m)] * ipow(abs(k) - abs(m) - abs(k - m)) *
               Acoef(n, m) * Acoef(j - n, k - m) * pow(rho, n) * Y[IDX(n, -m)] /
               Acoef(j, k);
        }
      M[IDX(j, k)] += s;
    }
  free(Y);
}

/* constant factor of the Greengard-Rokhlin M2L theorem,
 *   i^{|k-m|-|k|-|m|} A_n^m A_j^k / ((-1)^n A_{j+n}^{m-k}),
 * tabulated for one p at a time as a (p+1)^2 x (p+1)^2 table */
static cplx *m2l_tab = NULL;
static int m2l_tab_p = -1;
static const cplx *m2l_const_table(int p) {
  if (m2l_tab_p == p) return m2l_tab;
  int C = (p + 1) * (p + 1);
  free(m2l_tab);
  m2l_tab = (cplx *)malloc(sizeof(cplx) * C * C);
  for (int j = 0; j <= p; ++j)
    for (int k = -j; k <= j; ++k)
      for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m) {
          double sg = (n % 2 == 0) ? 1.0 : -1.0;
          m2l_tab[(size_t)IDX(j, k) * C + IDX(n, m)] =
              ipow(abs(k - m) - abs(k) - abs(m)) * Acoef(n, m) * Acoef(j, k) /
              (sg * Acoef(j + n, m - k));
        }
  m2l_tab_p = p;
  return m2l_tab;
}

/* M2L (Greengard-Rokhlin): a multipole expansion O about a source centre
 * is converted into a local expansion about a target centre; d = source
 * centre - target centre. Result added to L:
 *   L_j^k += sum_{n,m} O_n^m [const(j,k,n,m)] Y_{j+n}^{m-k}(d^) / |d|^{j+n+1} */
void orc_m2l(int p, const double *Oin, const double *d, double *Lout) {
  const cplx *O = (const cplx *)Oin;
  cplx *L = (cplx *)Lout;
  double rho, al, be;
  spherical(d, &rho, &al, &be);
  int P2 = 2 * p, C = (p + 1) * (p + 1);
  cplx *Y = (cplx *)malloc(sizeof(cplx) * (P2 + 1) * (P2 + 1));
  orc_ylm(P2, al, be, (double *)Y);
  for (int l = 0; l <= P2; ++l)
    for (int mu = -l; mu <= l; ++mu) Y[IDX(l, mu)] /= pow(rho, l + 1);
  const cplx *T = m2l_const_table(p);
  for (int j = 0; j <= p; ++j)
    for (int k = -j; k <= j; ++k) {
      cplx s = 0.0;
      const cplx *Trow = &T[(size_t)IDX(j, k) * C];
      for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m)
          s += O[IDX(n, m)] * Trow[IDX(n, m)] * Y[IDX(j + n, m - k)];
      L[IDX(j, k)] += s;
    }
  free(Y);
}

/* L2L (Greengard-Rokhlin): a local expansion O about centre Q is
 * re-expanded about the origin; d = Q - (new centre). Result added to L.
 * Not on the method's path (the per-level expansions are never pushed
 * down, Sec. 3.2); kept as a check of the harmonic conventions. */
void orc_l2l(int p, const double *Oin, const double *d, double *Lout) {
  const cplx *O = (const cplx *)Oin;
  cplx *L = (cplx *)Lout;
  double rho, al, be;
  spherical(d, &rho, &al, &be);
  cplx *Y = (cplx *)malloc(sizeof(cplx) * (p + 1) * (p + 1));
  orc_ylm(p, al, be, (double *)Y);
  for (int j = 0; j <= p; ++j)
    for (int k = -j; k <= j; ++k) {
      cplx s = 0.0;
      for (int n = j; n <= p; ++n)
        for (int m = -n; m <= n; ++m) {
          if (abs(m - k) > n - j) continue;
          double sg = ((n + j) % 2 == 0) ? 1.0 : -1.0;
          s += O[IDX(n, m)] * ipow(abs(m) - abs(m - k) - abs(k)) *
               Acoef(n - j, m - k) * Acoef(j, k) * pow(rho, n - j) *
               Y[IDX(n - j, m - k)] / (sg * Acoef(n, m));
        }
      L[IDX(j, k)] += s;
    }
  free(Y);
}

/* ------------------------------------------------------------------ */
/* geometry (Sec. 3.1, Sec. 3.4)                                        */
/* ------------------------------------------------------------------ */

/* Interaction list of a cell, straight from its definition (Sec. 3.1):
 * IL(alpha) = children(N_b(parent(alpha))) \ (alpha u N_b(alpha)).
 * With alpha = 2 P + oct (oct in {0,1}^3) placed at the origin, the
 * children of parent-neighbour P+e are 2(P+e)+c, i.e. at offsets
 * 2e + c - oct from alpha; alpha and its 26 neighbours are the offsets
 * with max |o_k| <= 1. Offsets are written to out[3*i..]; returns count. */
int orc_il_offsets(const int *oct, int *out) {
  int cnt = 0;
  for (int ex = -1; ex <= 1; ++ex)
    for (int ey = -1; ey <= 1; ++ey)
      for (int ez = -1; ez <= 1; ++ez)
        for (int cx = 0; cx <= 1; ++cx)
          for (int cy = 0; cy <= 1; ++cy)
            for (int cz = 0; cz <= 1; ++cz) {
              int o[3] = {2 * ex + cx - oct[0], 2 * ey + cy - oct[1],
                          2 * ez + cz - oct[2]};
              int mx = abs(o[0]);
              if (abs(o[1]) > mx) mx = abs(o[1]);
              if (abs(o[2]) > mx) mx = abs(o[2]);
              if (mx >= 2) {
                out[3 * cnt + 0] = o[0];
                out[3 * cnt + 1] = o[1];
                out[3 * cnt + 2] = o[2];
                ++cnt;
              }
            }
  return cnt;
}

/* wrap a coordinate into [0, a): x - a floor(x/a); a result equal to a is
 * mapped to 0 */
double orc_wrap(double x, double a) {
  double w = x - a * floor(x / a);
  if (w >= a) w = 0.0;
  if (w < 0.0) w = 0.0;
  return w;
}

/* integer cell coordinate of x on a level with n cells per side:
 * floor(x * (n/a)), clamped to [0, n-1]; a point on a face belongs to the
 * upper cell */
int orc_cell_coord(double x, double a, int n) {
  double inv = (double)n / a;
  int i = (int)floor(x * inv);
  if (i < 0) i = 0;
  if (i > n - 1) i = n - 1;
  return i;
}

static int imod(int i, int n) { return ((i % n) + n) % n; }
static int ifloordiv(int i, int n) { return (i - imod(i, n)) / n; }

/* ------------------------------------------------------------------ */
/* periodic lattice sums (Sec. 3.4)                                     */
/* ------------------------------------------------------------------ */

/* upper incomplete gamma Gamma(l+1/2, x) by Gamma(1/2,x) = sqrt(pi) erfc(sqrt x)
 * and Gamma(s+1,x) = s Gamma(s,x) + x^s e^{-x} */
static double upper_gamma_half(int l, double x) {
  double g = sqrt(M_PI) * erfc(sqrt(x));
  double s = 0.5;
  for (int i = 0; i < l; ++i) {
    g = s * g + pow(x, s) * exp(-x);
    s += 1.0;
  }
  return g;
}

/* Lattice sums over the far images: for 0 <= l <= lmax, |mu| <= l,
 *   S_l^mu = sum_{nu in Z^3, max|nu_k| >= 2} Y_l^mu(nu^) / |a nu|^{l+1}
 * (cube order). The full sum over nu != 0 is taken by the incomplete-gamma
 * split of 1/|nu|^{2l+1} with the solid harmonic h_l(nu) = |nu|^l Y_l^mu:
 *   sum' h_l(v)/|v|^{2l+1} = Gamma(l+1/2)^{-1} [ sum'_v h_l(v) Gamma(l+1/2, pi v^2)/|v|^{2l+1}
 *                         + pi^{l-1/2} (-i)^l sum'_k h_l(k) e^{-pi k^2}/k^2 ]
 * (Poisson summation of h_l(x) e^{-t x^2}), then the 26 images with
 * max|nu_k| = 1 are removed. For l <= 2 the value is set to zero: l = 0
 * multiplies the total charge (zero, neutral cell), l = 1 vanishes by
 * inversion symmetry, and l = 2 vanishes for cube-order summation by cubic
 * symmetry. Output S[IDX(l,mu)], complex. */
void orc_lattice_sums(int lmax, double a, int cut, double *Sout) {
  cplx *S = (cplx *)Sout;
  int C = (lmax + 1) * (lmax + 1);
  for (int i = 0; i < C; ++i) S[i] = 0.0;
  cplx *Y = (cplx *)malloc(sizeof(cplx) * C);
  cplx *real_part = (cplx *)calloc((size_t)C, sizeof(cplx));
  cplx *recip_part = (cplx *)calloc((size_t)C, sizeof(cplx));
  cplx *near_part = (cplx *)calloc((size_t)C, sizeof(cplx));
  for (int x = -cut; x <= cut; ++x)
    for (int y = -cut; y <= cut; ++y)
      for (int z = -cut; z <= cut; ++z) {
        if (x == 0 && y == 0 && z == 0) continue;
        double v[3] = {(double)x, (double)y, (double)z}, r, th, ph;
        if (x * x + y * y + z * z > cut * cut) continue;
        spherical(v, &r, &th, &ph);
        orc_ylm(lmax, th, ph, (double *)Y);
        int nearshell = (abs(x) <= 1 && abs(y) <= 1 && abs(z) <= 1);
        for (int l = 0; l <= lmax; ++l) {
          double gr = upper_gamma_half(l, M_PI * r * r) / pow(r, l + 1);
          double gk = exp(-M_PI * r * r) * pow(r, l) / (r * r);
          for (int mu = -l; mu <= l; ++mu) {
            real_part[IDX(l, mu)] += Y[IDX(l, mu)] * gr;
            recip_part[IDX(l, mu)] += Y[IDX(l, mu)] * gk;
            if (nearshell) near_part[IDX(l, mu)] += Y[IDX(l, mu)] / pow(r, l + 1);
          }
        }
      }
  for (int l = 3; l <= lmax; ++l) {
    double gl = tgamma(l + 0.5);
    cplx pref = pow(M_PI, l - 0.5) * ipow(-l);
    for (int mu = -l; mu <= l; ++mu) {
      cplx full = (real_part[IDX(l, mu)] + pref * recip_part[IDX(l, mu)]) / gl;
      S[IDX(l, mu)] = (full - near_part[IDX(l, mu)]) / pow(a, l + 1);
    }
  }
  free(Y);
  free(real_part);
  free(recip_part);
  free(near_part);
}

/* the lattice operator: H = R(K), the M2L operator of Greengard-Rokhlin
 * with Y_{j+n}^{m-k}(d)/|d|^{j+n+1} replaced by the far-image lattice sum
 * S_{j+n}^{m-k} (source boxes at a nu, target box at the origin) */
void orc_lattice_apply(int p, const double *Sin, const double *Kin, double *Hout) {
  const cplx *S = (const cplx *)Sin;
  const cplx *K = (const cplx *)Kin;
  cplx *H = (cplx *)Hout;
  int C = (p + 1) * (p + 1);
  const cplx *T = m2l_const_table(p);
  for (int j = 0; j <= p; ++j)
    for (int k = -j; k <= j; ++k) {
      cplx s = 0.0;
      const cplx *Trow = &T[(size_t)IDX(j, k) * C];
      for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m) s += K[IDX(n, m)] * Trow[IDX(n, m)] * S[IDX(j + n, m - k)];
      H[IDX(j, k)] = s;
    }
}

/* self-image constant of the periodic self-interaction correction (Sec. 3.4):
 * sum over the 26 nearest images of 1/|nu| = 6 + 12/sqrt2 + 8/sqrt3 */
double orc_self_image_constant(void) {
  return 6.0 + 8.0 / sqrt(3.0) + 12.0 / sqrt(2.0);
}

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11)                   */
/* ------------------------------------------------------------------ */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 prod = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(prod >> 64);
  *lo = (uint64_t)prod;
}

void orc_philox4x64_10(const uint64_t *ctr, const uint64_t *key, uint64_t *out) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, x0, &hi0, &lo0);
    mulhilo64(M1, x2, &hi1, &lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* the proposal stream of one MH step: key (seed, chain), counter (step, s, 0, 0).
 * Stream 0: idx = floor(w0 * N / 2^64), displacement component k from w_k,
 *   delta_k = D * (2 * ((w_k >> 11) * 2^-53) - 1), k = 1..3.
 * Stream 1: u = (w0 >> 11) * 2^-53. */
void orc_draw(uint64_t seed, uint64_t chain, uint64_t step, int64_t N, double D,
              int64_t *idx, double *delta, double *u) {
  uint64_t key[2] = {seed, chain}, c0[4] = {step, 0, 0, 0}, c1[4] = {step, 1, 0, 0};
  uint64_t w[4], v[4];
  orc_philox4x64_10(c0, key, w);
  orc_philox4x64_10(c1, key, v);
  uint64_t hi, lo;
  mulhilo64(w[0], (uint64_t)N, &hi, &lo);
  *idx = (int64_t)hi;
  const double two53 = 1.0 / 9007199254740992.0;
  for (int k = 0; k < 3; ++k) {
    double f = (double)(w[k + 1] >> 11) * two53;
    delta[k] = D * (2.0 * f - 1.0);
  }
  *u = (double)(v[0] >> 11) * two53;
}

/* ------------------------------------------------------------------ */
/* the multilevel state                                                 */
/* ------------------------------------------------------------------ */

typedef struct {
  int n, cap;
  int *ids;
} cell_list;

typedef struct {
  double pos[3];
  double newpos[3];
  double q;
} move_rec;

typedef struct {
  int N, d, L, p, C;
  double a;
  double *pos; /* 3N, wrapped into [0,a) */
  double *q;   /* N */
  int *leaf_of;
  cell_list *leaf; /* nL^3 lists of particle ids */
  cplx **Ld;       /* Ld[l], l = 2..L: per-level IL-only local expansions, n_l^3 * C */
  unsigned char **ready; /* lazy mode: Ld[l][cell] is valid */
  cplx **Mp;       /* lazy mode: multipoles of the initial state, levels 2..L */
  cplx *K, *E;     /* lattice moments about the box centre (Sec. 3.4) */
  cplx *S;         /* lattice sums, degree <= 2p */
  double dip[3];   /* dipole sum q_i r_i (wrapped positions) */
  int lazy;
  int multipole;   /* the multipole-based variant of Sec. 3.3: Mp is the live state */
  int free_space;  /* free-space boundary conditions (Sec. 3.4): no images, no lattice */
  move_rec *log;   /* lazy mode: accepted moves since setup */
  int nlog, caplog;
} orc_t;

static int nside(int l) { return 1 << (l - 1); }

static void cell_centre(const orc_t *st, int l, const int *c, double *R) {
  double h = st->a / (double)nside(l);
  for (int k = 0; k < 3; ++k) R[k] = ((double)c[k] + 0.5) * h;
}

static int cell_lin(int n, const int *c) { return c[0] + n * (c[1] + n * c[2]); }

/* is the (unwrapped) cell b of a level with n cells per side a cell of the
 * box itself? Under free-space boundary conditions the box is the whole
 * domain: a cell outside it holds nothing. */
static int in_box(int n, const int *b) {
  return b[0] >= 0 && b[0] < n && b[1] >= 0 && b[1] < n && b[2] >= 0 && b[2] < n;
}

/* does x lie in the box [0,a)^3? */
static int point_in_box(const double *x, double a) {
  return x[0] >= 0.0 && x[0] < a && x[1] >= 0.0 && x[1] < a && x[2] >= 0.0 && x[2] < a;
}

static void locate(const orc_t *st, int l, const double *x, int *c) {
  int n = nside(l);
  for (int k = 0; k < 3; ++k) c[k] = orc_cell_coord(x[k], st->a, n);
}

static void list_add(cell_list *cl, int id) {
  if (cl->n == cl->cap) {
    cl->cap = cl->cap ? 2 * cl->cap : 4;
    cl->ids = (int *)realloc(cl->ids, sizeof(int) * cl->cap);
  }
  cl->ids[cl->n++] = id;
}

static void list_remove(cell_list *cl, int id) {
  for (int i = 0; i < cl->n; ++i)
    if (cl->ids[i] == id) {
      for (int j = i + 1; j < cl->n; ++j) cl->ids[j - 1] = cl->ids[j];
      cl->n--;
      return;
    }
}

/* create the state; positions are wrapped into [0,a)^3. d is the octree
 * depth, so L = d+1 levels with 8^(l-1) cells on level l (Sec. 3.1). */
orc_t *orc_create(int N, const double *pos, const double *q, double a, int d, int p) {
  orc_t *st = (orc_t *)calloc(1, sizeof(orc_t));
  st->N = N;
  st->d = d;
  st->L = d + 1;
  st->p = p;
  st->C = (p + 1) * (p + 1);
  st->a = a;
  st->pos = (double *)malloc(sizeof(double) * 3 * (N > 0 ? N : 1));
  st->q = (double *)malloc(sizeof(double) * (N > 0 ? N : 1));
  st->leaf_of = (int *)malloc(sizeof(int) * (N > 0 ? N : 1));
  int nL = nside(st->L);
  st->leaf = (cell_list *)calloc((size_t)nL * nL * nL, sizeof(cell_list));
  for (int i = 0; i < N; ++i) {
    for (int k = 0; k < 3; ++k) st->pos[3 * i + k] = orc_wrap(pos[3 * i + k], a);
    st->q[i] = q[i];
    int c[3];
    locate(st, st->L, &st->pos[3 * i], c);
    st->leaf_of[i] = cell_lin(nL, c);
    list_add(&st->leaf[st->leaf_of[i]], i);
  }
  st->Ld = (cplx **)calloc((size_t)st->L + 1, sizeof(cplx *));
  st->ready = (unsigned char **)calloc((size_t)st->L + 1, sizeof(unsigned char *));
  st->Mp = (cplx **)calloc((size_t)st->L + 1, sizeof(cplx *));
  for (int l = 2; l <= st->L; ++l) {
    size_t nc = (size_t)nside(l) * nside(l) * nside(l);
    st->Ld[l] = (cplx *)calloc(nc * st->C, sizeof(cplx));
    st->ready[l] = (unsigned char *)calloc(nc, 1);
  }
  st->K = (cplx *)calloc((size_t)st->C, sizeof(cplx));
  st->E = (cplx *)calloc((size_t)st->C, sizeof(cplx));
  st->S = (cplx *)calloc((size_t)(2 * p + 1) * (2 * p + 1), sizeof(cplx));
  return st;
}

/* Free-space boundary conditions (Sec. 3.4): the box [0,a)^3 is the whole
 * domain. Interaction lists and near regions keep only cells inside the box
 * (so the lists of levels 1 and 2 are empty), the self correction keeps only
 * the charge's own old position, and there is no lattice or tin-foil term.
 * Positions are not wrapped; a move out of the box has dE = +inf. To be
 * called right after orc_create, before any setup, with every position
 * inside the box. */
void orc_set_free_space(orc_t *st) { st->free_space = 1; }

void orc_destroy(orc_t *st) {
  if (!st) return;
  int nL = nside(st->L);
  for (int i = 0; i < nL * nL * nL; ++i) free(st->leaf[i].ids);
  free(st->leaf);
  for (int l = 0; l <= st->L; ++l) {
    free(st->Ld[l]);
    free(st->ready[l]);
    free(st->Mp[l]);
  }
  free(st->Ld);
  free(st->ready);
  free(st->Mp);
  free(st->K);
  free(st->E);
  free(st->S);
  free(st->pos);
  free(st->q);
  free(st->leaf_of);
  free(st->log);
  free(st);
}

/* K and E moments about the box centre R_1, and the dipole (Sec. 3.4) */
static void init_lattice(orc_t *st) {
  double R1[3] = {0.5 * st->a, 0.5 * st->a, 0.5 * st->a};
  memset(st->K, 0, sizeof(cplx) * st->C);
  memset(st->E, 0, sizeof(cplx) * st->C);
  st->dip[0] = st->dip[1] = st->dip[2] = 0.0;
  for (int i = 0; i < st->N; ++i) {
    orc_p2m(st->p, st->q[i], &st->pos[3 * i], R1, (double *)st->K);
    orc_p2e(st->p, st->q[i], &st->pos[3 * i], R1, (double *)st->E);
    for (int k = 0; k < 3; ++k) st->dip[k] += st->q[i] * st->pos[3 * i + k];
  }
  if (!st->free_space) orc_lattice_sums(2 * st->p, st->a, 12, (double *)st->S);
}

/* multipoles of every cell on levels 2..L: P2M on the leaves, then M2M
 * upwards (the upward pass of the FMM, Sec. 3.1) */
static void upward_pass(orc_t *st) {
  int C = st->C;
  for (int l = 2; l <= st->L; ++l) {
    size_t nc = (size_t)nside(l) * nside(l) * nside(l);
    free(st->Mp[l]);
    st->Mp[l] = (cplx *)calloc(nc * C, sizeof(cplx));
  }
  int nL = nside(st->L);
  for (int i = 0; i < st->N; ++i) {
    int c[3];
    locate(st, st->L, &st->pos[3 * i], c);
    double R[3];
    cell_centre(st, st->L, c, R);
    orc_p2m(st->p, st->q[i], &st->pos[3 * i], R, (double *)&st->Mp[st->L][(size_t)cell_lin(nL, c) * C]);
  }
  for (int l = st->L - 1; l >= 2; --l) {
    int n = nside(l + 1);
    for (int z = 0; z < n; ++z)
      for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
          int c[3] = {x, y, z}, pc[3] = {x >> 1, y >> 1, z >> 1};
          double Rc[3], Rp[3], dv[3];
          cell_centre(st, l + 1, c, Rc);
          cell_centre(st, l, pc, Rp);
          for (int k = 0; k < 3; ++k) dv[k] = Rc[k] - Rp[k];
          orc_m2m(st->p, (double *)&st->Mp[l + 1][(size_t)cell_lin(n, c) * C], dv,
                  (double *)&st->Mp[l][(size_t)cell_lin(n >> 1, pc) * C]);
        }
  }
}

/* L^Delta of one cell by M2L from the multipoles of its interaction list,
 * images included (Sec. 3.2 initialisation by the FMM passes; Sec. 3.4) */
static void m2l_cell(orc_t *st, int l, const int *c, cplx *out) {
  int n = nside(l), oct[3] = {c[0] & 1, c[1] & 1, c[2] & 1}, off[189 * 3];
  double h = st->a / (double)n;
  int cnt = orc_il_offsets(oct, off);
  for (int i = 0; i < cnt; ++i) {
    int b[3] = {c[0] + off[3 * i], c[1] + off[3 * i + 1], c[2] + off[3 * i + 2]};
    if (st->free_space && !in_box(n, b)) continue;
    int s[3] = {imod(b[0], n), imod(b[1], n), imod(b[2], n)};
    double dv[3] = {off[3 * i] * h, off[3 * i + 1] * h, off[3 * i + 2] * h};
    orc_m2l(st->p, (double *)&st->Mp[l][(size_t)cell_lin(n, s) * st->C], dv, (double *)out);
  }
}

/* the P2L contribution (with sign) of one charge at r to one stored cell,
 * summed over every image of that cell lying in IL(cell of r): Alg. L.2
 * with the extended domain of Sec. 3.4 */
static void p2l_into_cell(orc_t *st, int l, int target, double q, const double *r, cplx *out) {
  int n = nside(l), a[3], oct[3], off[189 * 3];
  locate(st, l, r, a);
  for (int k = 0; k < 3; ++k) oct[k] = a[k] & 1;
  int cnt = orc_il_offsets(oct, off);
  for (int i = 0; i < cnt; ++i) {
    int b[3] = {a[0] + off[3 * i], a[1] + off[3 * i + 1], a[2] + off[3 * i + 2]};
    if (st->free_space && !in_box(n, b)) continue;
    int s[3] = {imod(b[0], n), imod(b[1], n), imod(b[2], n)};
    if (cell_lin(n, s) != target) continue;
    double R[3];
    cell_centre(st, l, b, R);
    orc_p2l(st->p, q, r, R, (double *)out);
  }
}

/* access to L^Delta of a cell; in lazy mode it is formed on first use from
 * the setup multipoles plus every accepted move logged since setup */
static cplx *local_of(orc_t *st, int l, int lin) {
  cplx *Lc = &st->Ld[l][(size_t)lin * st->C];
  if (st->lazy && !st->ready[l][lin]) {
    int n = nside(l), c[3] = {lin % n, (lin / n) % n, lin / (n * n)};
    memset(Lc, 0, sizeof(cplx) * st->C);
    m2l_cell(st, l, c, Lc);
    for (int t = 0; t < st->nlog; ++t) {
      p2l_into_cell(st, l, lin, -st->log[t].q, st->log[t].pos, Lc);
      p2l_into_cell(st, l, lin, st->log[t].q, st->log[t].newpos, Lc);
    }
    st->ready[l][lin] = 1;
  }
  return Lc;
}

/* Initialisation by the FMM passes (the variant of Sec. 3.2 with no L2L):
 * P2M, M2M, then M2L over each interaction list on levels 2..L; plus the
 * periodic K/E moments and lattice sums (Sec. 3.4). lazy != 0 defers the
 * M2L of each cell to its first use. */
void orc_setup_fmm(orc_t *st, int lazy) {
  st->lazy = lazy;
  st->multipole = 0;
  st->nlog = 0;
  upward_pass(st);
  init_lattice(st);
  /* the shared tables are formed before the cells are spread over threads */
  (void)fact(0);
  (void)m2l_const_table(st->p);
  for (int l = 2; l <= st->L; ++l) {
    int n = nside(l);
    memset(st->ready[l], 0, (size_t)n * n * n);
    if (lazy) continue;
    /* every cell's M2L sum is independent and formed in the same order by
     * one thread, so the result does not depend on the thread count */
    const long ncell = (long)n * n * n;
#pragma omp parallel for schedule(dynamic, 4)
    for (long lin = 0; lin < ncell; ++lin) {
      int c[3] = {(int)(lin % n), (int)((lin / n) % n), (int)(lin / ((long)n * n))};
      cplx *Lc = &st->Ld[l][(size_t)lin * st->C];
      memset(Lc, 0, sizeof(cplx) * st->C);
      m2l_cell(st, l, c, Lc);
      st->ready[l][lin] = 1;
    }
  }
}

/* No initialisation of the expansions: every L^Delta is zero, only the
 * lattice moments are formed. The per-step cost of propose/accept does not
 * depend on the coefficient values, so this state serves to time the
 * oracle's steps on sizes whose initialisation would take too long on one
 * core; it is never compared against. */
void orc_setup_none(orc_t *st) {
  st->lazy = 0;
  st->multipole = 0;
  st->nlog = 0;
  init_lattice(st);
  for (int l = 2; l <= st->L; ++l) {
    size_t nc = (size_t)nside(l) * nside(l) * nside(l);
    memset(st->Ld[l], 0, sizeof(cplx) * nc * st->C);
    memset(st->ready[l], 1, nc);
  }
}

/* Initialisation by direct P2L, Alg. L.3 (the paper's own setup): on every
 * level, every charge is added to the local expansion of every cell in the
 * interaction list of its cell (images included, Sec. 3.4). */
void orc_setup_direct(orc_t *st) {
  st->lazy = 0;
  st->multipole = 0;
  st->nlog = 0;
  init_lattice(st);
  for (int l = 2; l <= st->L; ++l) {
    int n = nside(l);
    size_t nc = (size_t)n * n * n;
    memset(st->Ld[l], 0, sizeof(cplx) * nc * st->C);
    memset(st->ready[l], 1, nc);
    double h = st->a / (double)n;
    for (int i = 0; i < st->N; ++i) {
      int a[3], oct[3], off[189 * 3];
      locate(st, l, &st->pos[3 * i], a);
      for (int k = 0; k < 3; ++k) oct[k] = a[k] & 1;
      int cnt = orc_il_offsets(oct, off);
      for (int j = 0; j < cnt; ++j) {
        int b[3] = {a[0] + off[3 * j], a[1] + off[3 * j + 1], a[2] + off[3 * j + 2]};
        if (st->free_space && !in_box(n, b)) continue;
        int s[3] = {imod(b[0], n), imod(b[1], n), imod(b[2], n)};
        double R[3] = {(b[0] + 0.5) * h, (b[1] + 0.5) * h, (b[2] + 0.5) * h};
        orc_p2l(st->p, st->q[i], &st->pos[3 * i], R,
                (double *)&st->Ld[l][(size_t)cell_lin(n, s) * st->C]);
      }
    }
  }
}

/* Initialisation of the multipole-based variant (Sec. 3.3). With
 * upward == 0 it follows Alg. M.3: on every level 2..L, every charge is
 * added to the multipole expansion of its own cell, Eq.
 * (multipole_expansion_coefficients). With upward != 0 the same
 * coefficients come from the FMM upward pass (P2M on the leaves, then M2M),
 * which reproduces them up to rounding since M2M loses nothing at orders
 * <= p. Levels 1 and the lattice moments K, E are those of Sec. 3.4. */
void orc_setup_multipole(orc_t *st, int upward) {
  st->lazy = 0;
  st->nlog = 0;
  st->multipole = 1;
  if (upward) {
    upward_pass(st);
  } else {
    for (int l = 2; l <= st->L; ++l) {
      int n = nside(l);
      size_t nc = (size_t)n * n * n;
      free(st->Mp[l]);
      st->Mp[l] = (cplx *)calloc(nc * st->C, sizeof(cplx));
      for (int i = 0; i < st->N; ++i) {
        int c[3];
        double R[3];
        locate(st, l, &st->pos[3 * i], c);
        cell_centre(st, l, c, R);
        orc_p2m(st->p, st->q[i], &st->pos[3 * i], R, (double *)&st->Mp[l][(size_t)cell_lin(n, c) * st->C]);
      }
    }
  }
  init_lattice(st);
}

/* the far field of the multipole-based variant at x: on every level
 * l = 2..L, the multipole expansion of every cell (image) in the
 * interaction list of the cell of x, evaluated at x (the inner loop of
 * Alg. M.1, over the extended domain of Sec. 3.4) */
static double m2p_far(orc_t *st, const double *x) {
  double acc = 0.0;
  for (int l = st->L; l >= 2; --l) {
    int n = nside(l), a[3], oct[3], off[189 * 3];
    double h = st->a / (double)n;
    locate(st, l, x, a);
    for (int k = 0; k < 3; ++k) oct[k] = a[k] & 1;
    int cnt = orc_il_offsets(oct, off);
    for (int j = 0; j < cnt; ++j) {
      int b[3] = {a[0] + off[3 * j], a[1] + off[3 * j + 1], a[2] + off[3 * j + 2]};
      if (st->free_space && !in_box(n, b)) continue;
      int s[3] = {imod(b[0], n), imod(b[1], n), imod(b[2], n)};
      double R[3] = {(b[0] + 0.5) * h, (b[1] + 0.5) * h, (b[2] + 0.5) * h};
      acc += orc_m2p(st->p, (double *)&st->Mp[l][(size_t)cell_lin(n, s) * st->C], x, R);
    }
  }
  return acc;
}

/* sum of q_j / |x - r_j - a nu| over the particles of the 27 leaf cells
 * around the leaf cell of x (with their images, Alg. 1 with the extended
 * domain of Sec. 3.4); the pair (skip_id, every image) is left out when
 * skip_all_images, only (skip_id, nu = 0) otherwise. When skip_nu is
 * non-NULL it receives, for each nu in {-1,0,1}^3 (index (nx+1)+3(ny+1)+9(nz+1)),
 * whether the image skip_id + a nu lies in the near region. */
static double near_sum(orc_t *st, const double *x, int skip_id, int skip_all_images,
                       unsigned char *skip_nu) {
  int L = st->L, n = nside(L), c[3];
  locate(st, L, x, c);
  double acc = 0.0;
  if (skip_nu) memset(skip_nu, 0, 27);
  for (int ez = -1; ez <= 1; ++ez)
    for (int ey = -1; ey <= 1; ++ey)
      for (int ex = -1; ex <= 1; ++ex) {
        int b[3] = {c[0] + ex, c[1] + ey, c[2] + ez};
        if (st->free_space && !in_box(n, b)) continue;
        int s[3] = {imod(b[0], n), imod(b[1], n), imod(b[2], n)};
        int w[3] = {ifloordiv(b[0], n), ifloordiv(b[1], n), ifloordiv(b[2], n)};
        cell_list *cl = &st->leaf[cell_lin(n, s)];
        for (int t = 0; t < cl->n; ++t) {
          int j = cl->ids[t];
          int is_self = (j == skip_id);
          if (is_self && skip_nu) skip_nu[(w[0] + 1) + 3 * (w[1] + 1) + 9 * (w[2] + 1)] = 1;
          if (is_self && (skip_all_images || (w[0] == 0 && w[1] == 0 && w[2] == 0))) continue;
          double dv[3];
          for (int k = 0; k < 3; ++k) dv[k] = x[k] - (st->pos[3 * j + k] + st->a * w[k]);
          acc += st->q[j] / sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        }
      }
  return acc;
}

/* the far-lattice energy U^inf = 1/2 sum E_n^m H_n^m with H = R(K) */
static double lattice_energy(const orc_t *st, const cplx *K, const cplx *E) {
  cplx *H = (cplx *)malloc(sizeof(cplx) * st->C);
  orc_lattice_apply(st->p, (const double *)st->S, (const double *)K, (double *)H);
  cplx acc = 0.0;
  for (int i = 0; i < st->C; ++i) acc += E[i] * H[i];
  free(H);
  return 0.5 * creal(acc);
}

/* Propose, Alg. L.1 + Alg. 1 with the periodic modifications of Sec. 3.4:
 *   dE = sum_{l=2..L} q [Psi^D_{l,a'_l}(r'-R) - Psi^D_{l,a_l}(r-R)]
 *      + q [near(r') - near(r)]
 *      - sum_{nu in {-1,0,1}^3} q^2/|r' - r - a nu| + (q^2/a)(6 + 8/sqrt3 + 12/sqrt2)
 *      + 1/2 (E'.R(K') - E.R(K)) - (2 pi / 3V)(|D'|^2 - |D|^2)
 * where the new-side direct sum leaves out the moving charge's old images
 * lying in the near region together with the matching self terms (the two
 * cancel exactly), and the last term converts the cube-order lattice sum
 * to tin-foil boundary conditions. newpos is wrapped first. In the
 * multipole-based variant (Sec. 3.3) the first sum is replaced by
 * q [Phi_far(r') - Phi_far(r)], the multipole expansions of the interaction
 * lists of both cells on every level (Alg. M.1). */
double orc_propose(orc_t *st, int k, const double *newpos_in) {
  double a = st->a, q = st->q[k], rn[3], *r = &st->pos[3 * k];
  for (int i = 0; i < 3; ++i) rn[i] = st->free_space ? newpos_in[i] : orc_wrap(newpos_in[i], a);
  /* free space: a move out of the box is never taken */
  if (st->free_space && !point_in_box(rn, a)) return INFINITY;
  double dE = 0.0;
  /* long range, multipole-based variant (Alg. M.1): the expansions of the
   * interaction lists of both cells on every level */
  if (st->multipole) dE += q * (m2p_far(st, rn) - m2p_far(st, r));
  /* long range: per-level local expansions, ancestors of both cells */
  for (int l = st->L; l >= 2 && !st->multipole; --l) {
    int n = nside(l), c0[3], c1[3];
    double R0[3], R1[3];
    locate(st, l, r, c0);
    locate(st, l, rn, c1);
    cell_centre(st, l, c0, R0);
    cell_centre(st, l, c1, R1);
    double vnew = orc_l2p(st->p, (double *)local_of(st, l, cell_lin(n, c1)), rn, R1);
    double vold = orc_l2p(st->p, (double *)local_of(st, l, cell_lin(n, c0)), r, R0);
    dE += q * (vnew - vold);
  }
  /* direct near field (Alg. 1) */
  unsigned char skip_nu[27];
  double dnew = near_sum(st, rn, k, 1, skip_nu);
  double dold = near_sum(st, r, k, 0, NULL);
  dE += q * (dnew - dold);
  /* periodic self-interaction correction (Sec. 3.4); in free space only
   * the charge's own old position (nu = 0) is subtracted */
  double self = 0.0;
  for (int nz = -1; nz <= 1; ++nz)
    for (int ny = -1; ny <= 1; ++ny)
      for (int nx = -1; nx <= 1; ++nx) {
        if (skip_nu[(nx + 1) + 3 * (ny + 1) + 9 * (nz + 1)]) continue;
        if (st->free_space && (nx || ny || nz)) continue;
        double dv[3] = {rn[0] - (r[0] + a * nx), rn[1] - (r[1] + a * ny), rn[2] - (r[2] + a * nz)};
        self += q * q / sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
      }
  dE += -self;
  if (st->free_space) return dE;
  dE += q * q / a * orc_self_image_constant();
  /* far lattice (Sec. 3.4, with the factor 1/2 of a pair energy) */
  double R1c[3] = {0.5 * a, 0.5 * a, 0.5 * a};
  cplx *K2 = (cplx *)malloc(sizeof(cplx) * st->C), *E2 = (cplx *)malloc(sizeof(cplx) * st->C);
  memcpy(K2, st->K, sizeof(cplx) * st->C);
  memcpy(E2, st->E, sizeof(cplx) * st->C);
  orc_p2m(st->p, q, rn, R1c, (double *)K2);
  orc_p2m(st->p, -q, r, R1c, (double *)K2);
  orc_p2e(st->p, q, rn, R1c, (double *)E2);
  orc_p2e(st->p, -q, r, R1c, (double *)E2);
  dE += lattice_energy(st, K2, E2) - lattice_energy(st, st->K, st->E);
  free(K2);
  free(E2);
  /* tin-foil boundary: -(2 pi / 3V) |D|^2 */
  double V = a * a * a, D2[3];
  for (int i = 0; i < 3; ++i) D2[i] = st->dip[i] + q * (rn[i] - r[i]);
  double dd = (D2[0] * D2[0] + D2[1] * D2[1] + D2[2] * D2[2]) -
              (st->dip[0] * st->dip[0] + st->dip[1] * st->dip[1] + st->dip[2] * st->dip[2]);
  dE += -2.0 * M_PI / (3.0 * V) * dd;
  return dE;
}

/* Accept, Alg. L.2 with the periodic modifications of Sec. 3.4: for every
 * level l = 2..L subtract the charge at r from the local expansion of every
 * cell (image) in IL(a_l) and add it at r' to every cell in IL(a'_l);
 * update K, E, the dipole, the position and the leaf lists. The
 * multipole-based variant updates instead the multipole expansions of the
 * old and new cell on every level (Alg. M.2). */
void orc_accept(orc_t *st, int k, const double *newpos_in) {
  double a = st->a, q = st->q[k], rn[3], r[3];
  for (int i = 0; i < 3; ++i) {
    rn[i] = st->free_space ? newpos_in[i] : orc_wrap(newpos_in[i], a);
    r[i] = st->pos[3 * k + i];
  }
  if (st->free_space && !point_in_box(rn, a)) return; /* never taken */
  /* multipole-based variant (Alg. M.2): the charge leaves the multipole
   * expansion of its old cell and joins that of its new cell, per level */
  for (int l = st->L; l >= 2 && st->multipole; --l) {
    int n = nside(l), c0[3], c1[3];
    double R0[3], R1[3];
    locate(st, l, r, c0);
    locate(st, l, rn, c1);
    cell_centre(st, l, c0, R0);
    cell_centre(st, l, c1, R1);
    orc_p2m(st->p, -q, r, R0, (double *)&st->Mp[l][(size_t)cell_lin(n, c0) * st->C]);
    orc_p2m(st->p, q, rn, R1, (double *)&st->Mp[l][(size_t)cell_lin(n, c1) * st->C]);
  }
  for (int l = st->L; l >= 2 && !st->multipole; --l) {
    int n = nside(l);
    double h = a / (double)n;
    for (int side = 0; side < 2; ++side) {
      const double *x = side == 0 ? r : rn;
      double qs = side == 0 ? -q : q;
      int c[3], oct[3], off[189 * 3];
      locate(st, l, x, c);
      for (int i = 0; i < 3; ++i) oct[i] = c[i] & 1;
      int cnt = orc_il_offsets(oct, off);
      for (int j = 0; j < cnt; ++j) {
        int b[3] = {c[0] + off[3 * j], c[1] + off[3 * j + 1], c[2] + off[3 * j + 2]};
        if (st->free_space && !in_box(n, b)) continue;
        int s[3] = {imod(b[0], n), imod(b[1], n), imod(b[2], n)};
        int lin = cell_lin(n, s);
        if (st->lazy && !st->ready[l][lin]) continue; /* formed later from the log */
        double R[3] = {(b[0] + 0.5) * h, (b[1] + 0.5) * h, (b[2] + 0.5) * h};
        orc_p2l(st->p, qs, x, R, (double *)&st->Ld[l][(size_t)lin * st->C]);
      }
    }
  }
  if (st->lazy) {
    if (st->nlog == st->caplog) {
      st->caplog = st->caplog ? 2 * st->caplog : 64;
      st->log = (move_rec *)realloc(st->log, sizeof(move_rec) * st->caplog);
    }
    move_rec *m = &st->log[st->nlog++];
    memcpy(m->pos, r, sizeof r);
    memcpy(m->newpos, rn, sizeof rn);
    m->q = q;
  }
  double R1c[3] = {0.5 * a, 0.5 * a, 0.5 * a};
  orc_p2m(st->p, q, rn, R1c, (double *)st->K);
  orc_p2m(st->p, -q, r, R1c, (double *)st->K);
  orc_p2e(st->p, q, rn, R1c, (double *)st->E);
  orc_p2e(st->p, -q, r, R1c, (double *)st->E);
  for (int i = 0; i < 3; ++i) st->dip[i] += q * (rn[i] - r[i]);
  int nL = nside(st->L), c[3];
  locate(st, st->L, rn, c);
  int newleaf = cell_lin(nL, c);
  list_remove(&st->leaf[st->leaf_of[k]], k);
  list_add(&st->leaf[newleaf], k);
  st->leaf_of[k] = newleaf;
  for (int i = 0; i < 3; ++i) st->pos[3 * k + i] = rn[i];
}

/* total energy U = 1/2 sum_i q_i [sum_l Psi^D_l(r_i) + near(r_i)]
 *                  + 1/2 E.R(K) - (2 pi / 3V)|D|^2  (tin-foil) */
double orc_energy(orc_t *st) {
  double U = 0.0;
  for (int i = 0; i < st->N; ++i) {
    double *r = &st->pos[3 * i], phi = 0.0;
    if (st->multipole) phi += m2p_far(st, r);
    for (int l = 2; l <= st->L && !st->multipole; ++l) {
      int n = nside(l), c[3];
      double R[3];
      locate(st, l, r, c);
      cell_centre(st, l, c, R);
      phi += orc_l2p(st->p, (double *)local_of(st, l, cell_lin(n, c)), r, R);
    }
    phi += near_sum(st, r, i, 0, NULL);
    U += 0.5 * st->q[i] * phi;
  }
  if (st->free_space) return U;
  U += lattice_energy(st, st->K, st->E);
  double V = st->a * st->a * st->a;
  U += -2.0 * M_PI / (3.0 * V) *
       (st->dip[0] * st->dip[0] + st->dip[1] * st->dip[1] + st->dip[2] * st->dip[2]);
  return U;
}

/* copy of L^Delta of one cell (complex, (p+1)^2) */
void orc_get_local(orc_t *st, int l, int lin, double *out) {
  memcpy(out, local_of(st, l, lin), sizeof(cplx) * st->C);
}

/* copy of the multipole expansion of one cell (complex, (p+1)^2); valid
 * after orc_setup_multipole, or after orc_setup_fmm for the setup state */
void orc_get_multipole(orc_t *st, int l, int lin, double *out) {
  memcpy(out, &st->Mp[l][(size_t)lin * st->C], sizeof(cplx) * st->C);
}

void orc_get_K(orc_t *st, double *out) { memcpy(out, st->K, sizeof(cplx) * st->C); }

void orc_get_positions(orc_t *st, double *out) {
  memcpy(out, st->pos, sizeof(double) * 3 * st->N);
}

int orc_leaf_of(orc_t *st, int k) { return st->leaf_of[k]; }

/* The Metropolis-Hastings loop of the user (Sec. 4.1), over steps
 * [t0, t0+nsteps): draw (idx, delta, u) from the Philox stream, propose
 * r' = wrap(r_idx + delta), accept iff u < exp(-beta dE). Per-step traces
 * are written when the pointers are non-NULL. Returns the number accepted. */
int64_t orc_run(orc_t *st, uint64_t seed, uint64_t chain, int64_t t0, int64_t nsteps,
                double beta, double D, int64_t *tr_idx, double *tr_newpos, double *tr_dE,
                double *tr_u, unsigned char *tr_acc) {
  int64_t nacc = 0;
  for (int64_t t = t0; t < t0 + nsteps; ++t) {
    int64_t idx;
    double delta[3], u, rn[3];
    orc_draw(seed, chain, (uint64_t)t, st->N, D, &idx, delta, &u);
    for (int k = 0; k < 3; ++k)
      rn[k] = st->free_space ? st->pos[3 * idx + k] + delta[k] : orc_wrap(st->pos[3 * idx + k] + delta[k], st->a);
    double dE = orc_propose(st, (int)idx, rn);
    int acc = u < exp(-beta * dE);
    if (acc) {
      orc_accept(st, (int)idx, rn);
      ++nacc;
    }
    int64_t o = t - t0;
    if (tr_idx) tr_idx[o] = idx;
    if (tr_newpos)
      for (int k = 0; k < 3; ++k) tr_newpos[3 * o + k] = rn[k];
    if (tr_dE) tr_dE[o] = dE;
    if (tr_u) tr_u[o] = u;
    if (tr_acc) tr_acc[o] = (unsigned char)acc;
  }
  return nacc;
}
