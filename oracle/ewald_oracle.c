/*
 * ewald_oracle.c -- plain CPU FP64 Ewald summation with tin-foil boundary
 * conditions and per-move structure-factor updates: the O(sqrt N)-per-move
 * scheme the paper compares against (Sec. 2, Sec. 5.3).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check of the entry
 * module and the cpu_baseline leg of the benchmark may load this library.
 *
 * U = U_real + U_recip + U_self, Gaussian units (k_e = 1), box side a, V = a^3:
 *   U_real  = sum_{i<j} q_i q_j erfc(alpha d_ij)/d_ij  (minimum image, d_ij < rc <= a/2)
 *   U_recip = (2 pi / V) sum_{k != 0} exp(-k^2/(4 alpha^2))/k^2 |S(k)|^2,
 *             S(k) = sum_j q_j exp(i k.r_j), k = 2 pi n / a, |n| <= kmax
 *   U_self  = -(alpha/sqrt(pi)) sum_i q_i^2
 * A move of charge k from r to r' changes S by q (e^{ik.r'} - e^{ik.r}); the
 * energy change is the real-space change over the other charges plus the
 * change of the quadratic form in S.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
  int N, kmax, nk;
  double a, alpha, rc;
  double *pos, *q;
  int *kn;      /* 3 * nk integer wave vectors of the half space */
  double *kfac; /* (4 pi / V) exp(-k^2/4alpha^2)/k^2 : the factor of the half space */
  cplx *S;
} ewd_t;

static double wrapc(double x, double a) {
  double w = x - a * floor(x / a);
  if (w >= a) w = 0.0;
  if (w < 0.0) w = 0.0;
  return w;
}

/* minimum-image distance */
static double mi_dist(const double *x, const double *y, double a) {
  double s = 0.0;
  for (int k = 0; k < 3; ++k) {
    double d = x[k] - y[k];
    d -= a * nearbyint(d / a);
    s += d * d;
  }
  return sqrt(s);
}

static double greal(double d, double alpha, double rc) {
  if (d >= rc) return 0.0;
  return erfc(alpha * d) / d;
}

static void axis_phases(const double *r, double a, int kmax, cplx *ph) {
  /* ph[(axis)*(2kmax+1) + (n+kmax)] = exp(i 2 pi n r_axis / a) */
  for (int ax = 0; ax < 3; ++ax)
    for (int n = -kmax; n <= kmax; ++n)
      ph[ax * (2 * kmax + 1) + n + kmax] = cexp(I * 2.0 * M_PI * (double)n * r[ax] / a);
}

static cplx phase_of(const cplx *ph, int kmax, const int *n) {
  int w = 2 * kmax + 1;
  return ph[n[0] + kmax] * ph[w + n[1] + kmax] * ph[2 * w + n[2] + kmax];
}

ewd_t *ewd_create(int N, const double *pos, const double *q, double a, double alpha,
                  double rc, int kmax) {
  ewd_t *e = (ewd_t *)calloc(1, sizeof(ewd_t));
  e->N = N;
  e->a = a;
  e->alpha = alpha;
  e->rc = rc;
  e->kmax = kmax;
  e->pos = (double *)malloc(sizeof(double) * 3 * N);
  e->q = (double *)malloc(sizeof(double) * N);
  for (int i = 0; i < N; ++i) {
    for (int k = 0; k < 3; ++k) e->pos[3 * i + k] = wrapc(pos[3 * i + k], a);
    e->q[i] = q[i];
  }
  int cap = (2 * kmax + 1) * (2 * kmax + 1) * (2 * kmax + 1);
  e->kn = (int *)malloc(sizeof(int) * 3 * cap);
  e->kfac = (double *)malloc(sizeof(double) * cap);
  double V = a * a * a;
  int nk = 0;
  for (int nx = 0; nx <= kmax; ++nx)
    for (int ny = -kmax; ny <= kmax; ++ny)
      for (int nz = -kmax; nz <= kmax; ++nz) {
        /* half space: nx > 0, or nx == 0 and ny > 0, or nx == ny == 0 and nz > 0 */
        if (nx == 0 && (ny < 0 || (ny == 0 && nz <= 0))) continue;
        if (nx * nx + ny * ny + nz * nz > kmax * kmax) continue;
        double kx = 2 * M_PI * nx / a, ky = 2 * M_PI * ny / a, kz = 2 * M_PI * nz / a;
        double k2 = kx * kx + ky * ky + kz * kz;
        e->kn[3 * nk] = nx;
        e->kn[3 * nk + 1] = ny;
        e->kn[3 * nk + 2] = nz;
        e->kfac[nk] = 4.0 * M_PI / V * exp(-k2 / (4.0 * alpha * alpha)) / k2;
        ++nk;
      }
  e->nk = nk;
  e->S = (cplx *)calloc((size_t)nk, sizeof(cplx));
  cplx *ph = (cplx *)malloc(sizeof(cplx) * 3 * (2 * kmax + 1));
  for (int i = 0; i < N; ++i) {
    axis_phases(&e->pos[3 * i], a, kmax, ph);
    for (int t = 0; t < nk; ++t) e->S[t] += e->q[i] * phase_of(ph, kmax, &e->kn[3 * t]);
  }
  free(ph);
  return e;
}

void ewd_destroy(ewd_t *e) {
  if (!e) return;
  free(e->pos);
  free(e->q);
  free(e->kn);
  free(e->kfac);
  free(e->S);
  free(e);
}

double ewd_energy(ewd_t *e) {
  double ur = 0.0, uk = 0.0, us = 0.0;
  for (int i = 0; i < e->N; ++i)
    for (int j = i + 1; j < e->N; ++j)
      ur += e->q[i] * e->q[j] * greal(mi_dist(&e->pos[3 * i], &e->pos[3 * j], e->a), e->alpha, e->rc);
  for (int t = 0; t < e->nk; ++t) {
    double s2 = creal(e->S[t]) * creal(e->S[t]) + cimag(e->S[t]) * cimag(e->S[t]);
    uk += e->kfac[t] * s2;
  }
  for (int i = 0; i < e->N; ++i) us += e->q[i] * e->q[i];
  us *= -e->alpha / sqrt(M_PI);
  return ur + uk + us;
}

/* energy change of moving charge k to newpos (wrapped first) */
double ewd_propose(ewd_t *e, int k, const double *newpos) {
  double rn[3], *r = &e->pos[3 * k], q = e->q[k];
  for (int i = 0; i < 3; ++i) rn[i] = wrapc(newpos[i], e->a);
  double dr = 0.0;
  for (int j = 0; j < e->N; ++j) {
    if (j == k) continue;
    dr += e->q[j] * (greal(mi_dist(rn, &e->pos[3 * j], e->a), e->alpha, e->rc) -
                     greal(mi_dist(r, &e->pos[3 * j], e->a), e->alpha, e->rc));
  }
  dr *= q;
  int kmax = e->kmax;
  cplx *p0 = (cplx *)malloc(sizeof(cplx) * 3 * (2 * kmax + 1));
  cplx *p1 = (cplx *)malloc(sizeof(cplx) * 3 * (2 * kmax + 1));
  axis_phases(r, e->a, kmax, p0);
  axis_phases(rn, e->a, kmax, p1);
  double dk = 0.0;
  for (int t = 0; t < e->nk; ++t) {
    cplx S1 = e->S[t] + q * (phase_of(p1, kmax, &e->kn[3 * t]) - phase_of(p0, kmax, &e->kn[3 * t]));
    double a1 = creal(S1) * creal(S1) + cimag(S1) * cimag(S1);
    double a0 = creal(e->S[t]) * creal(e->S[t]) + cimag(e->S[t]) * cimag(e->S[t]);
    dk += e->kfac[t] * (a1 - a0);
  }
  free(p0);
  free(p1);
  return dr + dk;
}

void ewd_accept(ewd_t *e, int k, const double *newpos) {
  double rn[3], *r = &e->pos[3 * k], q = e->q[k];
  for (int i = 0; i < 3; ++i) rn[i] = wrapc(newpos[i], e->a);
  int kmax = e->kmax;
  cplx *p0 = (cplx *)malloc(sizeof(cplx) * 3 * (2 * kmax + 1));
  cplx *p1 = (cplx *)malloc(sizeof(cplx) * 3 * (2 * kmax + 1));
  axis_phases(r, e->a, kmax, p0);
  axis_phases(rn, e->a, kmax, p1);
  for (int t = 0; t < e->nk; ++t)
    e->S[t] += q * (phase_of(p1, kmax, &e->kn[3 * t]) - phase_of(p0, kmax, &e->kn[3 * t]));
  free(p0);
  free(p1);
  for (int i = 0; i < 3; ++i) r[i] = rn[i];
}

int ewd_num_k(ewd_t *e) { return e->nk; }
