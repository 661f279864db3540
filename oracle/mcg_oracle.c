/*
 * mcg_oracle.c -- plain FP64 CPU oracle for stout-preconditioned MCG fixing
 * (arXiv:0807.0264).  TEST INFRASTRUCTURE ONLY: only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code
 * with the HIP library.
 *
 * Everything is written for a reader checking it against the paper: 3x3
 * matrices are row-major arrays of nine C99 complex doubles, every product
 * is a full matrix product, and every path of links is walked one step at
 * a time.  Speed is not a goal; OpenMP only splits loops whose iterations
 * are independent (sites of one checkerboard parity, or links of a Jacobi
 * smearing step), so results do not depend on the thread count.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (oracle/build.py).
 */
#include "mcg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ========================================================================
 * 3x3 complex matrices
 * ====================================================================== */
static void m_zero(ocx *a) { for (int k = 0; k < 9; k++) a[k] = 0; }
static void m_ident(ocx *a) { m_zero(a); a[0] = a[4] = a[8] = 1; }
static void m_copy(ocx *dst, const ocx *src) { memcpy(dst, src, 9 * sizeof(ocx)); }

/* c = a b ; c must not alias a or b */
static void m_mul(const ocx *a, const ocx *b, ocx *c) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      ocx s = 0;
      for (int k = 0; k < 3; k++) s += a[3 * i + k] * b[3 * k + j];
      c[3 * i + j] = s;
    }
}
/* a = a b, via a temporary */
static void m_mul_right(ocx *a, const ocx *b) {
  ocx t[9];
  m_mul(a, b, t);
  m_copy(a, t);
}
/* b = a b, via a temporary */
static void m_mul_left(const ocx *a, ocx *b) {
  ocx t[9];
  m_mul(a, b, t);
  m_copy(b, t);
}
static void m_adj(const ocx *a, ocx *c) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) c[3 * i + j] = conj(a[3 * j + i]);
}
static ocx m_tr(const ocx *a) { return a[0] + a[4] + a[8]; }
/* c += s a */
static void m_axpy(ocx s, const ocx *a, ocx *c) {
  for (int k = 0; k < 9; k++) c[k] += s * a[k];
}
/* Re tr(a^dagger b): the real inner product on complex matrices */
static double m_dot(const ocx *a, const ocx *b) {
  double s = 0;
  for (int k = 0; k < 9; k++) s += creal(conj(a[k]) * b[k]);
  return s;
}
/* traceless anti-Hermitian part: (1/2)(M - M^dag) - (1/6) tr(M - M^dag) 1 */
static void m_ta(const ocx *m, ocx *out) {
  ocx md[9];
  m_adj(m, md);
  for (int k = 0; k < 9; k++) out[k] = 0.5 * (m[k] - md[k]);
  ocx tr = m_tr(m) - m_tr(md);
  for (int i = 0; i < 3; i++) out[4 * i] -= tr / 6.0;
}

/* Gram-Schmidt on the rows, third row = conj(row0 x row1) so det = +1 */
void or_reunit(ocx M[9]) {
  ocx *r0 = M, *r1 = M + 3, *r2 = M + 6;
  double n0 = 0;
  for (int k = 0; k < 3; k++) n0 += creal(conj(r0[k]) * r0[k]);
  n0 = sqrt(n0);
  for (int k = 0; k < 3; k++) r0[k] /= n0;
  ocx ip = 0;
  for (int k = 0; k < 3; k++) ip += conj(r0[k]) * r1[k];
  for (int k = 0; k < 3; k++) r1[k] -= ip * r0[k];
  double n1 = 0;
  for (int k = 0; k < 3; k++) n1 += creal(conj(r1[k]) * r1[k]);
  n1 = sqrt(n1);
  for (int k = 0; k < 3; k++) r1[k] /= n1;
  r2[0] = conj(r0[1] * r1[2] - r0[2] * r1[1]);
  r2[1] = conj(r0[2] * r1[0] - r0[0] * r1[2]);
  r2[2] = conj(r0[0] * r1[1] - r0[1] * r1[0]);
}

/* ========================================================================
 * Matrix exponential, two independent ways
 * ====================================================================== */

/* Cyclic complex Jacobi diagonalisation of a Hermitian 3x3 matrix.
 * On return Q_in = V diag(lam) V^dagger. */
static void herm_eig3(const ocx *Qin, double lam[3], ocx V[9]) {
  ocx Q[9];
  m_copy(Q, Qin);
  m_ident(V);
  static const int P[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (int sweep = 0; sweep < 60; sweep++) {
    double off = 0, diag = 0;
    for (int k = 0; k < 3; k++) {
      ocx q = Q[3 * P[k][0] + P[k][1]];
      off += creal(q * conj(q));
      diag += creal(Q[4 * k]) * creal(Q[4 * k]);
    }
    if (off == 0 || off < 1e-36 * diag) break;
    for (int k = 0; k < 3; k++) {
      int p = P[k][0], q = P[k][1];
      double apq = cabs(Q[3 * p + q]);
      if (apq == 0) continue;
      ocx phase = Q[3 * p + q] / apq;
      double app = creal(Q[4 * p]), aqq = creal(Q[4 * q]);
      double tau = (aqq - app) / (2 * apq);
      double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
      double c = 1 / sqrt(1 + t * t), s = t * c;
      /* R = D J: D = diag(..., conj(phase) at q), J real rotation in (p,q) */
      ocx R[9], Rd[9], T[9];
      m_ident(R);
      R[3 * p + p] = c;
      R[3 * p + q] = s;
      R[3 * q + p] = -s * conj(phase);
      R[3 * q + q] = c * conj(phase);
      m_adj(R, Rd);
      m_mul(Rd, Q, T);
      m_mul(T, R, Q);
      m_mul_right(V, R);
    }
  }
  for (int k = 0; k < 3; k++) lam[k] = creal(Q[4 * k]);
}

void or_exp_su3_eigen(const ocx A[9], ocx E[9]) {
  ocx Q[9], V[9], Vd[9], D[9], T[9];
  for (int k = 0; k < 9; k++) Q[k] = -I * A[k];
  /* symmetrise against rounding so the Jacobi input is exactly Hermitian */
  ocx Qd[9];
  m_adj(Q, Qd);
  for (int k = 0; k < 9; k++) Q[k] = 0.5 * (Q[k] + Qd[k]);
  double lam[3];
  herm_eig3(Q, lam, V);
  m_zero(D);
  for (int k = 0; k < 3; k++) D[4 * k] = cos(lam[k]) + I * sin(lam[k]);
  m_adj(V, Vd);
  m_mul(V, D, T);
  m_mul(T, Vd, E);
}

/* exp of an n x n matrix (n <= 6): scale by 2^-s until the 1-norm is below
 * 1/2, sum the Taylor series to convergence, square s times. */
void or_exp_taylor(const ocx *A, int n, ocx *E) {
  ocx B[36], term[36], tmp[36];
  double nrm = 0;
  for (int j = 0; j < n; j++) {
    double col = 0;
    for (int i = 0; i < n; i++) col += cabs(A[n * i + j]);
    if (col > nrm) nrm = col;
  }
  int s = 0;
  while (nrm > 0.5) { nrm *= 0.5; s++; }
  double scale = ldexp(1.0, -s);
  for (int k = 0; k < n * n; k++) B[k] = A[k] * scale;
  for (int k = 0; k < n * n; k++) E[k] = term[k] = (k % (n + 1) == 0) ? 1 : 0;
  for (int it = 1; it <= 40; it++) {
    for (int i = 0; i < n; i++)
      for (int j = 0; j < n; j++) {
        ocx acc = 0;
        for (int k = 0; k < n; k++) acc += term[n * i + k] * B[n * k + j];
        tmp[n * i + j] = acc / it;
      }
    double tn = 0;
    for (int k = 0; k < n * n; k++) {
      term[k] = tmp[k];
      E[k] += term[k];
      tn += cabs(term[k]);
    }
    if (tn < 1e-40) break;
  }
  for (int q = 0; q < s; q++) {
    for (int i = 0; i < n; i++)
      for (int j = 0; j < n; j++) {
        ocx acc = 0;
        for (int k = 0; k < n; k++) acc += E[n * i + k] * E[n * k + j];
        tmp[n * i + j] = acc;
      }
    for (int k = 0; k < n * n; k++) E[k] = tmp[k];
  }
}

/* Frechet derivative of exp at A in direction Ed: the upper-right block of
 * exp([[A, Ed], [0, A]]). */
static void exp_frechet(const ocx *A, const ocx *Ed, ocx *Lout) {
  ocx Big[36], EB[36];
  for (int k = 0; k < 36; k++) Big[k] = 0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      Big[6 * i + j] = A[3 * i + j];
      Big[6 * (i + 3) + (j + 3)] = A[3 * i + j];
      Big[6 * i + (j + 3)] = Ed[3 * i + j];
    }
  or_exp_taylor(Big, 6, EB);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) Lout[3 * i + j] = EB[6 * i + (j + 3)];
}

/* ========================================================================
 * Lattice
 * ====================================================================== */
typedef struct {
  int32_t L[4];
  int64_t V;
} lat_t;

static lat_t mklat(const int32_t L[4]) {
  lat_t lt;
  for (int k = 0; k < 4; k++) lt.L[k] = L[k];
  lt.V = (int64_t)L[0] * L[1] * L[2] * L[3];
  return lt;
}
int64_t or_volume(const int32_t L[4]) { return mklat(L).V; }

static void coords(const lat_t *lt, int64_t i, int c[4]) {
  for (int k = 0; k < 4; k++) {
    c[k] = (int)(i % lt->L[k]);
    i /= lt->L[k];
  }
}
static int64_t index_of(const lat_t *lt, const int c[4]) {
  return c[0] + (int64_t)lt->L[0] * (c[1] + (int64_t)lt->L[1] * (c[2] + (int64_t)lt->L[2] * c[3]));
}
/* site i moved by `step` lattice units along direction mu, periodic */
static int64_t shift(const lat_t *lt, int64_t i, int mu, int step) {
  int c[4];
  coords(lt, i, c);
  c[mu] = ((c[mu] + step) % lt->L[mu] + lt->L[mu]) % lt->L[mu];
  return index_of(lt, c);
}
static int parity_of(const lat_t *lt, int64_t i) {
  int c[4];
  coords(lt, i, c);
  return (c[0] + c[1] + c[2] + c[3]) & 1;
}
static const ocx *link(const ocx *U, int64_t i, int mu) { return U + (i * 4 + mu) * 9; }
static ocx *link_w(ocx *U, int64_t i, int mu) { return U + (i * 4 + mu) * 9; }

/* Product of links along a path.  steps[k] = +(d+1) walks forward along d
 * (factor U_d(y), then y -> y+d), -(d+1) walks backward (y -> y-d, then
 * factor U_d(y)^dagger). */
static void walk(const lat_t *lt, const ocx *U, int64_t x, const int *steps,
                 int n, ocx P[9]) {
  m_ident(P);
  int64_t y = x;
  for (int k = 0; k < n; k++) {
    int d = abs(steps[k]) - 1;
    if (steps[k] > 0) {
      m_mul_right(P, link(U, y, d));
      y = shift(lt, y, d, +1);
    } else {
      y = shift(lt, y, d, -1);
      ocx ud[9];
      m_adj(link(U, y, d), ud);
      m_mul_right(P, ud);
    }
  }
}

/* ========================================================================
 * Gauge transform, functional, gauge-invariant observables (Sec. II.A)
 * ====================================================================== */
void or_apply_gauge(const int32_t L[4], const ocx *U, const ocx *G, ocx *out) {
  lat_t lt = mklat(L);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < lt.V; i++)
    for (int mu = 0; mu < 4; mu++) {
      ocx t[9], gd[9];
      m_mul(G + i * 9, link(U, i, mu), t);
      m_adj(G + shift(&lt, i, mu, +1) * 9, gd);
      m_mul(t, gd, link_w(out, i, mu));
    }
}

/* Kahan-compensated sum in index order */
static double kahan(const double *a, int64_t n) {
  double s = 0, c = 0;
  for (int64_t k = 0; k < n; k++) {
    double y = a[k] - c, t = s + y;
    c = (t - s) - y;
    s = t;
  }
  return s;
}

/* V_U = (1/N_l) sum_{x,mu} |tr U_mu(x) / 3|^2, N_l = 4V  (Sec. II.A) */
double or_functional(const int32_t L[4], const ocx *U) {
  lat_t lt = mklat(L);
  int64_t nl = 4 * lt.V;
  double *a = malloc(nl * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t l = 0; l < nl; l++) {
    ocx t = m_tr(U + l * 9);
    a[l] = creal(t * conj(t));
  }
  double s = kahan(a, nl);
  free(a);
  return s / (9.0 * nl);
}

double or_plaquette(const int32_t L[4], const ocx *U) {
  lat_t lt = mklat(L);
  double *a = malloc(lt.V * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < lt.V; i++) {
    double s = 0;
    for (int mu = 0; mu < 4; mu++)
      for (int nu = mu + 1; nu < 4; nu++) {
        int st[4] = {mu + 1, nu + 1, -(mu + 1), -(nu + 1)};
        ocx P[9];
        walk(&lt, U, i, st, 4, P);
        s += creal(m_tr(P));
      }
    a[i] = s;
  }
  double s = kahan(a, lt.V);
  free(a);
  return s / (18.0 * lt.V);
}

/* on-axis r x t Wilson loop, r along each spatial direction 0..2, t along 3 */
double or_wilson_loop(const int32_t L[4], const ocx *U, int r, int t) {
  lat_t lt = mklat(L);
  double *a = malloc(lt.V * sizeof(double));
  int n = 2 * (r + t);
  int *st = malloc(3 * n * sizeof(int));
  for (int i = 0; i < 3; i++) {
    int *s = st + i * n, k = 0;
    for (int q = 0; q < r; q++) s[k++] = i + 1;
    for (int q = 0; q < t; q++) s[k++] = 4;
    for (int q = 0; q < r; q++) s[k++] = -(i + 1);
    for (int q = 0; q < t; q++) s[k++] = -4;
  }
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < lt.V; x++) {
    double s = 0;
    for (int i = 0; i < 3; i++) {
      ocx P[9];
      walk(&lt, U, x, st + i * n, n, P);
      s += creal(m_tr(P));
    }
    a[x] = s;
  }
  double s = kahan(a, lt.V);
  free(a);
  free(st);
  return s / (9.0 * lt.V);
}

/* tr(prod_t U_3(x,t)) / 3 for every spatial site (index x + Lx(y + Ly z)) */
void or_polyakov(const int32_t L[4], const ocx *U, ocx *P) {
  lat_t lt = mklat(L);
  int64_t vs = lt.V / L[3];
  for (int64_t s = 0; s < vs; s++) {
    ocx M[9];
    m_ident(M);
    int64_t y = s;
    for (int t = 0; t < L[3]; t++) {
      m_mul_right(M, link(U, y, 3));
      y = shift(&lt, y, 3, +1);
    }
    P[s] = m_tr(M) / 3.0;
  }
}

/* ========================================================================
 * Stout and over-improved stout smearing (Sec. II.B, Sec. III)
 * ====================================================================== */

/* The paths from x to x+mu that make up C_mu(x).  For each nu != mu and
 * each sign of nu: the plaquette staple, and the three rectangle staples
 * (2x1 ahead in mu, 2x1 behind in mu, 1x2 long in nu). */
#define NPATH_PER_NU_SIGN 4
static int path_steps(int mu, int nu, int sg, int which, int st[5]) {
  int m = mu + 1, n = sg * (nu + 1);
  switch (which) {
  case 0: st[0] = n; st[1] = m; st[2] = -n; return 3;
  case 1: st[0] = n; st[1] = m; st[2] = m; st[3] = -n; st[4] = -m; return 5;
  case 2: st[0] = -m; st[1] = n; st[2] = m; st[3] = m; st[4] = -n; return 5;
  default: st[0] = n; st[1] = n; st[2] = m; st[3] = -n; st[4] = -n; return 5;
  }
}

/* plaquette part Cp and rectangle part Cr of the staple sum (no weights) */
static void staple_parts(const lat_t *lt, const ocx *U, int64_t x, int mu,
                         ocx Cp[9], ocx Cr[9]) {
  m_zero(Cp);
  m_zero(Cr);
  for (int nu = 0; nu < 4; nu++) {
    if (nu == mu) continue;
    for (int sg = 1; sg >= -1; sg -= 2)
      for (int w = 0; w < NPATH_PER_NU_SIGN; w++) {
        int st[5];
        int n = path_steps(mu, nu, sg, w, st);
        ocx P[9];
        walk(lt, U, x, st, n, P);
        m_axpy(1.0, P, w == 0 ? Cp : Cr);
      }
  }
}

static void weights(double eps, double *wp, double *wr) {
  *wp = (5.0 - 2.0 * eps) / 3.0;
  *wr = -(1.0 - eps) / 12.0;
}

void or_staple_sum(const int32_t L[4], const ocx *U, int64_t site, int mu,
                   double rho, double eps, ocx C[9]) {
  lat_t lt = mklat(L);
  ocx Cp[9], Cr[9];
  double wp, wr;
  weights(eps, &wp, &wr);
  staple_parts(&lt, U, site, mu, Cp, Cr);
  for (int k = 0; k < 9; k++) C[k] = rho * (wp * Cp[k] + wr * Cr[k]);
}

/* Plain stout staples, written out as explicit products:
 * sum_{nu != mu} U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
 *              + U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)                 */
void or_stout_staple_plain(const int32_t L[4], const ocx *U, int64_t x,
                           int mu, double rho, ocx C[9]) {
  lat_t lt = mklat(L);
  m_zero(C);
  int64_t xpm = shift(&lt, x, mu, +1);
  for (int nu = 0; nu < 4; nu++) {
    if (nu == mu) continue;
    int64_t xpn = shift(&lt, x, nu, +1), xmn = shift(&lt, x, nu, -1);
    int64_t xmnpm = shift(&lt, xmn, mu, +1);
    ocx a[9], b[9], d[9];
    m_mul(link(U, x, nu), link(U, xpn, mu), a);
    m_adj(link(U, xpm, nu), d);
    m_mul(a, d, b);
    m_axpy(1.0, b, C);
    m_adj(link(U, xmn, nu), d);
    m_mul(d, link(U, xmn, mu), a);
    m_mul(a, link(U, xmnpm, nu), b);
    m_axpy(1.0, b, C);
  }
  for (int k = 0; k < 9; k++) C[k] *= rho;
}

/* U' = exp(TA(C U^dag)) U for one link */
void or_smear_link(const int32_t L[4], const ocx *U, int64_t site, int mu,
                   double rho, double eps, ocx out[9]) {
  ocx C[9], Ud[9], Om[9], A[9], E[9];
  or_staple_sum(L, U, site, mu, rho, eps, C);
  m_adj(link(U, site, mu), Ud);
  m_mul(C, Ud, Om);
  m_ta(Om, A);
  or_exp_su3_eigen(A, E);
  m_mul(E, link(U, site, mu), out);
}

/* one Jacobi step: every new link is computed from the old field */
void or_smear_step(const int32_t L[4], const ocx *U, ocx *out, double rho,
                   double eps) {
  lat_t lt = mklat(L);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < lt.V; i++)
    for (int mu = 0; mu < 4; mu++) or_smear_link(L, U, i, mu, rho, eps, link_w(out, i, mu));
}

void or_smear(const int32_t L[4], const ocx *U, ocx *out, double rho,
              double eps, int n) {
  lat_t lt = mklat(L);
  size_t bytes = (size_t)lt.V * 36 * sizeof(ocx);
  memcpy(out, U, bytes);
  if (n <= 0) return;
  ocx *tmp = malloc(bytes);
  for (int k = 0; k < n; k++) {
    or_smear_step(L, out, tmp, rho, eps);
    memcpy(out, tmp, bytes);
  }
  free(tmp);
}

/* ========================================================================
 * MCG fixing (Sec. II.A): maximise R = (1/N_l) sum |tr U^G / 3|^2
 * ====================================================================== */

/* One local update.  The eight links touching x enter as
 * F(g) = sum_k |tr(g M_k)|^2.  Because |z|^2 is convex,
 * F(g) >= F(1) + 2 Re tr(g X) - 2 Re tr X with X = sum_k conj(tr M_k) M_k,
 * so any g that raises Re tr(g X) cannot lower F.  g is built from three
 * SU(2) subgroup steps, each maximising Re tr(s Y) over the subgroup and
 * then over-relaxed towards the identity with weight omega. */
/* the three SU(2) subgroup steps (0,1), (1,2), (0,2): each left-multiplies Y
 * and g by the over-relaxed maximiser s of Re tr(s Y) on that subgroup */
static void subgroup_steps(ocx Y[9], ocx g[9], double omega) {
  static const int SUB[3][2] = {{0, 1}, {1, 2}, {0, 2}};
  for (int q = 0; q < 3; q++) {
    int i = SUB[q][0], j = SUB[q][1];
    ocx y11 = Y[3 * i + i], y12 = Y[3 * i + j], y21 = Y[3 * j + i], y22 = Y[3 * j + j];
    /* Re tr(s y) = a . v for s = a0 + i a.sigma in the basis used below */
    double v[4] = {creal(y11 + y22), -cimag(y12 + y21), creal(y21 - y12), -cimag(y11 - y22)};
    double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3]);
    if (nv == 0) continue;
    double a[4];
    a[0] = (1 - omega) + omega * v[0] / nv;
    for (int k = 1; k < 4; k++) a[k] = omega * v[k] / nv;
    double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
    if (na == 0) continue;
    for (int k = 0; k < 4; k++) a[k] /= na;
    ocx S[9];
    m_ident(S);
    S[3 * i + i] = a[0] + I * a[3];
    S[3 * i + j] = a[2] + I * a[1];
    S[3 * j + i] = -a[2] + I * a[1];
    S[3 * j + j] = a[0] - I * a[3];
    m_mul_left(S, Y);
    m_mul_left(S, g);
  }
}

/* ---- exact maximisation over one SU(2) subgroup (an update-rule variant) --
 * For s = a0 + i a.sigma acting on rows (i, j) and Y_k = g M_k,
 *   tr(s Y_k) = Y_kk' + a . b_k,  b_k = (Y_ii + Y_jj, i(Y_ji + Y_ij), Y_ji - Y_ij, i(Y_ii - Y_jj))
 * (k' the third index), so sum_k |tr(s Y_k)|^2 = const + 2 h.a + a^T Q a with
 * h = sum_k Re(conj(Y_k'k') b_k), Q = sum_k Re(b_k b_k^dagger).  Its maximum on
 * the unit sphere solves (lambda - Q) a = h with lambda >= the largest
 * eigenvalue of Q (found from the eigenvalues of Q and the secular equation
 * sum_m (h'_m / (lambda - q_m))^2 = 1 by bisection). */

/* cyclic Jacobi eigendecomposition of a real symmetric 4x4 matrix: A is
 * overwritten by diag(q), the columns of V are the eigenvectors */
static void sym4_eig(double A[4][4], double V[4][4]) {
  for (int r = 0; r < 4; r++)
    for (int c = 0; c < 4; c++) V[r][c] = r == c;
  for (int sweep = 0; sweep < 60; sweep++) {
    double off = 0;
    for (int p = 0; p < 4; p++)
      for (int q = p + 1; q < 4; q++) off += A[p][q] * A[p][q];
    if (off < 1e-300) break;
    for (int p = 0; p < 4; p++)
      for (int q = p + 1; q < 4; q++) {
        if (A[p][q] == 0) continue;
        double th = (A[q][q] - A[p][p]) / (2 * A[p][q]);
        double t = (th >= 0 ? 1 : -1) / (fabs(th) + sqrt(th * th + 1));
        double c = 1 / sqrt(t * t + 1), sn = t * c;
        for (int k = 0; k < 4; k++) { /* A <- J^T A J */
          double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 4; k++) {
          double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < 4; k++) {
          double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - sn * vkq;
          V[k][q] = sn * vkp + c * vkq;
        }
      }
  }
}

/* argmax of a^T Q a + 2 h.a over |a| = 1 */
void or_sphere_max(const double Qin[16], const double h[4], double a[4]) {
  double A[4][4], V[4][4], q[4], hp[4];
  for (int r = 0; r < 4; r++)
    for (int c = 0; c < 4; c++) A[r][c] = Qin[4 * r + c];
  sym4_eig(A, V);
  int top = 0;
  for (int m = 0; m < 4; m++) {
    q[m] = A[m][m];
    if (q[m] > q[top]) top = m;
  }
  double hn = 0;
  for (int m = 0; m < 4; m++) {
    hp[m] = 0;
    for (int r = 0; r < 4; r++) hp[m] += V[r][m] * h[r];
    hn += hp[m] * hp[m];
  }
  hn = sqrt(hn);
  double ap[4];
  /* phi(lambda) = sum (hp/(lambda - q))^2 falls from +inf (just above q_top)
   * to at most 1 at lambda = q_top + |h| */
  double lo = q[top], hi = q[top] + hn;
  double phi_lo = 0;
  int hard = fabs(hp[top]) <= 1e-300;
  if (hard) { /* h has no component along the top eigenvector */
    for (int m = 0; m < 4; m++)
      if (m != top && q[m] < q[top]) phi_lo += (hp[m] / (q[top] - q[m])) * (hp[m] / (q[top] - q[m]));
  }
  if (!(hi > lo)) { /* |h| negligible against q_top: the top eigenvector */
    for (int m = 0; m < 4; m++) ap[m] = m == top;
  } else if (hard && phi_lo <= 1) {
    for (int m = 0; m < 4; m++) ap[m] = (m == top || !(q[m] < q[top])) ? 0 : hp[m] / (q[top] - q[m]);
    ap[top] = sqrt(1 - phi_lo);
  } else {
    for (int it = 0; it < 200; it++) {
      double mid = 0.5 * (lo + hi);
      if (!(mid > lo && mid < hi)) break;
      double phi = 0;
      for (int m = 0; m < 4; m++) phi += (hp[m] / (mid - q[m])) * (hp[m] / (mid - q[m]));
      if (phi > 1) lo = mid; else hi = mid;
    }
    double n2 = 0;
    for (int m = 0; m < 4; m++) {
      ap[m] = hp[m] / (hi - q[m]);
      n2 += ap[m] * ap[m];
    }
    for (int m = 0; m < 4; m++) ap[m] /= sqrt(n2);
  }
  for (int r = 0; r < 4; r++) {
    a[r] = 0;
    for (int m = 0; m < 4; m++) a[r] += V[r][m] * ap[m];
  }
}

/* the three subgroup steps with exact maximisation, over-relaxed like the
 * linearised ones: a = normalise((1 - omega) e0 + omega a*) */
static void subgroup_steps_exact(const ocx M[72], ocx g[9], double omega) {
  static const int SUB[3][2] = {{0, 1}, {1, 2}, {0, 2}};
  for (int qq = 0; qq < 3; qq++) {
    int i = SUB[qq][0], j = SUB[qq][1], kk = 3 - i - j;
    double Q[16] = {0}, h[4] = {0};
    for (int k = 0; k < 8; k++) {
      ocx Y[9];
      m_mul(g, M + 9 * k, Y);
      ocx b[4] = {Y[3 * i + i] + Y[3 * j + j], I * (Y[3 * j + i] + Y[3 * i + j]), Y[3 * j + i] - Y[3 * i + j],
                  I * (Y[3 * i + i] - Y[3 * j + j])};
      ocx c = Y[3 * kk + kk];
      for (int r = 0; r < 4; r++) {
        h[r] += creal(conj(c) * b[r]);
        for (int t = 0; t < 4; t++) Q[4 * r + t] += creal(b[r] * conj(b[t]));
      }
    }
    double a[4];
    or_sphere_max(Q, h, a);
    a[0] = (1 - omega) + omega * a[0];
    for (int k = 1; k < 4; k++) a[k] = omega * a[k];
    double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
    if (na == 0) continue;
    for (int k = 0; k < 4; k++) a[k] /= na;
    ocx S[9];
    m_ident(S);
    S[3 * i + i] = a[0] + I * a[3];
    S[3 * i + j] = a[2] + I * a[1];
    S[3 * j + i] = -a[2] + I * a[1];
    S[3 * j + j] = a[0] - I * a[3];
    m_mul_left(S, g);
  }
}

/* a site update with exact subgroup maximisation, repeated `hits` times */
void or_site_g_exact(const ocx M[8 * 9], double omega, int hits, ocx g[9]) {
  m_ident(g);
  for (int h = 0; h < hits; h++) subgroup_steps_exact(M, g, omega);
}

void or_site_g(const ocx M[8 * 9], double omega, ocx g[9]) {
  ocx X[9], Y[9];
  m_zero(X);
  for (int k = 0; k < 8; k++) m_axpy(conj(m_tr(M + 9 * k)), M + 9 * k, X);
  m_copy(Y, X);
  m_ident(g);
  subgroup_steps(Y, g, omega);
}

/* Re-linearisation hits: hit 1 is or_site_g; each further hit linearises the
 * local functional sum_k |tr(g' M_k)|^2 at the current g,
 * X_g = sum_k conj(tr(g M_k)) M_k, and runs the subgroup steps on Y = g X_g,
 * continuing g (g' = s g raises Re tr(g' X_g) = Re tr(s Y)); each hit is again
 * a minorise-maximise step. */
void or_site_g_hits(const ocx M[8 * 9], double omega, int hits, ocx g[9]) {
  or_site_g(M, omega, g);
  for (int h = 1; h < hits; h++) {
    ocx X[9], Y[9];
    m_zero(X);
    for (int k = 0; k < 8; k++) {
      ocx gm[9];
      m_mul(g, M + 9 * k, gm);
      m_axpy(conj(m_tr(gm)), M + 9 * k, X);
    }
    m_mul(g, X, Y);
    subgroup_steps(Y, g, omega);
  }
}

/* the eight links at x: W_mu(x), then W_mu(x - mu)^dagger */
static void gather8(const lat_t *lt, const ocx *W, int64_t x, ocx M[72]) {
  for (int mu = 0; mu < 4; mu++) {
    m_copy(M + 9 * mu, link(W, x, mu));
    m_adj(link(W, shift(lt, x, mu, -1), mu), M + 9 * (4 + mu));
  }
}

void or_site_g_at(const int32_t L[4], const ocx *W, int64_t site,
                  double omega, ocx g[9]) {
  lat_t lt = mklat(L);
  ocx M[72];
  gather8(&lt, W, site, M);
  or_site_g(M, omega, g);
}

/* update every site of one parity; such sites share no link */
void or_halfsweep(const int32_t L[4], ocx *W, ocx *G, int parity,
                  double omega) {
  or_halfsweep_hits(L, W, G, parity, omega, 1);
}
void or_halfsweep_hits(const int32_t L[4], ocx *W, ocx *G, int parity,
                       double omega, int hits) {
  or_halfsweep_v(L, W, G, parity, omega, hits, 0);
}
/* exact != 0: exact per-subgroup maximisation (or_site_g_exact) */
void or_halfsweep_v(const int32_t L[4], ocx *W, ocx *G, int parity,
                    double omega, int hits, int exact) {
  lat_t lt = mklat(L);
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < lt.V; x++) {
    if (parity_of(&lt, x) != parity) continue;
    ocx M[72], g[9], gd[9];
    gather8(&lt, W, x, M);
    if (exact)
      or_site_g_exact(M, omega, hits, g);
    else
      or_site_g_hits(M, omega, hits, g);
    m_adj(g, gd);
    for (int mu = 0; mu < 4; mu++) {
      m_mul_left(g, link_w(W, x, mu));
      m_mul_right(link_w(W, shift(&lt, x, mu, -1), mu), gd);
    }
    m_mul_left(g, G + 9 * x);
  }
}

/* (1/V) sum_x |TA X(x)|_F^2 ; zero exactly at a stationary point of R */
double or_theta(const int32_t L[4], const ocx *W) {
  lat_t lt = mklat(L);
  double *a = malloc(lt.V * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < lt.V; x++) {
    ocx M[72], X[9], T[9];
    gather8(&lt, W, x, M);
    m_zero(X);
    for (int k = 0; k < 8; k++) m_axpy(conj(m_tr(M + 9 * k)), M + 9 * k, X);
    m_ta(X, T);
    a[x] = m_dot(T, T);
  }
  double s = kahan(a, lt.V);
  free(a);
  return s / lt.V;
}

static void reunit_all(const lat_t *lt, ocx *G) {
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < lt->V; x++) or_reunit(G + 9 * x);
}

/* Iterate full (even, then odd) sweeps from the start transform G until
 * R_s - R_{s-1} < tol or max_sweeps.  Sweeps are numbered globally,
 * s = start_sweep + k for the k-th sweep of this call.  The transform is
 * re-unitarised, and the working field re-derived from U, before every
 * sweep with (s-1) % reunit_every == 0 except the first of the call (whose
 * working field has just been derived from G), and once more at exit.  So a
 * run stopped at a multiple of reunit_every and resumed with start_sweep
 * repeats the bits of an uninterrupted run.
 * traj (nullable, max_sweeps+1 entries) receives R before sweep 1 and
 * after each sweep. */
int or_mcg_fix(const int32_t L[4], const ocx *U, ocx *G, double tol,
               int32_t max_sweeps, double omega, int32_t reunit_every,
               int32_t start_sweep, double *traj, or_fix_result *res) {
  return or_mcg_fix_v(L, U, G, tol, max_sweeps, omega, reunit_every,
                      start_sweep, 1, 1, 0, traj, res);
}
/* variants of the update rule: `hits` re-linearisation hits per site visit
 * (exact != 0: exact per-subgroup maximisation instead, repeated `hits`
 * times); the stop test only after sweeps whose global number
 * (start_sweep + k) is a multiple of stop_every */
int or_mcg_fix_v(const int32_t L[4], const ocx *U, ocx *G, double tol,
                 int32_t max_sweeps, double omega, int32_t reunit_every,
                 int32_t start_sweep, int32_t hits, int32_t stop_every,
                 int32_t exact, double *traj, or_fix_result *res) {
  lat_t lt = mklat(L);
  ocx *W = malloc((size_t)lt.V * 36 * sizeof(ocx));
  or_apply_gauge(L, U, G, W);
  double Rprev = or_functional(L, W);
  if (traj) traj[0] = Rprev;
  int status = 1, done = 0;
  double dR = 0;
  for (int k = 1; k <= max_sweeps; k++) {
    int s = start_sweep + k;
    if (reunit_every > 0 && k > 1 && (s - 1) % reunit_every == 0) {
      reunit_all(&lt, G);
      or_apply_gauge(L, U, G, W);
      Rprev = or_functional(L, W);
    }
    or_halfsweep_v(L, W, G, 0, omega, hits, exact);
    or_halfsweep_v(L, W, G, 1, omega, hits, exact);
    double R = or_functional(L, W);
    if (traj) traj[k] = R;
    dR = R - Rprev;
    done = k;
    if (s % stop_every == 0 && dR < tol) {
      status = 0;
      break;
    }
    Rprev = R;
  }
  reunit_all(&lt, G);
  or_apply_gauge(L, U, G, W);
  res->R = or_functional(L, W);
  res->dR = dR;
  res->theta = or_theta(L, W);
  res->sweeps = done;
  res->status = status;
  free(W);
  return status;
}

/* ========================================================================
 * Centre projection and P-vortices (Sec. II.A)
 * ====================================================================== */

/* Z_mu(x) = exp(2 pi i m / 3) with m the centre phase nearest to the phase
 * of t = tr(G(x) U_mu(x) G(x+mu)^dag): m maximises Re(t e^{-2 pi i m/3}),
 * candidates tried in the order 0, +1, -1 (first wins a tie); t = 0 gives
 * m = 0.  margin = pi/3 - |arg(t e^{-2 pi i m/3})|.  G may be NULL. */
void or_center_project(const int32_t L[4], const ocx *U, const ocx *G,
                       int8_t *Z, double *margin) {
  lat_t lt = mklat(L);
  static const int cand[3] = {0, 1, -1};
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < lt.V; x++)
    for (int mu = 0; mu < 4; mu++) {
      ocx W[9];
      if (G) {
        ocx t1[9], gd[9];
        m_mul(G + 9 * x, link(U, x, mu), t1);
        m_adj(G + 9 * shift(&lt, x, mu, +1), gd);
        m_mul(t1, gd, W);
      } else {
        m_copy(W, link(U, x, mu));
      }
      ocx t = m_tr(W);
      int best = 0;
      double mg = 0;
      if (t != 0) {
        double rbest = -INFINITY;
        for (int c = 0; c < 3; c++) {
          double r = creal(t * cexp(-2.0 * M_PI * I * cand[c] / 3.0));
          if (r > rbest) {
            rbest = r;
            best = cand[c];
          }
        }
        mg = M_PI / 3.0 - fabs(carg(t * cexp(-2.0 * M_PI * I * best / 3.0)));
      }
      Z[4 * x + mu] = (int8_t)best;
      if (margin) margin[4 * x + mu] = mg;
    }
}

/* Sec. III.B: a field splits into its projected centre part Z and the rest,
 * U^G = Z (Z^dagger U^G); the vortex-removed field is Z^dagger U^G. */
void or_vortex_field(const int32_t L[4], const ocx *U, const ocx *G,
                     const int8_t *Z, int mode, ocx *out) {
  lat_t lt = mklat(L);
  if (mode == 1) {
    if (G)
      or_apply_gauge(L, U, G, out);
    else
      memcpy(out, U, sizeof(ocx) * 36 * lt.V);
  }
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < lt.V; x++)
    for (int mu = 0; mu < 4; mu++) {
      ocx z = cexp(2.0 * M_PI * I * Z[4 * x + mu] / 3.0);
      ocx *o = link_w(out, x, mu);
      if (mode == 0) {
        m_ident(o);
        for (int k = 0; k < 9; k++) o[k] *= z;
      } else {
        for (int k = 0; k < 9; k++) o[k] *= conj(z);
      }
    }
}

double or_wilson_path(const int32_t L[4], const ocx *U, const int *spatial,
                      int n, int t) {
  lat_t lt = mklat(L);
  int len = 2 * (n + t);
  int *st = malloc(len * sizeof(int));
  int k = 0;
  for (int q = 0; q < n; q++) st[k++] = spatial[q];
  for (int q = 0; q < t; q++) st[k++] = 4;
  for (int q = n - 1; q >= 0; q--) st[k++] = -spatial[q];
  for (int q = 0; q < t; q++) st[k++] = -4;
  double *a = malloc(lt.V * sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < lt.V; x++) {
    ocx P[9];
    walk(&lt, U, x, st, len, P);
    a[x] = creal(m_tr(P)) / 3.0;
  }
  double s = kahan(a, lt.V);
  free(a);
  free(st);
  return s / lt.V;
}

/* n = (m_mu(x) + m_nu(x+mu) - m_mu(x+nu) - m_nu(x)) mod 3 for mu < nu; the
 * plaquette is a P-vortex when n != 0.  Planes in the order
 * (0,1),(0,2),(0,3),(1,2),(1,3),(2,3). */
void or_count_vortices(const int32_t L[4], const int8_t *Z, int64_t *total,
                       int64_t per_plane[6], int64_t per_charge[2],
                       int8_t *n_out) {
  lat_t lt = mklat(L);
  int64_t tot = 0, pp[6] = {0}, pc[2] = {0};
  for (int64_t x = 0; x < lt.V; x++) {
    int pl = 0;
    for (int mu = 0; mu < 4; mu++)
      for (int nu = mu + 1; nu < 4; nu++, pl++) {
        int s = Z[4 * x + mu] + Z[4 * shift(&lt, x, mu, +1) + nu] -
                Z[4 * shift(&lt, x, nu, +1) + mu] - Z[4 * x + nu];
        int n = ((s % 3) + 3) % 3;
        if (n_out) n_out[6 * x + pl] = (int8_t)n;
        if (n != 0) {
          tot++;
          pp[pl]++;
          pc[n - 1]++;
        }
      }
  }
  *total = tot;
  for (int k = 0; k < 6; k++) per_plane[k] = pp[k];
  per_charge[0] = pc[0];
  per_charge[1] = pc[1];
}

/* ========================================================================
 * L = R(S^G*) with S = n smearing steps of U, and its FP64 adjoint.
 * Gradients are ambient: grad_M L = dL/dRe M + i dL/dIm M, so that
 * dL = Re tr(grad^dag dM).
 * ====================================================================== */
double or_smear_loss(const int32_t L[4], const ocx *U, double rho, double eps,
                     int n, const ocx *Gstar) {
  lat_t lt = mklat(L);
  size_t bytes = (size_t)lt.V * 36 * sizeof(ocx);
  ocx *S = malloc(bytes), *W = malloc(bytes);
  or_smear(L, U, S, rho, eps, n);
  or_apply_gauge(L, S, Gstar, W);
  double r = or_functional(L, W);
  free(S);
  free(W);
  return r;
}

/* per-link forward quantities of one smearing step */
typedef struct {
  ocx Cp[9], Cr[9], C[9], A[9], E[9];
} step_fw;

static void step_forward_link(const lat_t *lt, const ocx *U, int64_t x, int mu,
                              double rho, double eps, step_fw *f) {
  double wp, wr;
  weights(eps, &wp, &wr);
  staple_parts(lt, U, x, mu, f->Cp, f->Cr);
  for (int k = 0; k < 9; k++) f->C[k] = rho * (wp * f->Cp[k] + wr * f->Cr[k]);
  ocx Ud[9], Om[9];
  m_adj(link(U, x, mu), Ud);
  m_mul(f->C, Ud, Om);
  m_ta(Om, f->A);
  or_exp_su3_eigen(f->A, f->E);
}

/* Tangent of one step: dU' = dE U + E dU with dE = L(A, TA(dC U^dag + C dU^dag)) */
void or_step_jvp(const int32_t L[4], const ocx *U, const ocx *dU, double rho,
                 double eps, ocx *dOut) {
  lat_t lt = mklat(L);
  double wp, wr;
  weights(eps, &wp, &wr);
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < lt.V; x++)
    for (int mu = 0; mu < 4; mu++) {
      step_fw f;
      step_forward_link(&lt, U, x, mu, rho, eps, &f);
      /* dC: product rule along every path */
      ocx dC[9];
      m_zero(dC);
      for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        for (int sg = 1; sg >= -1; sg -= 2)
          for (int w = 0; w < NPATH_PER_NU_SIGN; w++) {
            int st[5];
            int n = path_steps(mu, nu, sg, w, st);
            double wt = rho * (w == 0 ? wp : wr);
            for (int j = 0; j < n; j++) {
              /* product with factor j replaced by its tangent */
              ocx P[9];
              m_ident(P);
              int64_t y = x;
              for (int k = 0; k < n; k++) {
                int d = abs(st[k]) - 1;
                ocx fac[9];
                if (st[k] > 0) {
                  m_copy(fac, (k == j ? dU : U) + (y * 4 + d) * 9);
                  y = shift(&lt, y, d, +1);
                } else {
                  y = shift(&lt, y, d, -1);
                  m_adj((k == j ? dU : U) + (y * 4 + d) * 9, fac);
                }
                m_mul_right(P, fac);
              }
              m_axpy(wt, P, dC);
            }
          }
      }
      ocx Ud[9], dUd[9], t1[9], t2[9], dOm[9], dA[9], dE[9], o1[9], o2[9];
      m_adj(link(U, x, mu), Ud);
      m_adj(link(dU, x, mu), dUd);
      m_mul(dC, Ud, t1);
      m_mul(f.C, dUd, t2);
      for (int k = 0; k < 9; k++) dOm[k] = t1[k] + t2[k];
      m_ta(dOm, dA);
      exp_frechet(f.A, dA, dE);
      m_mul(dE, link(U, x, mu), o1);
      m_mul(f.E, link(dU, x, mu), o2);
      for (int k = 0; k < 9; k++) link_w(dOut, x, mu)[k] = o1[k] + o2[k];
    }
}

/* Cotangent of one step.  For U' = E U, E = exp(A), A = TA(Omega),
 * Omega = C U^dag, C = rho sum_paths w_path prod(path):
 *   grad_U += E^dag grad_U'
 *   grad_E  = grad_U' U^dag,  grad_A = L(A^dag, grad_E),  grad_Omega = TA(grad_A)
 *   grad_U += grad_Omega^dag C,  grad_C = grad_Omega U
 *   each factor V_j of a path gets w (V_1..V_{j-1})^dag grad_C (V_{j+1}..V_k)^dag
 *   (its dagger when the path walks the link backwards)
 *   dL/drho = sum <grad_C, C/rho>,  dL/deps = sum <grad_C, rho(-2/3 Cp + 1/12 Cr)>
 * absEps (nullable): sum over links of |<grad_C, rho(-2/3 Cp + 1/12 Cr)>|, the size of the
 * terms whose sum is dL/deps (they largely cancel, so this, not dL/deps, scales its rounding) */
void or_step_vjp(const int32_t L[4], const ocx *U, const ocx *gOut,
                 double rho, double eps, ocx *gU, double *dRho, double *dEps, double *absEps) {
  lat_t lt = mklat(L);
  double wp, wr;
  weights(eps, &wp, &wr);
  int64_t nl = 4 * lt.V;
  memset(gU, 0, (size_t)nl * 9 * sizeof(ocx));
  ocx *gC = malloc((size_t)nl * 9 * sizeof(ocx));
  double *dr = malloc(nl * sizeof(double)), *de = malloc(nl * sizeof(double));
  /* pass 1: per-link terms (independent across links) */
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < lt.V; x++)
    for (int mu = 0; mu < 4; mu++) {
      step_fw f;
      step_forward_link(&lt, U, x, mu, rho, eps, &f);
      const ocx *u = link(U, x, mu), *go = link(gOut, x, mu);
      ocx Ud[9], Ed[9], Ad[9], gE[9], gA[9], gOm[9], gOmd[9], t[9];
      m_adj(u, Ud);
      m_adj(f.E, Ed);
      m_adj(f.A, Ad);
      m_mul(go, Ud, gE);
      exp_frechet(Ad, gE, gA);
      m_ta(gA, gOm);
      ocx *gu = link_w(gU, x, mu);
      m_mul(Ed, go, t);
      m_axpy(1.0, t, gu);
      m_adj(gOm, gOmd);
      m_mul(gOmd, f.C, t);
      m_axpy(1.0, t, gu);
      ocx *gc = gC + (x * 4 + mu) * 9;
      m_mul(gOm, u, gc);
      ocx Cunit[9], dCde[9];
      for (int k = 0; k < 9; k++) {
        Cunit[k] = wp * f.Cp[k] + wr * f.Cr[k];
        dCde[k] = rho * (-2.0 / 3.0 * f.Cp[k] + 1.0 / 12.0 * f.Cr[k]);
      }
      dr[x * 4 + mu] = m_dot(gc, Cunit);
      de[x * 4 + mu] = m_dot(gc, dCde);
    }
  /* pass 2: scatter grad_C along the paths (serial: paths overlap) */
  for (int64_t x = 0; x < lt.V; x++)
    for (int mu = 0; mu < 4; mu++) {
      const ocx *gc = gC + (x * 4 + mu) * 9;
      for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        for (int sg = 1; sg >= -1; sg -= 2)
          for (int w = 0; w < NPATH_PER_NU_SIGN; w++) {
            int st[5];
            int n = path_steps(mu, nu, sg, w, st);
            double wt = rho * (w == 0 ? wp : wr);
            /* factors and the link each one is, walking the path */
            ocx fac[5][9];
            int64_t site[5];
            int dir[5];
            int64_t y = x;
            for (int k = 0; k < n; k++) {
              int d = abs(st[k]) - 1;
              if (st[k] > 0) {
                m_copy(fac[k], link(U, y, d));
                site[k] = y;
                y = shift(&lt, y, d, +1);
              } else {
                y = shift(&lt, y, d, -1);
                m_adj(link(U, y, d), fac[k]);
                site[k] = y;
              }
              dir[k] = d;
            }
            for (int j = 0; j < n; j++) {
              ocx pre[9], post[9], pred[9], postd[9], t1[9], c[9];
              m_ident(pre);
              for (int k = 0; k < j; k++) m_mul_right(pre, fac[k]);
              m_ident(post);
              for (int k = j + 1; k < n; k++) m_mul_right(post, fac[k]);
              m_adj(pre, pred);
              m_adj(post, postd);
              m_mul(pred, gc, t1);
              m_mul(t1, postd, c);
              ocx *dst = link_w(gU, site[j], dir[j]);
              if (st[j] > 0) {
                m_axpy(wt, c, dst);
              } else {
                ocx cd[9];
                m_adj(c, cd);
                m_axpy(wt, cd, dst);
              }
            }
          }
      }
    }
  *dRho = kahan(dr, nl);
  *dEps = kahan(de, nl);
  if (absEps) {
    for (int64_t q = 0; q < nl; q++) de[q] = fabs(de[q]);
    *absEps = kahan(de, nl);
  }
  free(gC);
  free(dr);
  free(de);
}

/* Gradient of L = R(S_n(U)^G*) at fixed G*.  With ckpt_every > 0 only every
 * ckpt_every-th smeared field is kept and the others are recomputed.  absEps
 * (nullable): the sum over steps and links of the magnitudes of the terms of
 * dL/deps (see or_step_vjp). */
void or_smear_loss_grad(const int32_t L[4], const ocx *U, double rho,
                        double eps, int n, const ocx *Gstar, int ckpt_every,
                        ocx *gradU, double *dRho, double *dEps, double *loss, double *absEps) {
  lat_t lt = mklat(L);
  int64_t nl = 4 * lt.V;
  size_t bytes = (size_t)nl * 9 * sizeof(ocx);
  if (ckpt_every <= 0 || ckpt_every > n) ckpt_every = n > 0 ? n : 1;
  int nck = n / ckpt_every + 1;
  ocx **ck = calloc(nck, sizeof(ocx *));
  ocx *cur = malloc(bytes), *nxt = malloc(bytes);
  memcpy(cur, U, bytes);
  for (int k = 0; k < n; k++) {
    if (k % ckpt_every == 0) {
      ck[k / ckpt_every] = malloc(bytes);
      memcpy(ck[k / ckpt_every], cur, bytes);
    }
    or_smear_step(L, cur, nxt, rho, eps);
    ocx *t = cur; cur = nxt; nxt = t;
  }
  /* cur = S_n.  grad wrt S of R(S^G): W = G S G'^dag, grad_W = 2c tr(W) 1 */
  double c = 1.0 / (9.0 * nl);
  ocx *g = malloc(bytes);
  {
    ocx *W = malloc(bytes);
    or_apply_gauge(L, cur, Gstar, W);
    *loss = or_functional(L, W);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < lt.V; x++)
      for (int mu = 0; mu < 4; mu++) {
        ocx gw[9], Gd[9], t1[9];
        m_zero(gw);
        ocx tw = m_tr(link(W, x, mu));
        gw[0] = gw[4] = gw[8] = 2.0 * c * tw;
        m_adj(Gstar + 9 * x, Gd);
        m_mul(Gd, gw, t1);
        m_mul(t1, Gstar + 9 * shift(&lt, x, mu, +1), link_w(g, x, mu));
      }
    free(W);
  }
  double drho = 0, deps = 0, aeps = 0;
  ocx *seg = malloc(bytes), *gnew = malloc(bytes);
  for (int k = n - 1; k >= 0; k--) {
    /* rebuild S_k from the nearest checkpoint at or below k */
    int base = (k / ckpt_every) * ckpt_every;
    memcpy(seg, ck[k / ckpt_every], bytes);
    for (int q = base; q < k; q++) {
      or_smear_step(L, seg, nxt, rho, eps);
      memcpy(seg, nxt, bytes);
    }
    double dr, de, ae;
    or_step_vjp(L, seg, g, rho, eps, gnew, &dr, &de, &ae);
    drho += dr;
    deps += de;
    aeps += ae;
    memcpy(g, gnew, bytes);
  }
  memcpy(gradU, g, bytes);
  *dRho = drho;
  *dEps = deps;
  if (absEps) *absEps = aeps;
  for (int q = 0; q < nck; q++) free(ck[q]);
  free(ck);
  free(cur);
  free(nxt);
  free(g);
  free(seg);
  free(gnew);
}
