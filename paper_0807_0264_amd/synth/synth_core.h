/*
 * synth_core.h -- seeded synthetic gauge-field generator.
 *
 * Inputs only: Haar-random SU(3) links and gauge transforms, random Z3
 * integers, Gaussian numbers, and thermalised-like fields from a
 * Cabibbo-Marinari heatbath of the Wilson plaquette action.  Nothing here
 * smears, gauge-fixes, projects or counts; the MCG method lives elsewhere.
 *
 * The same functions are compiled for the host (gcc, synth_cpu.c) and for
 * gfx950 (hipcc, synth_gpu.hip), both with -ffp-contract=off.  Every
 * floating-point step is an IEEE +, - or * written in a fixed order, and
 * every non-trivial function (reciprocal, square root, log, sin, cos) is
 * built here from those operations, so the two builds produce bit-identical
 * fields.
 *
 * Random numbers: counter-based.  draw(key, n) = mix(key ^ mix(n)) with mix
 * the SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014); a key
 * is derived from (seed, purpose).  Every draw is addressed by its own
 * counter, so results do not depend on thread count or visiting order.
 *
 * Field layout (interchange): link (site, mu) at
 *   ((site * 4 + mu) * 9 + 3 * row + col) * 2 + {0: re, 1: im}   (doubles)
 * site = x + Lx * (y + Ly * (z + Lz * t)).  Gauge fields: (site*9 + ..)*2.
 */
#ifndef SYNTH_CORE_H
#define SYNTH_CORE_H

#include <stdint.h>

#ifdef __HIPCC__
#define SY_FN __host__ __device__ static inline
#else
#define SY_FN static inline
#endif

/* ---- counter-based random numbers ------------------------------------- */
SY_FN uint64_t sy_mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
SY_FN uint64_t sy_key(uint64_t seed, uint64_t purpose) {
  return sy_mix(seed ^ sy_mix(purpose ^ 0x5DEECE66Dull));
}
SY_FN uint64_t sy_draw(uint64_t key, uint64_t n) { return sy_mix(key ^ sy_mix(n)); }
/* uniform in (0, 1] with 53 random bits */
SY_FN double sy_unit(uint64_t key, uint64_t n) {
  return (double)((sy_draw(key, n) >> 11) + 1) * (1.0 / 9007199254740992.0);
}

/* ---- arithmetic from +, -, * only ------------------------------------- */
SY_FN uint64_t sy_bits(double x) {
  union { double d; uint64_t u; } v;
  v.d = x;
  return v.u;
}
SY_FN double sy_from_bits(uint64_t u) {
  union { double d; uint64_t u; } v;
  v.u = u;
  return v.d;
}
/* 1/sqrt(x), x > 0 normal: bit-level first guess, then Newton steps */
SY_FN double sy_rsqrt(double x) {
  double y = sy_from_bits(0x5FE6EB50C7B537A9ull - (sy_bits(x) >> 1));
  double h = 0.5 * x;
  for (int k = 0; k < 6; k++) y = y * (1.5 - (h * y) * y);
  return y;
}
SY_FN double sy_sqrt(double x) { return x > 0.0 ? x * sy_rsqrt(x) : 0.0; }
/* 1/x, x != 0 normal: Newton on the magnitude */
SY_FN double sy_recip(double x) {
  double a = x < 0.0 ? -x : x;
  double r = sy_from_bits(0x7FDE623822FC16E6ull - sy_bits(a));
  for (int k = 0; k < 7; k++) r = r * (2.0 - a * r);
  return x < 0.0 ? -r : r;
}
/* natural log for normal x > 0: x = 2^e m, m in [sqrt(1/2), sqrt(2)),
 * log m = 2 atanh(s) with s = (m-1)/(m+1), |s| < 0.172 */
SY_FN double sy_log(double x) {
  uint64_t b = sy_bits(x);
  int e = (int)((b >> 52) & 0x7FF) - 1023;
  double m = sy_from_bits((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
  if (m > 1.4142135623730951) {
    m = m * 0.5;
    e = e + 1;
  }
  double s = (m - 1.0) * sy_recip(m + 1.0);
  double z = s * s;
  /* 1/(2k+1) for k = 0..13, folded at compile time */
  const double c[14] = {1.0 / 1.0,  1.0 / 3.0,  1.0 / 5.0,  1.0 / 7.0,  1.0 / 9.0,
                        1.0 / 11.0, 1.0 / 13.0, 1.0 / 15.0, 1.0 / 17.0, 1.0 / 19.0,
                        1.0 / 21.0, 1.0 / 23.0, 1.0 / 25.0, 1.0 / 27.0};
  double p = c[13];
  for (int k = 12; k >= 0; k--) p = p * z + c[k];
  double lm = 2.0 * s * p;
  return (double)e * 6.93147180369123816490e-01 + (lm + (double)e * 1.90821492927058770002e-10);
}
/* sin and cos of 2 pi r for r in [0, 1]: the reduction is exact on r */
SY_FN void sy_sincos_turn(double r, double *sn, double *cs) {
  double q4 = r * 4.0;
  int k = (int)(q4 + 0.5);
  double f = q4 - (double)k;           /* in [-1/2, 1/2] */
  double t = f * 1.5707963267948966;   /* in [-pi/4, pi/4] */
  double t2 = t * t;
  /* 1/((2n)(2n+1)) and 1/((2n-1)(2n)) for n = 1..10, folded at compile time */
  const double is[10] = {1.0 / 6.0,   1.0 / 20.0,  1.0 / 42.0,  1.0 / 72.0,  1.0 / 110.0,
                         1.0 / 156.0, 1.0 / 210.0, 1.0 / 272.0, 1.0 / 342.0, 1.0 / 420.0};
  const double ic[10] = {1.0 / 2.0,   1.0 / 12.0,  1.0 / 30.0,  1.0 / 56.0,  1.0 / 90.0,
                         1.0 / 132.0, 1.0 / 182.0, 1.0 / 240.0, 1.0 / 306.0, 1.0 / 380.0};
  double ps = 1.0, pc = 1.0;
  for (int n = 9; n >= 0; n--) {
    ps = 1.0 - (ps * t2) * is[n];
    pc = 1.0 - (pc * t2) * ic[n];
  }
  double s0 = t * ps, c0 = pc;
  switch (k & 3) {
  case 0: *sn = s0; *cs = c0; break;
  case 1: *sn = c0; *cs = -s0; break;
  case 2: *sn = -s0; *cs = -c0; break;
  default: *sn = -c0; *cs = s0; break;
  }
}
/* one standard normal from two uniforms (Box-Muller) */
SY_FN double sy_gauss(uint64_t key, uint64_t n) {
  double u1 = sy_unit(key, 2 * n), u2 = sy_unit(key, 2 * n + 1);
  double sn, cs;
  sy_sincos_turn(u2, &sn, &cs);
  return sy_sqrt(-2.0 * sy_log(u1)) * cs;
}

/* ---- complex 3x3 helpers (generator-local) ------------------------------ */
typedef struct { double re, im; } sy_c;
SY_FN sy_c sy_cmul(sy_c a, sy_c b) {
  sy_c r;
  r.re = a.re * b.re - a.im * b.im;
  r.im = a.re * b.im + a.im * b.re;
  return r;
}
SY_FN sy_c sy_cmulc(sy_c a, sy_c b) { /* a * conj(b) */
  sy_c r;
  r.re = a.re * b.re + a.im * b.im;
  r.im = a.im * b.re - a.re * b.im;
  return r;
}
SY_FN void sy_load(const double *p, sy_c m[9]) {
  for (int k = 0; k < 9; k++) { m[k].re = p[2 * k]; m[k].im = p[2 * k + 1]; }
}
SY_FN void sy_store(double *p, const sy_c m[9]) {
  for (int k = 0; k < 9; k++) { p[2 * k] = m[k].re; p[2 * k + 1] = m[k].im; }
}
/* c = a b, or a b^dag, or a^dag b */
SY_FN void sy_mm(const sy_c a[9], const sy_c b[9], sy_c c[9]) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      sy_c s = sy_cmul(a[3 * i], b[j]);
      for (int k = 1; k < 3; k++) {
        sy_c t = sy_cmul(a[3 * i + k], b[3 * k + j]);
        s.re = s.re + t.re;
        s.im = s.im + t.im;
      }
      c[3 * i + j] = s;
    }
}
SY_FN void sy_mmd(const sy_c a[9], const sy_c b[9], sy_c c[9]) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      sy_c s = sy_cmulc(a[3 * i], b[3 * j]);
      for (int k = 1; k < 3; k++) {
        sy_c t = sy_cmulc(a[3 * i + k], b[3 * j + k]);
        s.re = s.re + t.re;
        s.im = s.im + t.im;
      }
      c[3 * i + j] = s;
    }
}
SY_FN void sy_mdm(const sy_c a[9], const sy_c b[9], sy_c c[9]) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      sy_c s = sy_cmulc(b[j], a[i]);
      for (int k = 1; k < 3; k++) {
        sy_c t = sy_cmulc(b[3 * k + j], a[3 * k + i]);
        s.re = s.re + t.re;
        s.im = s.im + t.im;
      }
      c[3 * i + j] = s;
    }
}
/* rows 0,1 orthonormalised (Gram-Schmidt), row 2 = conj(row0 x row1) */
SY_FN void sy_reunit(sy_c m[9]) {
  double n0 = m[0].re * m[0].re + m[0].im * m[0].im + m[1].re * m[1].re +
              m[1].im * m[1].im + m[2].re * m[2].re + m[2].im * m[2].im;
  double i0 = sy_rsqrt(n0);
  for (int k = 0; k < 3; k++) { m[k].re = m[k].re * i0; m[k].im = m[k].im * i0; }
  sy_c ip = sy_cmulc(m[3], m[0]); /* <r0, r1> = sum conj(r0) r1 */
  for (int k = 1; k < 3; k++) {
    sy_c t = sy_cmulc(m[3 + k], m[k]);
    ip.re = ip.re + t.re;
    ip.im = ip.im + t.im;
  }
  for (int k = 0; k < 3; k++) {
    sy_c t = sy_cmul(ip, m[k]);
    m[3 + k].re = m[3 + k].re - t.re;
    m[3 + k].im = m[3 + k].im - t.im;
  }
  double n1 = m[3].re * m[3].re + m[3].im * m[3].im + m[4].re * m[4].re +
              m[4].im * m[4].im + m[5].re * m[5].re + m[5].im * m[5].im;
  double i1 = sy_rsqrt(n1);
  for (int k = 3; k < 6; k++) { m[k].re = m[k].re * i1; m[k].im = m[k].im * i1; }
  for (int k = 0; k < 3; k++) {
    int a = (k + 1) % 3, b = (k + 2) % 3;
    sy_c p = sy_cmul(m[a], m[3 + b]), q = sy_cmul(m[b], m[3 + a]);
    m[6 + k].re = p.re - q.re;
    m[6 + k].im = -(p.im - q.im);
  }
}
/* Haar-random SU(3): two complex Gaussian rows orthonormalised; the third
 * row conj(r0 x r1) fixes det = 1.  (The first two rows of a Haar U(3)
 * matrix and of a Haar SU(3) matrix have the same law.) */
SY_FN void sy_haar_su3(uint64_t key, uint64_t n, sy_c m[9]) {
  for (int k = 0; k < 6; k++) {
    m[k].re = sy_gauss(key, 12 * n + 2 * k);
    m[k].im = sy_gauss(key, 12 * n + 2 * k + 1);
  }
  for (int k = 6; k < 9; k++) { m[k].re = 0.0; m[k].im = 0.0; }
  sy_reunit(m);
}

/* ---- lattice ------------------------------------------------------------- */
typedef struct {
  int32_t L[4];
  int64_t V;
} sy_lat;

SY_FN int64_t sy_shift(const sy_lat *lt, int64_t i, int mu, int step) {
  int64_t c[4], r = i;
  for (int k = 0; k < 4; k++) { c[k] = r % lt->L[k]; r = r / lt->L[k]; }
  c[mu] = (c[mu] + step + lt->L[mu]) % lt->L[mu];
  return c[0] + (int64_t)lt->L[0] * (c[1] + (int64_t)lt->L[1] * (c[2] + (int64_t)lt->L[2] * c[3]));
}
SY_FN int sy_parity(const sy_lat *lt, int64_t i) {
  int64_t s = 0, r = i;
  for (int k = 0; k < 4; k++) { s += r % lt->L[k]; r = r / lt->L[k]; }
  return (int)(s & 1);
}
/* i-th site of the given parity (i < V/2); extents are even */
SY_FN int64_t sy_site_of_parity(const sy_lat *lt, int64_t i, int parity) {
  int64_t s = 2 * i;
  return sy_parity(lt, s) == parity ? s : s + 1;
}

/* ---- Cabibbo-Marinari heatbath for the Wilson action -------------------- */
#define SY_KP_TRIES 64

/* Sum of the six staples A such that the action's dependence on U_mu(x)
 * is (beta/3) Re tr(U_mu(x) A). */
SY_FN void sy_wilson_staple(const sy_lat *lt, const double *U, int64_t x,
                            int mu, sy_c A[9]) {
  for (int k = 0; k < 9; k++) { A[k].re = 0.0; A[k].im = 0.0; }
  int64_t xpm = sy_shift(lt, x, mu, 1);
  for (int nu = 0; nu < 4; nu++) {
    if (nu == mu) continue;
    int64_t xpn = sy_shift(lt, x, nu, 1), xmn = sy_shift(lt, x, nu, -1);
    int64_t xpmmn = sy_shift(lt, xpm, nu, -1);
    sy_c a[9], b[9], t[9], s[9];
    /* U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
    sy_load(U + (xpm * 4 + nu) * 18, a);
    sy_load(U + (xpn * 4 + mu) * 18, b);
    sy_mmd(a, b, t);
    sy_load(U + (x * 4 + nu) * 18, b);
    sy_mmd(t, b, s);
    for (int k = 0; k < 9; k++) { A[k].re = A[k].re + s[k].re; A[k].im = A[k].im + s[k].im; }
    /* U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu) = (U_mu(x-nu) U_nu(x+mu-nu))^dag U_nu(x-nu) */
    sy_load(U + (xmn * 4 + mu) * 18, a);
    sy_load(U + (xpmmn * 4 + nu) * 18, b);
    sy_mm(a, b, t);
    sy_load(U + (xmn * 4 + nu) * 18, b);
    sy_mdm(t, b, s);
    for (int k = 0; k < 9; k++) { A[k].re = A[k].re + s[k].re; A[k].im = A[k].im + s[k].im; }
  }
}

/* New value of link (x, mu) at heatbath sweep `sweep`.  For each SU(2)
 * subgroup (0,1),(1,2),(0,2) a left factor s is drawn from
 * exp((beta/3) Re tr(s w)) with w the 2x2 block of U A; the Kennedy-Pendleton
 * algorithm samples the quaternion component X0. */
SY_FN void sy_heatbath_update(const sy_lat *lt, const double *U, int64_t x,
                              int mu, double beta, uint64_t key, int sweep,
                              const sy_c A[9], sy_c u[9]);
SY_FN void sy_heatbath_link(const sy_lat *lt, const double *U, int64_t x,
                            int mu, double beta, uint64_t key, int sweep,
                            sy_c u[9]) {
  sy_c A[9];
  sy_wilson_staple(lt, U, x, mu, A);
  sy_heatbath_update(lt, U, x, mu, beta, key, sweep, A, u);
}

/* ---- Luscher-Weisz (plaquette + rectangle) action ------------------------
 * S = beta sum_P c0 (1 - Re tr P / 3) + beta sum_R c1 (1 - Re tr R / 3),
 * c0 = 5/3, c1 = -1/(12 u0^2) (u0 = 1: tree level).  Its dependence on
 * U_mu(x) is (beta/3) Re tr(U_mu(x) A) with A = c0 (6 plaquette staples) +
 * c1 (18 rectangle staples). */

/* product of the links along `steps` (+-(d+1)) from site y */
SY_FN void sy_walk(const sy_lat *lt, const double *U, int64_t y, const int *steps, int n, sy_c P[9]) {
  sy_c a[9], t[9];
  for (int k = 0; k < 9; k++) { P[k].re = (k % 4 == 0) ? 1.0 : 0.0; P[k].im = 0.0; }
  for (int q = 0; q < n; q++) {
    int d = (steps[q] > 0 ? steps[q] : -steps[q]) - 1;
    if (steps[q] > 0) {
      sy_load(U + (y * 4 + d) * 18, a);
      sy_mm(P, a, t);
      y = sy_shift(lt, y, d, 1);
    } else {
      y = sy_shift(lt, y, d, -1);
      sy_load(U + (y * 4 + d) * 18, a);
      sy_mmd(P, a, t);
    }
    for (int k = 0; k < 9; k++) P[k] = t[k];
  }
}

SY_FN void sy_lw_staple(const sy_lat *lt, const double *U, int64_t x, int mu, double c0, double c1,
                        sy_c A[9]) {
  for (int k = 0; k < 9; k++) { A[k].re = 0.0; A[k].im = 0.0; }
  const int64_t xpm = sy_shift(lt, x, mu, 1);
  const int M = mu + 1;
  for (int nu = 0; nu < 4; nu++) {
    if (nu == mu) continue;
    for (int sg = 1; sg >= -1; sg -= 2) {
      const int N = sg * (nu + 1);
      /* closing paths from x + mu back to x: plaquette, then the rectangles
       * 2x1 ahead, 2x1 behind (long in mu) and 1x2 (long in nu) */
      const int pl[3] = {N, -M, -N};
      const int r1[5] = {M, N, -M, -M, -N};
      const int r2[5] = {N, -M, -M, -N, M};
      const int r3[5] = {N, N, -M, -N, -N};
      sy_c P[9];
      sy_walk(lt, U, xpm, pl, 3, P);
      for (int k = 0; k < 9; k++) { A[k].re = A[k].re + c0 * P[k].re; A[k].im = A[k].im + c0 * P[k].im; }
      const int *rs[3] = {r1, r2, r3};
      for (int r = 0; r < 3; r++) {
        sy_walk(lt, U, xpm, rs[r], 5, P);
        for (int k = 0; k < 9; k++) { A[k].re = A[k].re + c1 * P[k].re; A[k].im = A[k].im + c1 * P[k].im; }
      }
    }
  }
}

/* Update colour of link (x, mu), 0..7: (x_mu mod 2) + 2 ((sum of the other
 * coordinates) mod 4).  Two links of direction mu in a common plaquette or
 * rectangle are displaced by +-nu, +-2 nu or +-mu +-nu (nu != mu) and so get
 * different colours (extents divisible by 4), so all links of one colour can
 * be updated at once. */
SY_FN int sy_lw_colour(const sy_lat *lt, int64_t i, int mu) {
  int64_t c[4], r = i, s = 0;
  for (int k = 0; k < 4; k++) { c[k] = r % lt->L[k]; r = r / lt->L[k]; }
  for (int k = 0; k < 4; k++)
    if (k != mu) s += c[k];
  return (int)(c[mu] & 1) + 2 * (int)(s & 3);
}

SY_FN void sy_heatbath_update(const sy_lat *lt, const double *U, int64_t x,
                              int mu, double beta, uint64_t key, int sweep,
                              const sy_c A[9], sy_c u[9]) {
  sy_load(U + (x * 4 + mu) * 18, u);
  const int SI[3] = {0, 1, 0}, SJ[3] = {1, 2, 2};
  for (int q = 0; q < 3; q++) {
    int i = SI[q], j = SJ[q];
    sy_c w[4]; /* w11 w12 w21 w22 of the (i,j) block of u A */
    const int ra[4] = {i, i, j, j}, cb[4] = {i, j, i, j};
    for (int e = 0; e < 4; e++) {
      sy_c s = sy_cmul(u[3 * ra[e]], A[cb[e]]);
      for (int k = 1; k < 3; k++) {
        sy_c t = sy_cmul(u[3 * ra[e] + k], A[3 * k + cb[e]]);
        s.re = s.re + t.re;
        s.im = s.im + t.im;
      }
      w[e] = s;
    }
    double v0 = w[0].re + w[3].re, v1 = -(w[1].im + w[2].im);
    double v2 = w[2].re - w[1].re, v3 = -(w[0].im - w[3].im);
    double k2 = v0 * v0 + v1 * v1 + v2 * v2 + v3 * v3;
    if (!(k2 > 1e-300)) continue;
    double kinv = sy_rsqrt(k2), kk = k2 * kinv;
    double alpha = beta * (1.0 / 3.0) * kk;
    double inv2a = sy_recip(2.0 * alpha);
    uint64_t base = ((((uint64_t)sweep * 4 + (uint64_t)mu) * (uint64_t)lt->V + (uint64_t)x) * 3 + (uint64_t)q) * SY_KP_TRIES;
    double delta = -1.0;
    uint64_t ctr = 0;
    for (int tr = 0; tr < SY_KP_TRIES; tr++) {
      ctr = (base + (uint64_t)tr) * 8;
      double r1 = sy_unit(key, ctr), r2 = sy_unit(key, ctr + 1);
      double r3 = sy_unit(key, ctr + 2), r4 = sy_unit(key, ctr + 3);
      double sn, cs;
      sy_sincos_turn(r2, &sn, &cs);
      double d = -(sy_log(r1) + (cs * cs) * sy_log(r3)) * inv2a;
      if (r4 * r4 <= 1.0 - d) {
        delta = d;
        break;
      }
    }
    if (delta < 0.0) continue; /* every try rejected: keep this subgroup */
    double x0 = 1.0 - 2.0 * delta;
    double xr = sy_sqrt(1.0 - x0 * x0 > 0.0 ? 1.0 - x0 * x0 : 0.0);
    double ct = 2.0 * sy_unit(key, ctr + 4) - 1.0;
    double st = sy_sqrt(1.0 - ct * ct > 0.0 ? 1.0 - ct * ct : 0.0);
    double sp, cp;
    sy_sincos_turn(sy_unit(key, ctr + 5), &sp, &cp);
    double X[4] = {x0, xr * st * cp, xr * st * sp, xr * ct};
    double b[4] = {v0 * kinv, v1 * kinv, v2 * kinv, v3 * kinv};
    /* s = S(X) S(b), S(a) = [[a0 + i a3, a2 + i a1], [-a2 + i a1, a0 - i a3]] */
    sy_c SX[4], SB[4], S2[4];
    SX[0].re = X[0]; SX[0].im = X[3]; SX[1].re = X[2]; SX[1].im = X[1];
    SX[2].re = -X[2]; SX[2].im = X[1]; SX[3].re = X[0]; SX[3].im = -X[3];
    SB[0].re = b[0]; SB[0].im = b[3]; SB[1].re = b[2]; SB[1].im = b[1];
    SB[2].re = -b[2]; SB[2].im = b[1]; SB[3].re = b[0]; SB[3].im = -b[3];
    for (int r = 0; r < 2; r++)
      for (int c = 0; c < 2; c++) {
        sy_c p = sy_cmul(SX[2 * r], SB[c]), t = sy_cmul(SX[2 * r + 1], SB[2 + c]);
        S2[2 * r + c].re = p.re + t.re;
        S2[2 * r + c].im = p.im + t.im;
      }
    /* rows i, j of u <- s (rows i, j of u) */
    for (int c = 0; c < 3; c++) {
      sy_c ui = u[3 * i + c], uj = u[3 * j + c];
      sy_c a1 = sy_cmul(S2[0], ui), a2 = sy_cmul(S2[1], uj);
      sy_c b1 = sy_cmul(S2[2], ui), b2 = sy_cmul(S2[3], uj);
      u[3 * i + c].re = a1.re + a2.re;
      u[3 * i + c].im = a1.im + a2.im;
      u[3 * j + c].re = b1.re + b2.re;
      u[3 * j + c].im = b1.im + b2.im;
    }
  }
}

/* purposes (second argument of sy_key) */
#define SY_P_HAAR_LINKS 1
#define SY_P_HEATBATH 2
#define SY_P_HAAR_GAUGE 3
#define SY_P_Z3 4
#define SY_P_GAUSS 5
#define SY_P_HEATBATH_LW 6

#endif
