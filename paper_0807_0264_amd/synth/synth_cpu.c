/*
 * synth_cpu.c -- host build of the seeded synthetic-field generator
 * (synth_core.h).  Bit-identical to the gfx950 build in synth_gpu.hip.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "synth_core.h"

static sy_lat mk(const int32_t L[4]) {
  sy_lat lt;
  for (int k = 0; k < 4; k++) lt.L[k] = L[k];
  lt.V = (int64_t)L[0] * L[1] * L[2] * L[3];
  return lt;
}

/* Haar-random links, [V][4][3][3] complex as doubles */
void sy_cpu_haar_links(const int32_t L[4], uint64_t seed, double *out) {
  sy_lat lt = mk(L);
  uint64_t key = sy_key(seed, SY_P_HAAR_LINKS);
#pragma omp parallel for schedule(static)
  for (int64_t l = 0; l < 4 * lt.V; l++) {
    sy_c m[9];
    sy_haar_su3(key, (uint64_t)l, m);
    sy_store(out + l * 18, m);
  }
}

/* Haar-random gauge transform per site, [V][3][3]; `copy` selects an
 * independent stream (Gribov copies) */
void sy_cpu_haar_gauge(const int32_t L[4], uint64_t seed, uint64_t copy, double *out) {
  sy_lat lt = mk(L);
  uint64_t key = sy_key(sy_mix(seed ^ sy_mix(copy + 0x1234567ull)), SY_P_HAAR_GAUGE);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < lt.V; i++) {
    sy_c m[9];
    sy_haar_su3(key, (uint64_t)i, m);
    sy_store(out + i * 18, m);
  }
}

/* uniform Z3 integers m in {-1, 0, 1}, one per link, [V][4] */
void sy_cpu_z3(const int32_t L[4], uint64_t seed, int8_t *out) {
  sy_lat lt = mk(L);
  uint64_t key = sy_key(seed, SY_P_Z3);
#pragma omp parallel for schedule(static)
  for (int64_t l = 0; l < 4 * lt.V; l++) {
    uint64_t r = sy_draw(key, (uint64_t)l) >> 32;
    out[l] = (int8_t)((int)((r * 3) >> 32) - 1);
  }
}

/* n standard normals */
void sy_cpu_gauss(uint64_t seed, uint64_t stream, int64_t n, double *out) {
  uint64_t key = sy_key(sy_mix(seed ^ sy_mix(stream + 0x77ull)), SY_P_GAUSS);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; k++) out[k] = sy_gauss(key, (uint64_t)k);
}

/* Haar start, then nsweeps Cabibbo-Marinari heatbath sweeps of the Wilson
 * action at coupling beta.  A sweep visits mu = 0..3 and, within each mu,
 * the even then the odd sites; links of one (mu, parity) class do not
 * appear in each other's staples.  Links are re-unitarised after every
 * sweep. */
void sy_cpu_heatbath(const int32_t L[4], uint64_t seed, double beta, int nsweeps, double *U) {
  sy_lat lt = mk(L);
  sy_cpu_haar_links(L, seed, U);
  uint64_t key = sy_key(seed, SY_P_HEATBATH);
  int64_t half = lt.V / 2;
  for (int sw = 0; sw < nsweeps; sw++) {
    for (int mu = 0; mu < 4; mu++)
      for (int par = 0; par < 2; par++) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < half; i++) {
          int64_t x = sy_site_of_parity(&lt, i, par);
          sy_c u[9];
          sy_heatbath_link(&lt, U, x, mu, beta, key, sw, u);
          sy_store(U + (x * 4 + mu) * 18, u);
        }
      }
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < 4 * lt.V; l++) {
      sy_c m[9];
      sy_load(U + l * 18, m);
      sy_reunit(m);
      sy_store(U + l * 18, m);
    }
  }
}

/* Haar start, then nsweeps Cabibbo-Marinari heatbath sweeps of the
 * Luscher-Weisz action (c0 = 5/3, c1 = -1/(12 u0^2)) at coupling beta.  A
 * sweep visits mu = 0..3 and, within each mu, the eight link colours in turn
 * (sy_lw_colour); every extent must be divisible by 4.  Links are
 * re-unitarised after every sweep. */
void sy_cpu_heatbath_lw(const int32_t L[4], uint64_t seed, double beta, double u0, int nsweeps, double *U) {
  sy_lat lt = mk(L);
  sy_cpu_haar_links(L, seed, U);
  uint64_t key = sy_key(seed, SY_P_HEATBATH_LW);
  const double c0 = 5.0 / 3.0, c1 = -sy_recip(12.0 * u0 * u0);
  for (int sw = 0; sw < nsweeps; sw++) {
    for (int mu = 0; mu < 4; mu++)
      for (int col = 0; col < 8; col++) {
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < lt.V; x++) {
          if (sy_lw_colour(&lt, x, mu) != col) continue;
          sy_c A[9], u[9];
          sy_lw_staple(&lt, U, x, mu, c0, c1, A);
          sy_heatbath_update(&lt, U, x, mu, beta, key, sw, A, u);
          sy_store(U + (x * 4 + mu) * 18, u);
        }
      }
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < 4 * lt.V; l++) {
      sy_c m[9];
      sy_load(U + l * 18, m);
      sy_reunit(m);
      sy_store(U + l * 18, m);
    }
  }
}

/* the Luscher-Weisz staple and the update colour, exported for their tests */
void sy_cpu_lw_staple(const int32_t L[4], const double *U, int64_t x, int mu, double c0, double c1, double *A) {
  sy_lat lt = mk(L);
  sy_c a[9];
  sy_lw_staple(&lt, U, x, mu, c0, c1, a);
  sy_store(A, a);
}
int sy_cpu_lw_colour(const int32_t L[4], int64_t x, int mu) {
  sy_lat lt = mk(L);
  return sy_lw_colour(&lt, x, mu);
}

/* the generator's own elementary functions, exported for their tests */
double sy_cpu_log(double x) { return sy_log(x); }
double sy_cpu_sqrt(double x) { return sy_sqrt(x); }
double sy_cpu_recip(double x) { return sy_recip(x); }
void sy_cpu_sincos_turn(double r, double *s, double *c) { sy_sincos_turn(r, s, c); }
