/*
 * synth_gpu.hip -- gfx950 build of the seeded synthetic-field generator
 * (synth_core.h), for lattices too large to generate on the host in a few
 * seconds.  Bit-identical to synth_cpu.c; compiled with -ffp-contract=off.
 * Input generation only: it is not part of the MCG library.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "synth_core.h"

static sy_lat mk(const int32_t L[4]) {
  sy_lat lt;
  for (int k = 0; k < 4; k++) lt.L[k] = L[k];
  lt.V = (int64_t)L[0] * L[1] * L[2] * L[3];
  return lt;
}

__global__ void k_sy_haar(uint64_t key, int64_t n, double *out) {
  int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n) return;
  sy_c m[9];
  sy_haar_su3(key, (uint64_t)l, m);
  sy_store(out + l * 18, m);
}

__global__ void k_sy_heatbath(sy_lat lt, double *U, int mu, int par, double beta,
                              uint64_t key, int sweep) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= lt.V / 2) return;
  int64_t x = sy_site_of_parity(&lt, i, par);
  sy_c u[9];
  sy_heatbath_link(&lt, U, x, mu, beta, key, sweep, u);
  sy_store(U + (x * 4 + mu) * 18, u);
}

__global__ void k_sy_heatbath_lw(sy_lat lt, double *U, int mu, int col, double beta, double c0, double c1,
                                 uint64_t key, int sweep) {
  int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= lt.V || sy_lw_colour(&lt, x, mu) != col) return;
  sy_c A[9], u[9];
  sy_lw_staple(&lt, U, x, mu, c0, c1, A);
  sy_heatbath_update(&lt, U, x, mu, beta, key, sweep, A, u);
  sy_store(U + (x * 4 + mu) * 18, u);
}

__global__ void k_sy_reunit(int64_t n, double *U) {
  int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n) return;
  sy_c m[9];
  sy_load(U + l * 18, m);
  sy_reunit(m);
  sy_store(U + l * 18, m);
}

static int blocks(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

extern "C" {

/* all pointers are device pointers; returns a hipError_t value */
int sy_gpu_haar_links(const int32_t L[4], uint64_t seed, double *out, void *stream) {
  sy_lat lt = mk(L);
  hipStream_t s = (hipStream_t)stream;
  int64_t n = 4 * lt.V;
  k_sy_haar<<<blocks(n, 256), 256, 0, s>>>(sy_key(seed, SY_P_HAAR_LINKS), n, out);
  return (int)hipGetLastError();
}

int sy_gpu_haar_gauge(const int32_t L[4], uint64_t seed, uint64_t copy, double *out, void *stream) {
  sy_lat lt = mk(L);
  hipStream_t s = (hipStream_t)stream;
  uint64_t key = sy_key(sy_mix(seed ^ sy_mix(copy + 0x1234567ull)), SY_P_HAAR_GAUGE);
  k_sy_haar<<<blocks(lt.V, 256), 256, 0, s>>>(key, lt.V, out);
  return (int)hipGetLastError();
}

int sy_gpu_heatbath(const int32_t L[4], uint64_t seed, double beta, int nsweeps, double *U,
                    void *stream) {
  sy_lat lt = mk(L);
  hipStream_t s = (hipStream_t)stream;
  int rc = sy_gpu_haar_links(L, seed, U, stream);
  if (rc) return rc;
  uint64_t key = sy_key(seed, SY_P_HEATBATH);
  for (int sw = 0; sw < nsweeps; sw++) {
    for (int mu = 0; mu < 4; mu++)
      for (int par = 0; par < 2; par++)
        k_sy_heatbath<<<blocks(lt.V / 2, 128), 128, 0, s>>>(lt, U, mu, par, beta, key, sw);
    k_sy_reunit<<<blocks(4 * lt.V, 256), 256, 0, s>>>(4 * lt.V, U);
  }
  return (int)hipGetLastError();
}

int sy_gpu_heatbath_lw(const int32_t L[4], uint64_t seed, double beta, double u0, int nsweeps, double *U,
                       void *stream) {
  sy_lat lt = mk(L);
  hipStream_t s = (hipStream_t)stream;
  int rc = sy_gpu_haar_links(L, seed, U, stream);
  if (rc) return rc;
  uint64_t key = sy_key(seed, SY_P_HEATBATH_LW);
  const double c0 = 5.0 / 3.0, c1 = -sy_recip(12.0 * u0 * u0);
  for (int sw = 0; sw < nsweeps; sw++) {
    for (int mu = 0; mu < 4; mu++)
      for (int col = 0; col < 8; col++)
        k_sy_heatbath_lw<<<blocks(lt.V, 128), 128, 0, s>>>(lt, U, mu, col, beta, c0, c1, key, sw);
    k_sy_reunit<<<blocks(4 * lt.V, 256), 256, 0, s>>>(4 * lt.V, U);
  }
  return (int)hipGetLastError();
}

}  // extern "C"
