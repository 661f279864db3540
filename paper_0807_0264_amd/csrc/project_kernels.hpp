// project_kernels.hpp -- centre projection and vortex counting kernels (launchers in k_project.hip).
#pragma once

#include "internal.hpp"

namespace mcg {

template <typename T>
__global__ __launch_bounds__(256) void k_center_project(Geom g, const V2<T> *__restrict__ U,
                                                        const double2 *__restrict__ G,
                                                        int8_t *__restrict__ Z, double *part) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  double mmin = 10.0;
  if (h < g.Vh) {
    const Links<T> L{const_cast<V2<T> *>(U), g.Vh};
    const Gauge gg{const_cast<double2 *>(G), g.Vh};
    const double s3 = 0.86602540378443864676;  // sqrt(3)/2
    for (int par = 0; par < 2; par++) {
      int c[4];
      coords_of(g, par, h, c);
      const int i = lex_index(g, c);
      M3<double> Gx;
      if (G) Gx = gg.load(par, h);
#pragma unroll
      for (int mu = 0; mu < 4; mu++) {
        const M3<double> u = m_cvt<double>(L.load(mu, par, h));
        cx<double> t;
        if (G) {
          int e[4];
          moved(g, c, mu, +1, e);
          const M3<double> Gn = gg.load(1 - par, half_index(g, e));
          const M3<double> a = mul(Gx, u);
          // tr(a Gn^dag) = sum_ij a_ij conj(Gn_ij)
          t = cx<double>{0.0, 0.0};
#pragma unroll
          for (int k = 0; k < 9; k++) t = t + mulc(a.e[k], Gn.e[k]);
        } else {
          t = trace(u);
        }
        int m = 0;
        double margin = 0.0;
        if (t.re != 0.0 || t.im != 0.0) {
          const double r0 = t.re, rp = -0.5 * t.re + s3 * t.im, rm = -0.5 * t.re - s3 * t.im;
          double best = r0;
          if (rp > best) { best = rp; m = 1; }
          if (rm > best) { best = rm; m = -1; }
          // t e^{-2 pi i m/3}
          cx<double> rot = t;
          if (m == 1) rot = t * cx<double>{-0.5, -s3};
          if (m == -1) rot = t * cx<double>{-0.5, s3};
          margin = 1.04719755119659774615 - fabs(atan2(rot.im, rot.re));
        }
        Z[(size_t)mu * g.V + i] = (int8_t)m;
        mmin = fmin(mmin, margin);
      }
    }
  }
  const double s = block_min<256>(mmin);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_min_final(const double *part, int n, double *out) {
  double v = 10.0;
  for (int i = threadIdx.x; i < n; i += 256) v = fmin(v, part[i]);
  v = block_min<256>(v);
  if (threadIdx.x == 0) *out = v;
}

// Each thread walks sites i, i + grid size, ... and counts in registers; the block adds its counts
// (wave shuffles, then the four waves through LDS) and makes at most 12 atomic additions, so the
// integers meet in few atomics (one per site wave had serialised on the 12 counters: ~1 ms at
// 32^3x64).  Integer sums: the result does not depend on the order.
__global__ __launch_bounds__(256) void k_count_vortices(Geom g, const int8_t *__restrict__ Z,
                                                        unsigned long long *counts) {
  unsigned int cnt[12];
#pragma unroll
  for (int k = 0; k < 12; k++) cnt[k] = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < g.V; i += gridDim.x * 256) {
    int c[4];
    int r = i / g.L[0];
    c[0] = i - r * g.L[0];
    int r2 = r / g.L[1];
    c[1] = r - r2 * g.L[1];
    c[3] = r2 / g.L[2];
    c[2] = r2 - c[3] * g.L[2];
    int nb[4];
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
      int e[4];
      moved(g, c, mu, +1, e);
      nb[mu] = lex_index(g, e);
    }
    int m[4];
#pragma unroll
    for (int mu = 0; mu < 4; mu++) m[mu] = Z[(size_t)mu * g.V + i];
    int pl = 0;
#pragma unroll
    for (int mu = 0; mu < 4; mu++)
#pragma unroll
      for (int nu = mu + 1; nu < 4; nu++, pl++) {
        const int s = m[mu] + (int)Z[(size_t)nu * g.V + nb[mu]] - (int)Z[(size_t)mu * g.V + nb[nu]] - m[nu];
        const int n = ((s % 3) + 3) % 3;
        if (n == 1) cnt[2 * pl]++;
        if (n == 2) cnt[2 * pl + 1]++;
      }
  }
  __shared__ unsigned int wsum[4][12];
#pragma unroll
  for (int k = 0; k < 12; k++) {
    unsigned int v = cnt[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 12) {
    const unsigned long long v = (unsigned long long)wsum[0][threadIdx.x] + wsum[1][threadIdx.x] +
                                 wsum[2][threadIdx.x] + wsum[3][threadIdx.x];
    if (v) atomicAdd(&counts[threadIdx.x], v);
  }
}

}  // namespace mcg
