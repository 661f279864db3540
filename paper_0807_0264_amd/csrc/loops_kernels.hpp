// loops_kernels.hpp -- vortex-only / vortex-removed fields and Wilson loops
// (launchers in k_loops.hip).
#pragma once

#include "internal.hpp"

namespace mcg {

// site coordinates c moved by the spatial offset (o0, o1, o2) and dt in time,
// each |offset| < 2 L (periodic)
__device__ __forceinline__ void shifted(const Geom &g, const int c[4], int o0, int o1, int o2, int dt,
                                        int e[4]) {
  const int o[4] = {o0, o1, o2, dt};
#pragma unroll
  for (int k = 0; k < 4; k++) {
    int v = c[k] + o[k];
    v = v < 0 ? v + g.L[k] : v;
    v = v < 0 ? v + g.L[k] : v;
    v = v >= g.L[k] ? v - g.L[k] : v;
    v = v >= g.L[k] ? v - g.L[k] : v;
    e[k] = v;
  }
}

// z(m) = exp(2 pi i m / 3) for m in {-1, 0, 1}
__device__ __forceinline__ cx<double> center_elem(int m) {
  const double s3 = 0.86602540378443864676;  // sqrt(3)/2
  return m == 0 ? cx<double>{1.0, 0.0} : cx<double>{-0.5, m > 0 ? s3 : -s3};
}

// mode 0: out_mu(x) = z(m_mu(x)) 1; mode 1: out_mu(x) = conj(z(m_mu(x))) G(x) U_mu(x) G(x+mu)^dag
// (G may be null: identity).  One thread per half index h, both parities.  out may alias U: every
// element is read and written by the same thread.
template <typename T>
__global__ __launch_bounds__(256) void k_vortex_field(Geom g, const V2<T> *U, const double2 *__restrict__ G,
                                                      const int8_t *__restrict__ Z, int mode, V2<T> *out) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  if (h >= g.Vh) return;
  const Links<T> L{const_cast<V2<T> *>(U), g.Vh};
  const Links<T> O{out, g.Vh};
  const Gauge gg{const_cast<double2 *>(G), g.Vh};
  for (int par = 0; par < 2; par++) {
    int c[4];
    coords_of(g, par, h, c);
    const int i = lex_index(g, c);
    M3<double> Gx;
    if (mode == 1 && G) Gx = gg.load(par, h);
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
      const cx<double> z = center_elem(Z[(size_t)mu * g.V + i]);
      M3<double> r;
      if (mode == 0) {
        r = m_zero<double>();
        r.e[0] = r.e[4] = r.e[8] = z;
      } else {
        const M3<double> u = m_cvt<double>(L.load(mu, par, h));
        if (G) {
          int e[4];
          moved(g, c, mu, +1, e);
          r = mul_nd(mul(Gx, u), gg.load(1 - par, half_index(g, e)));
        } else {
          r = u;
        }
        const cx<double> zc = conj(z);
#pragma unroll
        for (int k = 0; k < 9; k++) r.e[k] = r.e[k] * zc;
      }
      O.store(mu, par, h, m_cvt<T>(r));
    }
  }
}

// For image blockIdx.y: line k of the image, out(x) = in(x) * (the path's links starting at
// x + (k - 1) d), in = line k - 1 (none for k = 1).  Line fields use the link layout with a single
// direction.  Grid: (2 * ceil(Vh / 256), images), the first half of x even sites, the second odd.
template <typename T>
__global__ __launch_bounds__(256) void k_line(Geom g, const V2<T> *__restrict__ U,
                                              const LoopImage<T> *__restrict__ imgs, int k) {
  const LoopImage<T> &im = imgs[blockIdx.y];
  const int nbp = gridDim.x >> 1;
  const int par = blockIdx.x >= nbp;
  // tiles of one parity in contiguous ranges per XCD (xcd_range)
  const int h = xcd_range((int)blockIdx.x - par * nbp, nbp) * 256 + threadIdx.x;
  if (h >= g.Vh) return;
  const Links<T> L{const_cast<V2<T> *>(U), g.Vh};
  const V2<T> *in = k == 1 ? nullptr : ((k & 1) ? im.b : im.a);
  V2<T> *out = (k & 1) ? im.a : im.b;
  int c[4];
  coords_of(g, par, h, c);
  M3<T> M = in ? Links<T>{const_cast<V2<T> *>(in), g.Vh}.load(0, par, h) : m_ident<T>();
  int y[4];
  shifted(g, c, (k - 1) * im.path.d[0], (k - 1) * im.path.d[1], (k - 1) * im.path.d[2], 0, y);
  for (int q = 0; q < im.path.n; q++) {
    const int st = im.path.s[q];
    const int a = (st > 0 ? st : -st) - 1;
    if (st > 0) {
      M = mul(M, L.at(g, y, a));
      int e[4];
      moved(g, y, a, +1, e);
#pragma unroll
      for (int q2 = 0; q2 < 4; q2++) y[q2] = e[q2];
    } else {
      int e[4];
      moved(g, y, a, -1, e);
#pragma unroll
      for (int q2 = 0; q2 < 4; q2++) y[q2] = e[q2];
      M = mul_nd(M, L.at(g, y, a));
    }
  }
  Links<T>{out, g.Vh}.store(0, par, h, M);
}

// For image blockIdx.y and every site x: the loops with spatial side S(x) (its line k, from x to
// x + D, D = k d) and time extents T = 1..tmax, Re tr[ S(x) B_T(x+D) S(x+T)^dag A_T(x)^dag ],
// A_T(y) = U_3(y) ... U_3(y+(T-1)), summed per block into
// part[(image * tmax + T - 1) * gridDim.x + blockIdx.x].  Each lane carries P = S(x) B_T(x+D) and
// A_T(x), one product each per T, and forms Q = A_T(x) S(x+T): Re tr(P Q^dag).
template <typename T, int BS>
__global__ __launch_bounds__(BS) void k_wloop(Geom g, const V2<T> *__restrict__ U,
                                              const LoopImage<T> *__restrict__ imgs, int k, int tmax,
                                              double *__restrict__ part) {
  const LoopImage<T> &im = imgs[blockIdx.y];
  const V2<T> *S = (k & 1) ? im.a : im.b;
  const int D0 = k * im.path.d[0], D1 = k * im.path.d[1], D2 = k * im.path.d[2];
  const int nbp = gridDim.x >> 1;
  const int par = blockIdx.x >= nbp;
  // tiles of one parity in contiguous ranges per XCD (xcd_range); the block sums are stored by tile
  const int tile = par * nbp + xcd_range((int)blockIdx.x - par * nbp, nbp);
  const int h = (tile - par * nbp) * BS + threadIdx.x;
  const bool live = h < g.Vh;
  const Links<T> L{const_cast<V2<T> *>(U), g.Vh};
  const Links<T> Sf{const_cast<V2<T> *>(S), g.Vh};
  int c[4] = {0, 0, 0, 0}, cd[4] = {0, 0, 0, 0};
  M3<T> P, A;
  if (live) {
    coords_of(g, par, h, c);
    shifted(g, c, D0, D1, D2, 0, cd);
    P = Sf.load(0, par, h);
    A = m_ident<T>();
  }
  double *pt = part + (size_t)blockIdx.y * tmax * gridDim.x;
  for (int t = 1; t <= tmax; t++) {
    double val = 0.0;
    if (live) {
      int e[4];
      shifted(g, c, 0, 0, 0, t - 1, e);
      A = mul(A, L.at(g, e, 3));
      shifted(g, cd, 0, 0, 0, t - 1, e);
      P = mul(P, L.at(g, e, 3));
      shifted(g, c, 0, 0, 0, t, e);
      const M3<T> Q = mul(A, Sf.load(0, parity_of(e), half_index(g, e)));
#pragma unroll
      for (int q = 0; q < 9; q++)
        val += (double)P.e[q].re * (double)Q.e[q].re + (double)P.e[q].im * (double)Q.e[q].im;
    }
    const double s = block_sum<BS>(val);
    if (threadIdx.x == 0) pt[(size_t)(t - 1) * gridDim.x + tile] = s;
  }
}

// res[t] += sum over the images, in order, of weight * sum_b part[(image * tmax + t) * nb + b]
// (each block sum in a fixed order); one block per t
template <typename T>
__global__ __launch_bounds__(256) void k_wloop_final(const double *__restrict__ part, int nb, int nimg, int tmax,
                                                     const LoopImage<T> *__restrict__ imgs, double *res) {
  double r = threadIdx.x == 0 ? res[blockIdx.x] : 0.0;
  for (int i = 0; i < nimg; i++) {
    const double s = sum_partials<256>(part + ((size_t)i * tmax + blockIdx.x) * nb, nb);
    if (threadIdx.x == 0) r += imgs[i].weight * s;
  }
  if (threadIdx.x == 0) res[blockIdx.x] = r;
}

__global__ __launch_bounds__(256) void k_zero(double *p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

}  // namespace mcg
