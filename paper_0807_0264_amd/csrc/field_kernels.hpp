// field_kernels.hpp -- layout conversion, gauge utilities and field sums (launchers in k_field.hip).
#pragma once

#include "internal.hpp"

namespace mcg {

static __device__ __forceinline__ void lex_coords(const Geom &g, int i, int c[4]) {
  int r = i / g.L[0];
  c[0] = i - r * g.L[0];
  int r2 = r / g.L[1];
  c[1] = r - r2 * g.L[1];
  c[3] = r2 / g.L[2];
  c[2] = r2 - c[3] * g.L[2];
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_pack_links(Geom g, const V2<Tin> *__restrict__ src,
                                                    V2<Tout> *__restrict__ dst) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l >= 4 * g.V) return;
  const int i = l >> 2, mu = l & 3;
  int c[4];
  lex_coords(g, i, c);
  const int par = parity_of(c), h = i >> 1;
  V2<Tout> *b = dst + (size_t)((mu * 2 + par) * 9) * g.Vh + h;
#pragma unroll
  for (int k = 0; k < 9; k++) {
    V2<Tin> v = src[(size_t)l * 9 + k];
    V2<Tout> w;
    w.x = (Tout)v.x;
    w.y = (Tout)v.y;
    b[(size_t)k * g.Vh] = w;
  }
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_unpack_links(Geom g, const V2<Tin> *__restrict__ src,
                                                      V2<Tout> *__restrict__ dst) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  if (l >= 4 * g.V) return;
  const int i = l >> 2, mu = l & 3;
  int c[4];
  lex_coords(g, i, c);
  const int par = parity_of(c), h = i >> 1;
  const V2<Tin> *b = src + (size_t)((mu * 2 + par) * 9) * g.Vh + h;
#pragma unroll
  for (int k = 0; k < 9; k++) {
    V2<Tin> v = b[(size_t)k * g.Vh];
    V2<Tout> w;
    w.x = (Tout)v.x;
    w.y = (Tout)v.y;
    dst[(size_t)l * 9 + k] = w;
  }
}

__global__ __launch_bounds__(256) void k_pack_gauge(Geom g, const double2 *__restrict__ src,
                                                    double2 *__restrict__ dst, int unpack) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= g.V) return;
  int c[4];
  lex_coords(g, i, c);
  const int par = parity_of(c), h = i >> 1;
#pragma unroll
  for (int k = 0; k < 9; k++) {
    const size_t soa = (size_t)(par * 9 + k) * g.Vh + h, aos = (size_t)i * 9 + k;
    if (unpack)
      dst[aos] = src[soa];
    else
      dst[soa] = src[aos];
  }
}

// what: 0 = identity, 1 = re-unitarise
__global__ __launch_bounds__(256) void k_gauge_op(Geom g, double2 *G, int what) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  if (h >= g.Vh) return;
  const Gauge gg{G, g.Vh};
  for (int par = 0; par < 2; par++) {
    M3<double> m;
    if (what == 0) {
      m = m_ident<double>();
    } else {
      m = gg.load(par, h);
      reunit(m);
    }
    gg.store(par, h, m);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_apply_gauge(Geom g, const V2<T> *U, const double2 *__restrict__ G,
                                                     V2<T> *out) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  if (h >= g.Vh) return;
  const Links<T> Ui{const_cast<V2<T> *>(U), g.Vh}, O{out, g.Vh};
  const Gauge gg{const_cast<double2 *>(G), g.Vh};
  for (int par = 0; par < 2; par++) {
    int c[4];
    coords_of(g, par, h, c);
    const M3<double> Gx = gg.load(par, h);
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
      int e[4];
      moved(g, c, mu, +1, e);
      const M3<double> Gn = gg.load(1 - par, half_index(g, e));
      const M3<double> u = m_cvt<double>(Ui.load(mu, par, h));
      O.store(mu, par, h, m_cvt<T>(mul_nd(mul(Gx, u), Gn)));
    }
  }
}

// what: 0 = sum |tr U|^2, 1 = sum_{mu<nu} Re tr U_P
template <typename T>
__global__ __launch_bounds__(256) void k_field_sum(Geom g, const V2<T> *__restrict__ U, double *part,
                                                   int what) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  double r = 0.0;
  if (h < g.Vh) {
    const Links<T> L{const_cast<V2<T> *>(U), g.Vh};
    for (int par = 0; par < 2; par++) {
      if (what == 0) {
#pragma unroll
        for (int mu = 0; mu < 4; mu++) r += tr2(L.load(mu, par, h));
      } else {
        int c[4];
        coords_of(g, par, h, c);
        M3<T> u[4];
#pragma unroll
        for (int mu = 0; mu < 4; mu++) u[mu] = L.load(mu, par, h);
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
          int e[4];
          moved(g, c, mu, +1, e);
#pragma unroll
          for (int nu = mu + 1; nu < 4; nu++) {
            int f[4];
            moved(g, c, nu, +1, f);
            // Re tr(U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag) = Re tr(P Q^dag)
            const M3<T> P = mul(u[mu], L.at(g, e, nu));
            const M3<T> Q = mul(u[nu], L.at(g, f, mu));
            r += (double)rdot(Q, P);
          }
        }
      }
    }
  }
  const double s = block_sum<256>(r);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// max over the nmu matrices per site (4: links, 1: a gauge field, FP64) of max_ij |(M M^dag - 1)_ij|,
// computed in FP64; a NaN anywhere in a matrix counts as +inf.  Per-block maxima into part.
template <typename T>
__global__ __launch_bounds__(256) void k_unitarity(Geom g, const V2<T> *__restrict__ U, int nmu, double *part) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  double dev = 0.0;
  if (h < g.Vh) {
    const Links<T> L{const_cast<V2<T> *>(U), g.Vh};
    for (int par = 0; par < 2; par++)
      for (int mu = 0; mu < nmu; mu++) {
        const M3<double> m = m_cvt<double>(L.load(mu, par, h));
        const M3<double> p = mul_nd(m, m);
#pragma unroll
        for (int k = 0; k < 9; k++) {
          const double re = p.e[k].re - ((k % 4 == 0) ? 1.0 : 0.0), im = p.e[k].im;
          const double a = fmax(fabs(re), fabs(im));
          dev = (a == a) ? fmax(dev, a) : __builtin_huge_val();
        }
      }
  }
  const double mx = -block_min<256>(-dev);
  if (threadIdx.x == 0) part[blockIdx.x] = mx;
}

__global__ __launch_bounds__(256) void k_max_final(const double *part, int n, double *out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v = fmax(v, part[i]);
  v = -block_min<256>(-v);
  if (threadIdx.x == 0) *out = v;
}

__global__ __launch_bounds__(256) void k_final_sum(const double *part, int n, double scale, double *out) {
  const double s = sum_partials<256>(part, n);
  if (threadIdx.x == 0) *out = s * scale;
}

}  // namespace mcg
