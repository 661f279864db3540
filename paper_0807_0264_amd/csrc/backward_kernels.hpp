// backward_kernels.hpp -- adjoint of one stout / over-improved stout step
// and the seed gradient of the smeared-field functional (launchers in
// k_backward.hip).
//
// Gradients are ambient: grad_M L = dL/dRe M + i dL/dIm M, so that
// dL = Re tr(grad^dag dM).  For one step U' = E U, E = exp(A), A = TA(Omega),
// Omega = C U^dag, C = rho sum_paths w_path prod(path):
//   grad_U  = E^dag grad_U' + grad_Omega^dag C + (path terms)
//   grad_E  = grad_U' U^dag
//   grad_A  = i M^dag,  M = s0 Q^2 + s1 Q + f1 Gam^dag + f2 (Q Gam^dag + Gam^dag Q)
//             with Gam = grad_E, Q = -iA, E = f0 + f1 Q + f2 Q^2 and
//             s0 = Re sum_j (df_j/dc0) tr(Gam^dag Q^j), s1 = Re sum_j (df_j/dc1) tr(Gam^dag Q^j)
//             (dc0 = tr(Q^2 dQ), dc1 = tr(Q dQ) for traceless dQ)
//   grad_Omega = TA(grad_A)  (TA is an orthogonal projection)
//   grad_C  = grad_Omega U
//   path terms: factor j of a path gets w (V_1..V_{j-1})^dag grad_C (V_{j+1}..V_k)^dag,
//   or its dagger when the path walks that link backwards.
// Pass A computes everything per link and stores grad_C; pass B gathers, for
// every link, the path terms of all staples that contain it (no atomics).
#pragma once

#include "internal.hpp"
#include "smear.hpp"

namespace mcg {

template <typename T> struct BwTerms;
template <> struct BwTerms<float> { static constexpr int N = 30; };
template <> struct BwTerms<double> { static constexpr int N = 40; };
// the unscaled series is used for spectral radius bound sqrt(4 c1 / 3) <= 4
constexpr double BW_MAX_R2 = 16.0;

template <typename T> __device__ __forceinline__ M3<T> cscale(cx<T> s, const M3<T> &a) {
  M3<T> c;
#pragma unroll
  for (int k = 0; k < 9; k++) c.e[k] = s * a.e[k];
  return c;
}
// tr(a^dag b) = sum_ij conj(a_ij) b_ij
template <typename T> __device__ __forceinline__ cx<T> trdot(const M3<T> &a, const M3<T> &b) {
  cx<T> s{T(0), T(0)};
#pragma unroll
  for (int k = 0; k < 9; k++) s = s + cmul(a.e[k], b.e[k]);
  return s;
}

// ------------------------------------------------------------------ seed
// L = (1/(9 N_l)) sum |tr W|^2 with W = G(x) S G(x+mu)^dag;
// grad_S = G(x)^dag (2c tr W) G(x+mu), c = 1/(9 N_l).
template <typename T>
__global__ __launch_bounds__(256) void k_loss_seed(Geom g, const V2<T> *__restrict__ S,
                                                   const double2 *__restrict__ G, V2<T> *__restrict__ grad,
                                                   double *part) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  double r = 0.0;
  if (h < g.Vh) {
    const Links<T> Ls{const_cast<V2<T> *>(S), g.Vh}, Lg{grad, g.Vh};
    const Gauge gg{const_cast<double2 *>(G), g.Vh};
    const double c = 1.0 / (9.0 * (double)(4 * g.V));
    for (int par = 0; par < 2; par++) {
      int cc[4];
      coords_of(g, par, h, cc);
      const M3<double> Gx = gg.load(par, h);
#pragma unroll
      for (int mu = 0; mu < 4; mu++) {
        int e[4];
        moved(g, cc, mu, +1, e);
        const M3<double> Gn = gg.load(1 - par, half_index(g, e));
        const M3<double> W = mul_nd(mul(Gx, m_cvt<double>(Ls.load(mu, par, h))), Gn);
        const cx<double> t = trace(W);
        r += t.re * t.re + t.im * t.im;
        Lg.store(mu, par, h, m_cvt<T>(cscale((2.0 * c) * t, mul_dn(Gx, Gn))));
      }
    }
  }
  const double s = block_sum<256>(r);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// The adjoint kernels run one block per (tile, direction, parity): the eight blocks of a tile follow
// each other and each XCD takes a contiguous range of tiles (xcd_range), so a site's neighbours
// mostly share an XCD's L2 and the links of a tile are loaded while still cached; per-block partial
// sums are stored by (direction and parity, tile), so their summation order does not depend on the
// mapping.
// --------------------------------------------------------------- pass A
template <typename T, bool OI>
__global__ __launch_bounds__(128) void k_step_adj_a(Geom g, const V2<T> *__restrict__ U,
                                                    const V2<T> *__restrict__ gOut, V2<T> *__restrict__ gU,
                                                    V2<T> *__restrict__ gC, T rho, T wp, T wr, double *part,
                                                    int *flag) {
  const int w = xcd_range((int)blockIdx.x, (int)gridDim.x), nT = (int)gridDim.x >> 3;
  const int tile = w >> 3, row = w & 7;
  const int h = tile * 128 + threadIdx.x;
  const int mu = row >> 1, par = row & 1;
  double drho = 0.0, deps = 0.0;
  if (h < g.Vh) {
    const Links<T> L{const_cast<V2<T> *>(U), g.Vh};
    int c[4];
    coords_of(g, par, h, c);
    M3<T> Cp, Cr;
    staples<T, OI>(g, L, c, mu, Cp, Cr);
    M3<T> Cu, C;
#pragma unroll
    for (int k = 0; k < 9; k++) {
      Cu.e[k] = OI ? wp * Cp.e[k] + wr * Cr.e[k] : wp * Cp.e[k];
      C.e[k] = rho * Cu.e[k];
    }
    const M3<T> u = L.load(mu, par, h);
    const M3<T> Q = minus_i(ta(mul_nd(C, u)));
    const M3<T> Q2 = mul(Q, Q);
    T c0, c1;
    ch_invariants(Q, Q2, c0, c1);
    if (T(4.0 / 3.0) * c1 > T(BW_MAX_R2)) atomicOr(flag, 1);
    CHCoef<T> co;
    ch_series<T, BwTerms<T>::N, true>(c0, c1, co);
    M3<T> E;
#pragma unroll
    for (int k = 0; k < 9; k++) E.e[k] = co.f[1] * Q.e[k] + co.f[2] * Q2.e[k];
    E.e[0] = E.e[0] + co.f[0];
    E.e[4] = E.e[4] + co.f[0];
    E.e[8] = E.e[8] + co.f[0];

    const M3<T> go = Links<T>{const_cast<V2<T> *>(gOut), g.Vh}.load(mu, par, h);
    const M3<T> Gam = mul_nd(go, u);  // grad_E
    // tr(Gam^dag Q^j), j = 0, 1, 2
    const cx<T> t0 = conj(trace(Gam)), t1 = trdot(Gam, Q), t2 = trdot(Gam, Q2);
    const T s0 = (co.df0[0] * t0 + co.df0[1] * t1 + co.df0[2] * t2).re;
    const T s1 = (co.df1[0] * t0 + co.df1[1] * t1 + co.df1[2] * t2).re;
    const M3<T> Gd = dag(Gam);
    M3<T> M = cscale(co.f[1], Gd);
    const M3<T> QG = mul(Q, Gd), GQ = mul(Gd, Q);
#pragma unroll
    for (int k = 0; k < 9; k++) M.e[k] = M.e[k] + s0 * Q2.e[k] + s1 * Q.e[k] + co.f[2] * (QG.e[k] + GQ.e[k]);
    // grad_A = i M^dag
    M3<T> gA;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) {
        const cx<T> m = M.e[3 * j + i];  // (M^dag)_ij = conj(m)
        gA.e[3 * i + j] = cx<T>{m.im, m.re};  // i * conj(m)
      }
    const M3<T> gOm = ta(gA);
    M3<T> gu = mul_dn(E, go);
    add_to(mul_dn(gOm, C), gu);
    const M3<T> gc = mul(gOm, u);
    Links<T>{gU, g.Vh}.store(mu, par, h, gu);
    Links<T>{gC, g.Vh}.store(mu, par, h, gc);
    drho = (double)rdot(gc, Cu);
    if (OI) {
      M3<T> dC;
#pragma unroll
      for (int k = 0; k < 9; k++) dC.e[k] = rho * (T(-2.0 / 3.0) * Cp.e[k] + T(1.0 / 12.0) * Cr.e[k]);
      deps = (double)rdot(gc, dC);
    } else {
      // eps = 1: Cr is not formed here; its term is added by the rectangle-only
      // kernel launched for the derivative in eps (see k_eps_rect)
      M3<T> dC = scale(rho * T(-2.0 / 3.0), Cp);
      deps = (double)rdot(gc, dC);
    }
  }
  const double a = block_sum<128>(drho);
  const double b = block_sum<128>(deps);
  if (threadIdx.x == 0) {
    const int blk = row * nT + tile;
    part[2 * blk] = a;
    part[2 * blk + 1] = b;
  }
}

// With eps = 1 the rectangle weight vanishes, but dC/deps = rho(-2/3 Cp + 1/12 Cr)
// still has a rectangle part: <grad_C, rho/12 Cr> per link.
template <typename T>
__global__ __launch_bounds__(128) void k_eps_rect(Geom g, const V2<T> *__restrict__ U,
                                                  const V2<T> *__restrict__ gC, T rho, double *part) {
  const int w = xcd_range((int)blockIdx.x, (int)gridDim.x), nT = (int)gridDim.x >> 3;
  const int tile = w >> 3, row = w & 7;
  const int h = tile * 128 + threadIdx.x;
  const int mu = row >> 1, par = row & 1;
  double deps = 0.0;
  if (h < g.Vh) {
    const Links<T> L{const_cast<V2<T> *>(U), g.Vh};
    int c[4];
    coords_of(g, par, h, c);
    M3<T> Cp, Cr;
    staples<T, true>(g, L, c, mu, Cp, Cr);
    const M3<T> gc = Links<T>{const_cast<V2<T> *>(gC), g.Vh}.load(mu, par, h);
    deps = (double)rdot(gc, scale(rho * T(1.0 / 12.0), Cr));
  }
  const double b = block_sum<128>(deps);
  if (threadIdx.x == 0) part[row * nT + tile] = b;
}

// --------------------------------------------------------------- pass B
// Staple paths of C_mu(x), from x to x+mu, as steps over two symbols:
// M = +mu and N = sg * nu (nu != mu, sg = +-1).
//   W0: N  M  -N            (plaquette)
//   W1: N  M  M  -N -M      (2x1 ahead)
//   W2: -M N  M  M  -N      (2x1 behind)
//   W3: N  N  M  -N -N      (1x2)
template <int W> struct Path;
template <> struct Path<0> {
  static constexpr int n = 3;
  static constexpr int sym[3] = {1, 0, 1};   // 0 = M, 1 = N
  static constexpr int sgn[3] = {+1, +1, -1};
};
template <> struct Path<1> {
  static constexpr int n = 5;
  static constexpr int sym[5] = {1, 0, 0, 1, 0};
  static constexpr int sgn[5] = {+1, +1, +1, -1, -1};
};
template <> struct Path<2> {
  static constexpr int n = 5;
  static constexpr int sym[5] = {0, 1, 0, 0, 1};
  static constexpr int sgn[5] = {-1, +1, +1, +1, -1};
};
template <> struct Path<3> {
  static constexpr int n = 5;
  static constexpr int sym[5] = {1, 1, 0, 1, 1};
  static constexpr int sgn[5] = {+1, +1, +1, -1, -1};
};

// The factor of step K of path W (K != J) joins the product before step J
// (pre) or after it (post); the first factor of each side is taken as it is
// (a product with the identity would cost a full 3x3 product: it cannot be
// folded away, because of signed zeros).
template <typename T, int K, int J>
__device__ __forceinline__ void take_factor(M3<T> &pre, M3<T> &post, const M3<T> &f, bool dagger) {
  if constexpr (K < J) {
    if constexpr (K == 0) pre = dagger ? dag(f) : f;
    else pre = dagger ? mul_nd(pre, f) : mul(pre, f);
  } else {
    if constexpr (K == J + 1) post = dagger ? dag(f) : f;
    else post = dagger ? mul_nd(post, f) : mul(post, f);
  }
}

// Walk path W from pos, step K onwards, collecting the factors of every step but J.
template <typename T, int W, int J, int K, class LD>
__device__ __forceinline__ void walk_path(const Geom &g, const LD &L, int pos[4], int mu, int nu, int sg,
                                          M3<T> &pre, M3<T> &post) {
  if constexpr (K < Path<W>::n) {
    constexpr int sym = Path<W>::sym[K], sgn = Path<W>::sgn[K];
    const int d = sym ? nu : mu, s = sym ? sgn * sg : sgn;
    int t[4];
    if (s > 0) {
      if constexpr (K != J) take_factor<T, K, J>(pre, post, L.at(g, pos, d), false);
      moved(g, pos, d, +1, t);
    } else {
      moved(g, pos, d, -1, t);
      if constexpr (K != J) take_factor<T, K, J>(pre, post, L.at(g, t, d), true);
    }
#pragma unroll
    for (int q = 0; q < 4; q++) pos[q] = t[q];
    walk_path<T, W, J, K + 1, LD>(g, L, pos, mu, nu, sg, pre, post);
  }
}

// Add to acc the terms of path W of C_mu(x) (over nu, sg) whose step J is the
// link (y, lnu) given by coordinates y.
template <typename T, int W, int J, class LD>
__device__ __forceinline__ void path_term(const Geom &g, const LD &L, const Links<T> &GC, const int y[4],
                                          int lnu, int mu, int nu, int sg, T wt, M3<T> &acc) {
  using P = Path<W>;
  const int dJ = P::sym[J] ? nu : mu;
  if (dJ != lnu) return;
  const int sJ = P::sym[J] ? P::sgn[J] * sg : P::sgn[J];
  // start of the path: undo the steps before J (and the backward step itself)
  int x[4] = {y[0], y[1], y[2], y[3]};
  if (sJ < 0) {
    int t[4];
    moved(g, x, dJ, +1, t);
    for (int k = 0; k < 4; k++) x[k] = t[k];
  }
#pragma unroll
  for (int k = J - 1; k >= 0; k--) {
    const int d = P::sym[k] ? nu : mu, s = P::sym[k] ? P::sgn[k] * sg : P::sgn[k];
    int t[4];
    moved(g, x, d, -s, t);
    for (int q = 0; q < 4; q++) x[q] = t[q];
  }
  // walk from x: factors before and after step J
  M3<T> pre, post;
  int pos[4] = {x[0], x[1], x[2], x[3]};
  walk_path<T, W, J, 0, LD>(g, L, pos, mu, nu, sg, pre, post);
  const M3<T> gc = GC.at(g, x, mu);
  M3<T> term;  // pre^dag gc post^dag, an empty side being the identity
  if constexpr (J == 0) term = mul_nd(gc, post);
  else if constexpr (J == P::n - 1) term = mul_dn(pre, gc);
  else term = mul_nd(mul_dn(pre, gc), post);
  if (sJ > 0) {
#pragma unroll
    for (int k = 0; k < 9; k++) acc.e[k] = acc.e[k] + wt * term.e[k];
  } else {
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) acc.e[3 * i + j] = acc.e[3 * i + j] + wt * conj(term.e[3 * j + i]);
  }
}

template <typename T, int W, class LD>
__device__ __forceinline__ void path_terms(const Geom &g, const LD &L, const Links<T> &GC, const int y[4],
                                           int lnu, int mu, int nu, int sg, T wt, M3<T> &acc) {
  path_term<T, W, 0, LD>(g, L, GC, y, lnu, mu, nu, sg, wt, acc);
  path_term<T, W, 1, LD>(g, L, GC, y, lnu, mu, nu, sg, wt, acc);
  path_term<T, W, 2, LD>(g, L, GC, y, lnu, mu, nu, sg, wt, acc);
  if (Path<W>::n == 5) {
    path_term<T, W, (Path<W>::n == 5 ? 3 : 0), LD>(g, L, GC, y, lnu, mu, nu, sg, wt, acc);
    path_term<T, W, (Path<W>::n == 5 ? 4 : 0), LD>(g, L, GC, y, lnu, mu, nu, sg, wt, acc);
  }
}

// U12: the links of U as their first two rows (the path factors; row 2 rebuilt as conj(r0 x r1)),
// two thirds of the bytes of the full matrices that each path term loads four of
template <typename T, bool OI>
__global__ __launch_bounds__(128) void k_step_adj_b(Geom g, const V2<T> *__restrict__ U12,
                                                    const V2<T> *__restrict__ gC, V2<T> *gU, T rho, T wp, T wr) {
  const int w = xcd_range((int)blockIdx.x, (int)gridDim.x);
  const int h = (w >> 3) * 128 + threadIdx.x;
  if (h >= g.Vh) return;
  const int lnu = (w & 7) >> 1, par = w & 1;
  const Links12<T> L{const_cast<V2<T> *>(U12), g.Vh};
  const Links<T> GC{const_cast<V2<T> *>(gC), g.Vh}, GU{gU, g.Vh};
  int y[4];
  coords_of(g, par, h, y);
  M3<T> acc = GU.load(lnu, par, h);
  const T wtp = rho * wp, wtr = rho * wr;
  for (int mu = 0; mu < 4; mu++)
    for (int nu = 0; nu < 4; nu++) {
      if (nu == mu) continue;
      for (int sg = 1; sg >= -1; sg -= 2) {
        path_terms<T, 0, Links12<T>>(g, L, GC, y, lnu, mu, nu, sg, wtp, acc);
        if (OI) {
          path_terms<T, 1, Links12<T>>(g, L, GC, y, lnu, mu, nu, sg, wtr, acc);
          path_terms<T, 2, Links12<T>>(g, L, GC, y, lnu, mu, nu, sg, wtr, acc);
          path_terms<T, 3, Links12<T>>(g, L, GC, y, lnu, mu, nu, sg, wtr, acc);
        }
      }
    }
  GU.store(lnu, par, h, acc);
}

}  // namespace mcg
