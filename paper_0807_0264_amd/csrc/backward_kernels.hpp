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
// every link, the path terms of all staples that contain it (no atomics), loop by loop.
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

// ---------------------------------------------------------- partial sums
// The loss and the two scalar derivatives from the per-block partials, laid out as the seed's
// nb_seed block sums and then, for each of the n steps, 3 nb entries: the (dL/drho, dL/deps) pair
// of each block, then the rectangle part of dL/deps of each block (zero where no kernel writes it).
// Block q (0: loss, 1: dL/drho, 2: dL/deps) sums its terms in a fixed order: thread t adds the
// terms t, t + 1024, ... of its sequence in turn (sixteen loads in flight), then block_sum, so the
// results do not depend on the launch.  A sequence is n runs of len terms, run k starting at
// base + k * 3 nb; term j of a run sits at offset off(j).
template <class F>
__device__ __forceinline__ double sum_runs(const double *base, int n, int len, long long nb3, F off) {
  double s = 0.0;
  int k = 0, j = threadIdx.x;  // this thread's next term: run k, index j
  while (j >= len && k < n) j -= len, k++;
  while (k < n) {
    double v[16];
    int m = 0;
#pragma unroll
    for (int u = 0; u < 16; u++) {
      v[u] = 0.0;
      if (k < n) {
        v[u] = base[(long long)k * nb3 + off(j)];
        m = u + 1;
        j += 1024;
        while (j >= len && k < n) j -= len, k++;
      }
    }
#pragma unroll
    for (int u = 0; u < 16; u++)
      if (u < m) s += v[u];
  }
  return s;
}
__global__ __launch_bounds__(1024) void k_reduce_parts(const double *__restrict__ part, int nb_seed, int n, int nb,
                                                       double *__restrict__ out) {
  const int q = blockIdx.x;
  const long long nb3 = 3LL * nb;
  double s;
  if (q == 0) s = sum_runs(part, 1, nb_seed, 0, [](int j) { return (long long)j; });
  else if (q == 1) s = sum_runs(part + nb_seed, n, nb, nb3, [](int j) { return 2LL * j; });
  else
    s = sum_runs(part + nb_seed, n, 2 * nb, nb3, [nb](int j) { return j < nb ? 2LL * j + 1 : (long long)nb + j; });
  s = block_sum<1024>(s);
  if (threadIdx.x == 0) out[q] = s;
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

// The adjoint kernels run one block per (tile, direction, parity), the tiles as gather_site lays
// them out: the eight blocks of a tile follow each other and each XCD takes a contiguous range of
// tiles (xcd_range), so a site's neighbours mostly share an XCD's L2 and the links of a tile are
// loaded while still cached; per-block partial sums are stored by (direction and parity, tile), so
// their summation order does not depend on which XCD runs a block or when.
// --------------------------------------------------------------- pass A
// STORED: Cst holds the staple sums Cp (and Cr, OI) of U, stored by the smearing kernel, and the
// pass reads them; otherwise it forms the staples itself (when the workspace for the sums does not
// fit).
template <typename T, bool OI, bool STORED>
__global__ __launch_bounds__(128) void k_step_adj_a(Geom g, const V2<T> *__restrict__ U,
                                                    const V2<T> *__restrict__ Cst,
                                                    const V2<T> *__restrict__ gOut, V2<T> *__restrict__ gU,
                                                    V2<T> *__restrict__ gC, T rho, T wp, T wr, double *part,
                                                    int *flag) {
  const int w = xcd_range((int)blockIdx.x, (int)gridDim.x), nT = (int)gridDim.x >> 3;
  const int tile = w >> 3, row = w & 7;
  const int h = gather_site(g, tile, (int)threadIdx.x);
  const int mu = row >> 1, par = row & 1;
  double drho = 0.0, deps = 0.0;
  if (h >= 0) {
    const Links<T> L{const_cast<V2<T> *>(U), g.Vh};
    M3<T> Cp, Cr;
    if constexpr (STORED) {
      Cp = Links<T>{const_cast<V2<T> *>(Cst), g.Vh}.load(mu, par, h);
      Cr = OI ? Links<T>{const_cast<V2<T> *>(Cst) + (size_t)72 * g.Vh, g.Vh}.load(mu, par, h) : m_zero<T>();
    } else {
      int c[4];
      coords_of(g, par, h, c);
      staples<T, OI>(g, L, c, mu, Cp, Cr);
    }
    // only C and dC/deps stay live through the adjoint of the exponential (C = rho Cu)
    M3<T> C, dC;
#pragma unroll
    for (int k = 0; k < 9; k++) {
      const cx<T> cu = OI ? wp * Cp.e[k] + wr * Cr.e[k] : wp * Cp.e[k];
      C.e[k] = rho * cu;
      dC.e[k] = OI ? rho * (T(-2.0 / 3.0) * Cp.e[k] + T(1.0 / 12.0) * Cr.e[k]) : rho * T(-2.0 / 3.0) * Cp.e[k];
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
    // d/drho of C is C / rho (Cu, the unscaled sum)
    drho = (double)rdot(gc, C) / (double)rho;
    // eps = 1 (stout): Cr is not formed here; its part of dC/deps is added by the rectangle-only
    // kernel launched for the derivative in eps (see k_eps_rect)
    deps = (double)rdot(gc, dC);
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
  const int h = gather_site(g, tile, (int)threadIdx.x);
  const int mu = row >> 1, par = row & 1;
  double deps = 0.0;
  if (h >= 0) {
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
// A staple term of C reaches a link through a closed loop: an output link l together with one of
// its staple paths.  Every such loop through a target link m = U_lam(y) is traversed here from m
// forwards, f_1 = m, f_2, ..., f_k (each a link or its dagger); the output link at position i
// (i >= 2) sends m the term w (f_2 .. f_{i-1} Gam_i f_{i+1} .. f_k)^dag, Gam_i being grad_C of
// that link, daggered when the loop walks it backwards (the factors of l's staple path before and
// after m, as the chain rule gives them, rearranged around the loop).  Summed over i the terms are
// the derivative of the product f_2 .. f_k along (Gam_2, .., Gam_k), built from the left with
// A <- A f_i + P Gam_i, P <- P f_i: 3k - 7 products and 2(k - 1) loads per loop instead of a
// product of the other k - 2 factors for each of the k - 1 outputs.
// Loops through U_lam(y) in the (lam, nu) plane for sg = +-1, as steps over L = +lam, N = sg nu:
//   S0: L  N -L -N          (plaquette: the stout staples)
//   S1: L  L  N -L -L -N    (2x1, m the first of the two links along lam)
//   S2: L  N -L -L -N  L    (2x1, m the second)
//   S3: L  N  N -L -N -N    (1x2)
// With the three other directions nu and both signs these are the 6 plaquettes and 18 rectangles
// that contain m, one per staple of each of their other links.
template <int S> struct Loop;
template <> struct Loop<0> {
  static constexpr int n = 4;
  static constexpr int sym[4] = {0, 1, 0, 1};  // 0 = L, 1 = N
  static constexpr int sgn[4] = {+1, +1, -1, -1};
};
template <> struct Loop<1> {
  static constexpr int n = 6;
  static constexpr int sym[6] = {0, 0, 1, 0, 0, 1};
  static constexpr int sgn[6] = {+1, +1, +1, -1, -1, -1};
};
template <> struct Loop<2> {
  static constexpr int n = 6;
  static constexpr int sym[6] = {0, 1, 0, 0, 1, 0};
  static constexpr int sgn[6] = {+1, +1, -1, -1, -1, +1};
};
template <> struct Loop<3> {
  static constexpr int n = 6;
  static constexpr int sym[6] = {0, 1, 1, 0, 1, 1};
  static constexpr int sgn[6] = {+1, +1, +1, -1, -1, -1};
};

// a b, or a b^dag
template <bool DAG, typename T> __device__ __forceinline__ M3<T> mul_o(const M3<T> &a, const M3<T> &b) {
  if constexpr (DAG) return mul_nd(a, b);
  else return mul(a, b);
}
// c += a b, or c += a b^dag
template <bool DAG, typename T> __device__ __forceinline__ void mac_o(const M3<T> &a, const M3<T> &b, M3<T> &c) {
  if constexpr (DAG) mac_nd(a, b, c);
  else mac(a, b, c);
}

// Steps K .. KEND-1 (K >= 1) of loop S (sign SG), from pos (left at the position after them): load
// f_K and Gam_K, advance the recurrence.  The sign is a template argument, so every dagger is known
// when the kernel is compiled.
template <typename T, int S, int SG, int K, int KEND, class LD>
__device__ __forceinline__ void loop_steps(const Geom &g, const LD &L, const Links<T> &GC, int pos[4], int lam,
                                           int nu, M3<T> &A, M3<T> &P) {
  if constexpr (K < KEND) {
    constexpr int sym = Loop<S>::sym[K], sgn = Loop<S>::sgn[K];
    constexpr bool back = (sym ? sgn * SG : sgn) < 0;
    const int d = sym ? nu : lam;
    int t[4];
    moved(g, pos, d, back ? -1 : +1, t);
    const int *at = back ? t : pos;
    const M3<T> f = L.at(g, at, d);
    const M3<T> G = GC.at(g, at, d);
    if constexpr (K == 1) {
      if constexpr (back) {
        A = dag(G);
        P = dag(f);
      } else {
        A = G;
        P = f;
      }
    } else {
      M3<T> a = mul_o<back>(A, f);
      mac_o<back>(P, G, a);
      A = a;
      if constexpr (K + 1 < Loop<S>::n) P = mul_o<back>(P, f);
    }
#pragma unroll
    for (int q = 0; q < 4; q++) pos[q] = t[q];
    loop_steps<T, S, SG, K + 1, KEND, LD>(g, L, GC, pos, lam, nu, A, P);
  }
}

template <typename T> __device__ __forceinline__ void add_dag(T w, const M3<T> &A, M3<T> &acc) {
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) acc.e[3 * i + j] = acc.e[3 * i + j] + w * conj(A.e[3 * j + i]);
}

// opaque copy of start coordinates: keeps the compiler from computing the addresses of every loop
// at once (a register-pressure hint with no run-time cost)
__device__ __forceinline__ void opaque_start(const int in[4], int out[4]) {
#pragma unroll
  for (int q = 0; q < 4; q++) out[q] = in[q];
  opaque_coords(out);
}

// The loops of one direction nu and sign SG through U_lam(y), added to acc with their weights.
// S0, S2 and S3 leave m along N through the same link, and S0 and S2 go on along -L through the
// same link too: those steps are taken once and the loops continue from copies of (A, P).
template <typename T, bool OI, int SG, class LD>
__device__ __forceinline__ void loops_of(const Geom &g, const LD &L, const Links<T> &GC, const int yl[4], int lam,
                                         int nu, T wp, T wr, M3<T> &acc) {
  M3<T> A, P;
  {  // S1: L L N -L -L -N
    if constexpr (OI) {
      int pos[4];
      opaque_start(yl, pos);
      loop_steps<T, 1, SG, 1, 6, LD>(g, L, GC, pos, lam, nu, A, P);
      add_dag(wr, A, acc);
    }
  }
  int pos[4];
  opaque_start(yl, pos);
  loop_steps<T, 0, SG, 1, 2, LD>(g, L, GC, pos, lam, nu, A, P);  // N, shared by S0, S2, S3
  if constexpr (OI) {  // S3: L N N -L -N -N
    int p3[4];
    opaque_start(pos, p3);
    M3<T> A3 = A, P3 = P;
    loop_steps<T, 3, SG, 2, 6, LD>(g, L, GC, p3, lam, nu, A3, P3);
    add_dag(wr, A3, acc);
  }
  loop_steps<T, 0, SG, 2, 3, LD>(g, L, GC, pos, lam, nu, A, P);  // -L, shared by S0 and S2
  if constexpr (OI) {  // S2: L N -L -L -N L
    int p2[4];
    opaque_start(pos, p2);
    M3<T> A2 = A, P2 = P;
    loop_steps<T, 2, SG, 3, 6, LD>(g, L, GC, p2, lam, nu, A2, P2);
    add_dag(wr, A2, acc);
  }
  loop_steps<T, 0, SG, 3, 4, LD>(g, L, GC, pos, lam, nu, A, P);  // S0: L N -L -N
  add_dag(wp, A, acc);
}

template <typename T, bool OI>
__global__ __launch_bounds__(128) void k_step_adj_b(Geom g, const V2<T> *__restrict__ U,
                                                    const V2<T> *__restrict__ gC, V2<T> *gU, T rho, T wp, T wr) {
  const int w = xcd_range((int)blockIdx.x, (int)gridDim.x);
  const int h = gather_site(g, w >> 3, (int)threadIdx.x);
  if (h < 0) return;
  const int lam = (w & 7) >> 1, par = w & 1;
  const Links<T> L{const_cast<V2<T> *>(U), g.Vh};
  const Links<T> GC{const_cast<V2<T> *>(gC), g.Vh}, GU{gU, g.Vh};
  int y[4];
  coords_of(g, par, h, y);
  M3<T> acc = GU.load(lam, par, h);
  const T wtp = rho * wp, wtr = rho * wr;
  int yl[4];  // the end of m: every loop's walk starts there
  moved(g, y, lam, +1, yl);
  for (int nu = 0; nu < 4; nu++) {
    if (nu == lam) continue;
    loops_of<T, OI, +1, Links<T>>(g, L, GC, yl, lam, nu, wtp, wtr, acc);
    loops_of<T, OI, -1, Links<T>>(g, L, GC, yl, lam, nu, wtp, wtr, acc);
  }
  GU.store(lam, par, h, acc);
}

}  // namespace mcg
