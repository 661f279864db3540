// mcg_kernels.hpp -- kernels of the fixing iteration (launchers in k_mcg.hip).
#pragma once

#include "fix_types.hpp"
#include "internal.hpp"

namespace mcg {

template <typename T>
__device__ __forceinline__ int find_field(const LatDesc<T> *__restrict__ D, int B) {
  int b = 0;
  for (int i = 1; i < B; i++)
    if ((int)blockIdx.x >= D[i].blk0) b = i;
  return b;
}

// The field of this grid block and the block's index within the field: the
// whole-field mapping for slab < 0, else the chunk of slab `slab`.  A field
// whose chunk is empty has the same start as the next one and is skipped.
// rev: the tiles in reverse dispatch order, so a launch that follows one in
// the forward order starts on the tiles its predecessor touched last (which
// the last-level cache may still hold).  Workgroups are dealt to the eight
// XCDs in turn (block i to XCD i mod 8), so the reversal runs within each
// residue class mod 8: grid block x + 8j takes tile x + 8(c_x - 1 - j), c_x
// the number of blocks of residue x; every tile stays on the XCD (and its
// L2) that handles it in the forward order.
__device__ __forceinline__ int tile_of_block(int rev) {
  const int b = (int)blockIdx.x;
  if (!(rev & 1)) return b;
  const int n = (int)gridDim.x, x = b & 7;
  const int cx = (n >> 3) + (x < (n & 7) ? 1 : 0);
  return x + 8 * (cx - 1 - (b >> 3));
}

// rev & 2: within each field's n blocks (or its chunk of a slab), xcd_range gives the blocks of
// one XCD a contiguous range of tiles, so a site's neighbours a few tiles away along z mostly lie
// on the same XCD and meet in its L2.  Applied after the reversal above, it keeps every tile on
// one XCD in both directions.

template <typename T>
__device__ __forceinline__ int block_of(const LatDesc<T> *__restrict__ D, int B, int slab, int rev, int &local) {
  const int vb = tile_of_block(rev);
  if (slab < 0) {
    int b = 0;
    for (int i = 1; i < B; i++)
      if (vb >= D[i].blk0) b = i;
    local = vb - D[b].blk0;
    if (rev & 2) local = xcd_range(local, D[b].nblk);
    return b;
  }
  int b = 0;
  for (int i = 1; i < B; i++)
    if (vb >= D[i].sblk0[slab]) b = i;
  const int ns = D[b].nslab > 1 ? D[b].nslab : 1;
  const int lo = ns > 1 ? (slab * D[b].nblk) / ns : 0, hi = ns > 1 ? ((slab + 1) * D[b].nblk) / ns : D[b].nblk;
  const int i = vb - D[b].sblk0[slab];
  local = lo + ((rev & 2) ? xcd_range(i, hi - lo) : i);
  return b;
}

// ---------------------------------------------------------- local update
// One SU(2) subgroup step on rows/columns (I, J): the subgroup element
// s = a0 + i a.sigma maximising Re tr(s Y) is a* = v/|v| with
// v = (Re(y11+y22), -Im(y12+y21), Re(y21-y12), -Im(y11-y22)); it is
// over-relaxed to a = normalise((1-omega) e0 + omega a*) and applied from
// the left to Y and g.
template <typename T, int I, int J, bool UPDATE_Y>
__device__ __forceinline__ void su2_step(M3<T> &Y, M3<T> &g, T omega) {
  const cx<T> y11 = Y.e[4 * I], y12 = Y.e[3 * I + J], y21 = Y.e[3 * J + I], y22 = Y.e[4 * J];
  const T v0 = y11.re + y22.re, v1 = -(y12.im + y21.im);
  const T v2 = y21.re - y12.re, v3 = -(y11.im - y22.im);
  const T n2 = v0 * v0 + v1 * v1 + v2 * v2 + v3 * v3;
  if (!(n2 > T(0))) return;
  const T inv = T(1) / sqrt(n2);
  T a0 = (T(1) - omega) + omega * (v0 * inv);
  T a1 = omega * (v1 * inv), a2 = omega * (v2 * inv), a3 = omega * (v3 * inv);
  const T na2 = a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
  if (!(na2 > T(0))) return;
  const T ia = T(1) / sqrt(na2);
  a0 *= ia;
  a1 *= ia;
  a2 *= ia;
  a3 *= ia;
  const cx<T> s00{a0, a3}, s01{a2, a1}, s10{-a2, a1}, s11{a0, -a3};
#pragma unroll
  for (int c = 0; c < 3; c++) {
    if (UPDATE_Y) {
      const cx<T> yi = Y.e[3 * I + c], yj = Y.e[3 * J + c];
      Y.e[3 * I + c] = s00 * yi + s01 * yj;
      Y.e[3 * J + c] = s10 * yi + s11 * yj;
    }
    const cx<T> gi = g.e[3 * I + c], gj = g.e[3 * J + c];
    g.e[3 * I + c] = s00 * gi + s01 * gj;
    g.e[3 * J + c] = s10 * gi + s11 * gj;
  }
}

// the subgroup steps (0,1), (1,2), (0,2), each left-multiplying Y and g
template <typename T> __device__ __forceinline__ void subgroup_steps(M3<T> &Y, M3<T> &g, T omega) {
  su2_step<T, 0, 1, true>(Y, g, omega);
  su2_step<T, 1, 2, true>(Y, g, omega);
  su2_step<T, 0, 2, false>(Y, g, omega);
}

// g from the linearisation X = sum_k conj(tr M_k) M_k
template <typename T> __device__ __forceinline__ M3<T> local_update(M3<T> Y, T omega) {
  M3<T> g = m_ident<T>();
  subgroup_steps(Y, g, omega);
  return g;
}

// ------------------------------------------- exact subgroup maximisation
// argmax over the unit sphere of R^4 of a^T Q a + 2 h.a (Q symmetric, destroyed): cyclic Jacobi
// eigendecomposition Q = V diag(q) V^T, then the secular equation sum_m (h'_m / (lam - q_m))^2 = 1,
// h' = V^T h, for lam in [q_top, q_top + |h|] by bisection; a = V h' / (lam - q), normalised.  When h
// has no component along the top eigenvector and the rest of a is shorter than 1, lam = q_top.
__device__ __forceinline__ void sphere_max(double Q[4][4], const double h[4], double a[4]) {
  double V[4][4];
#pragma unroll
  for (int r = 0; r < 4; r++)
#pragma unroll
    for (int c = 0; c < 4; c++) V[r][c] = r == c ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 10; sweep++) {
    // converged: the off-diagonal part is below rounding against the diagonal
    double off = 0.0, dia = 0.0;
#pragma unroll
    for (int p = 0; p < 4; p++) {
      dia += Q[p][p] * Q[p][p];
#pragma unroll
      for (int q = p + 1; q < 4; q++) off += Q[p][q] * Q[p][q];
    }
    if (!(off > 1e-34 * dia)) break;
#pragma unroll
    for (int p = 0; p < 4; p++)
#pragma unroll
      for (int q = p + 1; q < 4; q++) {
        const double apq = Q[p][q];
        if (fabs(apq) > 1e-300) {
          const double th = (Q[q][q] - Q[p][p]) / (2.0 * apq);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
#pragma unroll
          for (int k = 0; k < 4; k++) {
            const double akp = Q[k][p], akq = Q[k][q];
            Q[k][p] = c * akp - sn * akq;
            Q[k][q] = sn * akp + c * akq;
          }
#pragma unroll
          for (int k = 0; k < 4; k++) {
            const double apk = Q[p][k], aqk = Q[q][k];
            Q[p][k] = c * apk - sn * aqk;
            Q[q][k] = sn * apk + c * aqk;
          }
#pragma unroll
          for (int k = 0; k < 4; k++) {
            const double vkp = V[k][p], vkq = V[k][q];
            V[k][p] = c * vkp - sn * vkq;
            V[k][q] = sn * vkp + c * vkq;
          }
        }
      }
  }
  double q[4], hp[4], hn = 0.0, qtop = Q[0][0];
  int top = 0;
#pragma unroll
  for (int m = 0; m < 4; m++) {
    q[m] = Q[m][m];
    if (q[m] > qtop) {
      qtop = q[m];
      top = m;
    }
    hp[m] = V[0][m] * h[0] + V[1][m] * h[1] + V[2][m] * h[2] + V[3][m] * h[3];
    hn += hp[m] * hp[m];
  }
  double htop = 0.0;
#pragma unroll
  for (int m = 0; m < 4; m++)
    if (m == top) htop = hp[m];
  double ap[4];
  double rest = 0.0;
  if (fabs(htop) <= 1e-300) {
#pragma unroll
    for (int m = 0; m < 4; m++)
      if (m != top && q[m] < qtop) rest += (hp[m] / (qtop - q[m])) * (hp[m] / (qtop - q[m]));
  }
  if (!(qtop + sqrt(hn) > qtop)) {  // |h| negligible against q_top: the top eigenvector
#pragma unroll
    for (int m = 0; m < 4; m++) ap[m] = m == top ? 1.0 : 0.0;
  } else if (fabs(htop) <= 1e-300 && rest <= 1.0) {
#pragma unroll
    for (int m = 0; m < 4; m++) ap[m] = (m == top || !(q[m] < qtop)) ? 0.0 : hp[m] / (qtop - q[m]);
#pragma unroll
    for (int m = 0; m < 4; m++)
      if (m == top) ap[m] = sqrt(1.0 - rest);
  } else {
    double lo = qtop, hi = qtop + sqrt(hn);
    for (int it = 0; it < 80; it++) {
      const double mid = 0.5 * (lo + hi);
      if (!(mid > lo && mid < hi)) break;  // the bracket cannot be split further
      double phi = 0.0;
#pragma unroll
      for (int m = 0; m < 4; m++) phi += (hp[m] / (mid - q[m])) * (hp[m] / (mid - q[m]));
      if (phi > 1.0) lo = mid; else hi = mid;
    }
    double n2 = 0.0;
#pragma unroll
    for (int m = 0; m < 4; m++) {
      ap[m] = hp[m] / (hi - q[m]);
      n2 += ap[m] * ap[m];
    }
    const double inv = 1.0 / sqrt(n2);
#pragma unroll
    for (int m = 0; m < 4; m++) ap[m] *= inv;
  }
#pragma unroll
  for (int r = 0; r < 4; r++) a[r] = V[r][0] * ap[0] + V[r][1] * ap[1] + V[r][2] * ap[2] + V[r][3] * ap[3];
}

// Y = g M restricted to what tr(s Y) needs for subgroup (I, J): with K the third index,
// tr(s Y) = Y_KK + a.b, b = (Y_II + Y_JJ, i(Y_JI + Y_IJ), Y_JI - Y_IJ, i(Y_II - Y_JJ)); adds
// Re(conj(Y_KK) b) to h and Re(b b^dagger) to Q.  ND: M = m^dagger.
template <typename T, int I, int J, bool ND>
__device__ __forceinline__ void subgroup_form(const M3<T> &g, const M3<T> &m, double Q[4][4], double h[4]) {
  constexpr int K = 3 - I - J;
  auto Mel = [&](int r, int c) -> cx<double> {
    const cx<T> v = ND ? conj(m.e[3 * c + r]) : m.e[3 * r + c];
    return cx<double>{(double)v.re, (double)v.im};
  };
  auto Yel = [&](int r, int c) -> cx<double> {
    cx<double> s{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const cx<T> gv = g.e[3 * r + k];
      s = s + cx<double>{(double)gv.re, (double)gv.im} * Mel(k, c);
    }
    return s;
  };
  const cx<double> yii = Yel(I, I), yjj = Yel(J, J), yij = Yel(I, J), yji = Yel(J, I), ykk = Yel(K, K);
  const cx<double> s1 = yji + yij, s3 = yii - yjj;
  const cx<double> b[4] = {yii + yjj, cx<double>{-s1.im, s1.re}, yji - yij, cx<double>{-s3.im, s3.re}};
#pragma unroll
  for (int r = 0; r < 4; r++) {
    h[r] += ykk.re * b[r].re + ykk.im * b[r].im;
#pragma unroll
    for (int c = 0; c < 4; c++) Q[r][c] += b[r].re * b[c].re + b[r].im * b[c].im;
  }
}

// One exact subgroup step on (I, J), over-relaxed: g <- s g.
template <typename T, int I, int J, bool C12>
__device__ __forceinline__ void exact_step(const M3<T> F[4], const M3<T> Bk[4], M3<T> &g, T omega) {
  double Q[4][4], h[4];
#pragma unroll
  for (int r = 0; r < 4; r++) {
    h[r] = 0.0;
#pragma unroll
    for (int c = 0; c < 4; c++) Q[r][c] = 0.0;
  }
#pragma unroll
  for (int mu = 0; mu < 4; mu++) {
    M3<T> f = F[mu];
    if constexpr (C12) third_row(f);
    subgroup_form<T, I, J, false>(g, f, Q, h);
    M3<T> bk = Bk[mu];
    if constexpr (C12) third_row(bk);
    subgroup_form<T, I, J, true>(g, bk, Q, h);
  }
  double a[4];
  sphere_max(Q, h, a);
  const double w = (double)omega;
  a[0] = (1.0 - w) + w * a[0];
  a[1] *= w;
  a[2] *= w;
  a[3] *= w;
  const double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
  if (!(na > 0.0)) return;
  const T a0 = (T)(a[0] / na), a1 = (T)(a[1] / na), a2 = (T)(a[2] / na), a3 = (T)(a[3] / na);
  const cx<T> s00{a0, a3}, s01{a2, a1}, s10{-a2, a1}, s11{a0, -a3};
#pragma unroll
  for (int c = 0; c < 3; c++) {
    const cx<T> gi = g.e[3 * I + c], gj = g.e[3 * J + c];
    g.e[3 * I + c] = s00 * gi + s01 * gj;
    g.e[3 * J + c] = s10 * gi + s11 * gj;
  }
}

// X += t * B^dagger
template <typename T> __device__ __forceinline__ void axpy_dag(cx<T> t, const M3<T> &b, M3<T> &X) {
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) X.e[3 * i + j] = X.e[3 * i + j] + t * conj(b.e[3 * j + i]);
}

// rows 0 and 1 of the g at half index h in one ring slot (row 2 zero)
template <typename T> __device__ __forceinline__ M3<T> ring_g(const V2<T> *slot, int Vh, int h) {
  M3<T> m = m_zero<T>();
  const unsigned o = (unsigned)h * (unsigned)sizeof(V2<T>);
#pragma unroll
  for (int k = 0; k < 6; k++) {
    const V2<T> v = ld_plane(slot + (size_t)k * Vh, o);
    m.e[k] = cx<T>{v.x, v.y};
  }
  return m;
}

// ----------------------------------------------------------- half-sweep
// Every site x of parity `par` gathers its eight links (forward W_mu(x),
// backward W_mu(x-mu)^dag), builds X, g, and writes g W_mu(x),
// W_mu(x-mu) g^dag and g G(x).  Sites of one parity share no link, so the
// update is race-free.  With WR, per-block sums of |tr W|^2 over the eight
// written links are stored; on the odd half-sweep these cover every link of
// the lattice once (each link joins one even and one odd site).
// C12: W and G are stored as their first two rows; only those rows stay in
// registers and row 2 is rebuilt where a product needs it.
// slab >= 0: this launch covers only that slab's chunk of every field (see LatDesc).
// MULTI: `hits` re-linearisation hits per site: after the first update each further hit
// linearises sum_k |tr(g M_k)|^2 at the current g, X_g = sum_k conj(tr(g M_k)) M_k, and runs
// the subgroup steps on g X_g, continuing g.  EXACT: each subgroup step instead maximises
// sum_k |tr(s g M_k)|^2 over its subgroup exactly (then over-relaxes), `hits` rounds of three.
// Paired sweeps (C12): the first half-sweep of a sweep leaves the links alone (KEEP) and records
// its g in slot pend of d.gring (FP32: its ring slot; FP64: a one-slot handoff, G updated in
// place as usual); the second (PEND) applies the pending g of each neighbour, read from slot pend,
// to the links it loads, exactly as the first half-sweep would have stored them, before its own
// update.  Every link then joins one site of each parity, so it
// is read twice and written once per sweep instead of read and written twice, and the result is
// that of two plain half-sweeps bit for bit: the link products in both modes are fixed FMA
// sequences with row 2 of g rebuilt from rows 0 and 1, the form the ring keeps.
// MODE: PLAIN, KEEP (first half of a paired sweep) or PEND (second half); pend names the slot.
enum { PLAIN = 0, KEEP = 1, PEND = 2 };
template <typename T, int BS, bool WR, int OCC, bool C12, bool MULTI = false, bool EXACT = false,
          int MODE = PLAIN>
__global__ __launch_bounds__(BS, OCC) void k_halfsweep(const LatDesc<T> *__restrict__ D, int B, int par,
                                                       T omega, int gated, int slab, int rev, int gslot,
                                                       int pend, int hits = 1) {
  constexpr bool keep = MODE == KEEP;
  using WS = typename FixStore<T, C12>::W;
  using GS = typename FixStore<T, C12>::G;
  int lb;
  const int b = block_of(D, B, slab, rev, lb);
  const LatDesc<T> d = D[b];
  if (gated && d.st->done) return;
  const int h = lb * BS + (int)threadIdx.x;
  double r = 0.0;
  if (h < d.g.Vh) {
    const WS W{d.W, d.g.Vh};
    const GS G{d.G, d.g.Vh};
    int c[4];
    coords_of(d.g, par, h, c);
    const unsigned of = W.off(par, h);
    unsigned ob[4];
    int hb[4];
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
      int e[4];
      moved(d.g, c, mu, -1, e);
      hb[mu] = half_index(d.g, e);
      ob[mu] = W.off(1 - par, hb[mu]);
    }
    M3<T> F[4], Bk[4];
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
      if constexpr (C12) F[mu] = W.load_rows(mu, of);
      else F[mu] = W.load_off(mu, of);
    }
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
      if constexpr (C12) Bk[mu] = W.load_rows(mu, ob[mu]);
      else Bk[mu] = W.load_off(mu, ob[mu]);
    }
    if constexpr (C12 && MODE == PEND) {
      {
        // the other parity's g of this sweep, pending on the links: W_mu(x) g'(x+mu)^dag and
        // g'(x-mu) W_mu(x-mu), rows 0 and 1 as that half-sweep would have stored them
        // all eight loads issued before the first product, so they are in flight together
        const V2<T> *ring = d.gring + (size_t)pend * 6 * d.g.Vh;
        M3<T> gf[4], gb[4];
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
          int e[4];
          moved(d.g, c, mu, +1, e);
          gf[mu] = ring_g<T>(ring, d.g.Vh, half_index(d.g, e));
        }
#pragma unroll
        for (int mu = 0; mu < 4; mu++) gb[mu] = ring_g<T>(ring, d.g.Vh, hb[mu]);
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
          third_row_fixed(gf[mu]);
          F[mu] = mul_nd_fixed_rows(F[mu], gf[mu]);
        }
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
          third_row_fixed(gb[mu]);
          M3<T> b = Bk[mu];
          third_row_fixed(b);
          Bk[mu] = mul_fixed_rows(gb[mu], b);
        }
      }
    }

    M3<T> X = m_zero<T>();
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
      M3<T> f = F[mu];
      if constexpr (C12) third_row(f);
      axpy(conj(trace(f)), f, X);
    }
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
      M3<T> bk = Bk[mu];
      if constexpr (C12) third_row(bk);
      axpy_dag(trace(bk), bk, X);
    }
    M3<T> g;
    if constexpr (EXACT) {
      g = m_ident<T>();
      for (int it = 0; it < hits; it++) {
        exact_step<T, 0, 1, C12>(F, Bk, g, omega);
        exact_step<T, 1, 2, C12>(F, Bk, g, omega);
        exact_step<T, 0, 2, C12>(F, Bk, g, omega);
      }
    } else {
      g = local_update<T>(X, omega);
    }
    if constexpr (MULTI && !EXACT) {
      for (int it = 1; it < hits; it++) {
        M3<T> Xh = m_zero<T>();
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
          M3<T> f = F[mu];
          if constexpr (C12) third_row(f);
          axpy(conj(trace(mul(g, f))), f, Xh);
        }
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
          M3<T> bk = Bk[mu];
          if constexpr (C12) third_row(bk);
          // M = bk^dag: conj(tr(g M)) M = conj(tr(g bk^dag)) bk^dag
          cx<T> t{T(0), T(0)};
#pragma unroll
          for (int k = 0; k < 9; k++) t = t + mulc(g.e[k], bk.e[k]);
          axpy_dag(conj(t), bk, Xh);
        }
        M3<T> Y = mul(g, Xh);
        subgroup_steps(Y, g, omega);
      }
    }

    if constexpr (C12) {
      // g as the ring keeps it (rows 0 and 1, row 2 rebuilt), applied in a fixed FMA order
      M3<T> gr = g;
      third_row_fixed(gr);
      if (!keep) {
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
          M3<T> f = F[mu];
          opaque_rows(f);
          third_row_fixed(f);
          const M3<T> fn = mul(gr, f);
          W.store_off(mu, of, fn);
          if (WR) r += tr2(fn);
        }
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
          M3<T> bk = Bk[mu];
          opaque_rows(bk);
          third_row_fixed(bk);
          const M3<T> bn = mul_nd(bk, gr);
          W.store_off(mu, ob[mu], bn);
          if (WR) r += tr2(bn);
        }
      }
    } else {
#pragma unroll
      for (int mu = 0; mu < 4; mu++) {
        const M3<T> fn = mul(g, F[mu]);
        W.store_off(mu, of, fn);
        if (WR) r += tr2(fn);
      }
#pragma unroll
      for (int mu = 0; mu < 4; mu++) {
        const M3<T> bn = mul_nd(Bk[mu], g);
        W.store_off(mu, ob[mu], bn);
        if (WR) r += tr2(bn);
      }
    }
    const unsigned og = (unsigned)h * (unsigned)sizeof(V2<T>);
    if (keep) {
      // the first half of a paired sweep: rows 0 and 1 of g into slot pend, which the second half
      // reads next (plain stores, so the caches keep them for it); with the FP32 ring that slot is
      // also this half-sweep's ring slot
#pragma unroll
      for (int k = 0; k < 6; k++) {
        V2<T> v;
        v.x = g.e[k].re;
        v.y = g.e[k].im;
        st_plane(d.gring + ((size_t)pend * 6 + k) * d.g.Vh, og, v);
      }
    }
    if (gslot >= 0) {
      if (!keep || gslot != pend) {
        // deferred: rows 0 and 1 of g into ring slot gslot, folded into G later (k_fold); streaming
        // stores leave the last-level cache to the links that the next half-sweep reads
#pragma unroll
        for (int k = 0; k < 6; k++) {
          V2<T> v;
          v.x = g.e[k].re;
          v.y = g.e[k].im;
          st_plane_stream(d.gring + ((size_t)gslot * 6 + k) * d.g.Vh, og, v);
        }
      }
    } else {
      M3<double> gd = m_cvt<double>(g);
      // FP32 g: row 2 rebuilt in FP64 from rows 0 and 1; the same fixed arithmetic as k_fold, so
      // that updating G here and folding the ring later give the same bits
      if constexpr (sizeof(T) == 4) third_row_fixed(gd);
      G.store(par, h, mul(gd, G.load_fixed(par, h)));
    }
  }
  if (WR) {
    const double s = wave_sum(r);
    if ((threadIdx.x & 63) == 0) d.part[lb * (BS / 64) + (threadIdx.x >> 6)] = s;
  }
}

// W = U^G (FP64 products, rounded once), with per-block sums of |tr W|^2.
template <typename T, int BS, bool C12>
__global__ __launch_bounds__(BS) void k_rederive(const LatDesc<T> *__restrict__ D, int B, int gated) {
  using WS = typename FixStore<T, C12>::W;
  using GS = typename FixStore<T, C12>::G;
  const int b = find_field(D, B);
  const LatDesc<T> d = D[b];
  if (gated && d.st->done) return;
  // the field's tiles in contiguous ranges per XCD (xcd_range: the forward neighbours' G share an
  // L2); the partial sums are stored by tile, in the same order as ever
  const int lb = xcd_range((int)blockIdx.x - d.blk0, d.nblk);
  const int h = lb * BS + (int)threadIdx.x;
  double r = 0.0;
  if (h < d.g.Vh) {
    const WS W{d.W, d.g.Vh};
    const Links<T> U{const_cast<V2<T> *>(d.U), d.g.Vh};
    const GS G{d.G, d.g.Vh};
    for (int par = 0; par < 2; par++) {
      int c[4];
      coords_of(d.g, par, h, c);
      const M3<double> Gx = G.load(par, h);
#pragma unroll
      for (int mu = 0; mu < 4; mu++) {
        int e[4];
        moved(d.g, c, mu, +1, e);
        const M3<double> Gn = G.load(1 - par, half_index(d.g, e));
        const M3<T> w = m_cvt<T>(mul_nd(mul(Gx, m_cvt<double>(U.load(mu, par, h))), Gn));
        W.store(mu, par, h, w);
        r += tr2(w);
      }
    }
  }
  const double s = wave_sum(r);
  if ((threadIdx.x & 63) == 0) d.part[lb * (BS / 64) + (threadIdx.x >> 6)] = s;
}

// G <- g_{n-1} ... g_1 g_0 G for the transforms g_j that the half-sweeps of each parity left in
// the ring (slot 2j + parity, rows 0 and 1; row 2 rebuilt in FP64), one g at a time and in the
// storage form of G after each product, so the result is that of updating G in every half-sweep.
// n = the sweeps the field ran since its last fold (its FixState), or nfix for a field without one.
// Not gated: a field that has stopped still folds the sweeps it ran.
template <typename T, int BS, bool C12>
__global__ __launch_bounds__(BS) void k_fold(const LatDesc<T> *__restrict__ D, int B, int nfix) {
  using GS = typename FixStore<T, C12>::G;
  const int b = find_field(D, B);
  const LatDesc<T> d = D[b];
  const int n = d.st ? d.st->k - d.st->kfold : nfix;
  // the field's tiles in contiguous ranges per XCD (xcd_range), as the half-sweeps take them
  const int h = xcd_range((int)blockIdx.x - d.blk0, d.nblk) * BS + (int)threadIdx.x;
  if (h >= d.g.Vh || n <= 0 || !d.gring) return;
  const GS G{d.G, d.g.Vh};
  const unsigned o = (unsigned)h * (unsigned)sizeof(V2<T>);
  for (int par = 0; par < 2; par++) {
    M3<double> m = G.load_fixed_stream(par, h);
    for (int j = 0; j < n; j++) {
      M3<double> gj;
#pragma unroll
      for (int k = 0; k < 6; k++) {
        const V2<T> v = ld_plane_stream(d.gring + ((size_t)(2 * j + par) * 6 + k) * d.g.Vh, o);
        gj.e[k] = cx<double>{(double)v.x, (double)v.y};
      }
      third_row_fixed(gj);
      m = mul(gj, m);
      if constexpr (C12) third_row_fixed(m);  // as a store and a reload of the two-row form would
    }
    G.store_stream(par, h, m);
  }
}

template <typename T, int BS, bool C12>
__global__ __launch_bounds__(BS) void k_reunit(const LatDesc<T> *__restrict__ D, int B, int gated) {
  using GS = typename FixStore<T, C12>::G;
  const int b = find_field(D, B);
  const LatDesc<T> d = D[b];
  if (gated && d.st->done) return;
  const int h = xcd_range((int)blockIdx.x - d.blk0, d.nblk) * BS + (int)threadIdx.x;  // as k_fold
  if (h >= d.g.Vh) return;
  const GS G{d.G, d.g.Vh};
  for (int par = 0; par < 2; par++) {
    M3<double> m = G.load(par, h);
    reunit(m);
    G.store(par, h, m);
  }
}

// (1/V) sum_x |TA X(x)|^2 partials (both parities; X as in the half-sweep)
template <typename T, int BS, bool C12>
__global__ __launch_bounds__(BS) void k_theta(const LatDesc<T> *__restrict__ D, int B) {
  using WS = typename FixStore<T, C12>::W;
  const int b = find_field(D, B);
  const LatDesc<T> d = D[b];
  const int h = ((int)blockIdx.x - d.blk0) * BS + (int)threadIdx.x;
  double r = 0.0;
  if (h < d.g.Vh) {
    const WS W{d.W, d.g.Vh};
    for (int par = 0; par < 2; par++) {
      int c[4];
      coords_of(d.g, par, h, c);
      M3<T> X = m_zero<T>();
#pragma unroll
      for (int mu = 0; mu < 4; mu++) {
        const M3<T> f = W.load(mu, par, h);
        axpy(conj(trace(f)), f, X);
      }
#pragma unroll
      for (int mu = 0; mu < 4; mu++) {
        int e[4];
        moved(d.g, c, mu, -1, e);
        const M3<T> bk = W.load(mu, 1 - par, half_index(d.g, e));
        axpy_dag(trace(bk), bk, X);
      }
      const M3<T> t = ta(X);
      r += (double)rdot(t, t);
    }
  }
  const double s = wave_sum(r);
  if ((threadIdx.x & 63) == 0) d.part[((int)blockIdx.x - d.blk0) * (BS / 64) + (threadIdx.x >> 6)] = s;
}

// Conversion between the full and the two-row forms (to12: full -> rows;
// otherwise rows -> full with row 2 rebuilt).  Links: one thread per (h, mu,
// parity); gauge: one thread per (h, parity).
template <typename T>
__global__ __launch_bounds__(256) void k_links_form(Geom g, const V2<T> *__restrict__ src, V2<T> *__restrict__ dst,
                                                    int to12) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  if (h >= g.Vh) return;
  const int mu = blockIdx.y >> 1, par = blockIdx.y & 1;
  const Links<T> F{to12 ? const_cast<V2<T> *>(src) : dst, g.Vh};
  const Links12<T> C{to12 ? dst : const_cast<V2<T> *>(src), g.Vh};
  if (to12)
    C.store(mu, par, h, F.load(mu, par, h));
  else
    F.store(mu, par, h, C.load(mu, par, h));
}

__global__ __launch_bounds__(256) void k_gauge_form(Geom g, const double2 *__restrict__ src,
                                                    double2 *__restrict__ dst, int to12) {
  const int h = blockIdx.x * 256 + threadIdx.x;
  if (h >= g.Vh) return;
  const int par = blockIdx.y;
  const Gauge F{to12 ? const_cast<double2 *>(src) : dst, g.Vh};
  const Gauge12 C{to12 ? dst : const_cast<double2 *>(src), g.Vh};
  if (to12)
    C.store(par, h, F.load(par, h));
  else
    F.store(par, h, C.load(par, h));
}

// ------------------------------------------------------ bookkeeping
// One block per field (grid = B).  R is normalised as (1/(9 N_l)) sum |tr|^2, summed
// over the per-wavefront partials in index order (independent of the block size).
enum { BK_INIT = 0, BK_RESET = 1, BK_CHECK = 2, BK_FINAL = 3, BK_THETA = 4, BK_FOLD = 5 };

// 1024 threads with 16 loads in flight each: the 16384 wave partials of a 32^3x64 half-lattice
// arrive in one round trip (the sum is latency-bound, once per sweep; 256 threads took two).
template <typename T>
__global__ __launch_bounds__(1024) void k_book(const LatDesc<T> *__restrict__ D, int what) {
  const LatDesc<T> d = D[blockIdx.x];
  FixState *st = d.st;
  if (what == BK_FOLD) {  // after k_fold: every sweep run so far is in G
    if (threadIdx.x == 0) st->kfold = st->k;
    return;
  }
  // the state is read once, alongside the partial sums (the two loads do not wait for each
  // other); a finished field's block leaves after the sum, together (the exit is block-uniform)
  const FixState sv = *st;
  const double s = sum_partials<1024, 16>(d.part, d.npart);
  if ((what == BK_RESET || what == BK_CHECK) && sv.done) return;
  if (threadIdx.x != 0) return;
  const double R = s / (9.0 * (double)(4 * d.g.V));
  switch (what) {
  case BK_INIT:
    st->R_prev = R;
    st->R_last = R;
    st->dR = 0.0;
    st->k = 0;
    st->kfold = 0;
    st->done = sv.max_k <= 0 ? 1 : 0;
    st->status = 1;
    if (d.traj) d.traj[0] = R;
    break;
  case BK_RESET:
    st->R_prev = R;
    break;
  case BK_CHECK: {
    const double dR = R - sv.R_prev;
    const int k = sv.k + 1;
    st->k = k;
    st->dR = dR;
    st->R_last = R;
    if (d.traj) d.traj[k] = R;
    if (dR < sv.tol && (sv.start_sweep + k) % sv.stop_every == 0) {
      st->done = 1;
      st->status = 0;
    } else if (k >= sv.max_k) {
      st->done = 1;
      st->status = 1;
    } else {
      st->R_prev = R;
    }
    break;
  }
  case BK_FINAL:
    st->R_final = R;
    break;
  default:  // BK_THETA
    st->theta = s / (double)d.g.V;
    break;
  }
}

}  // namespace mcg
