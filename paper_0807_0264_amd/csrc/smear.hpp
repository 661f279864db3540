// smear.hpp -- device pieces of stout and over-improved stout smearing
// (Sec. II.B of arXiv:0807.0264; parameters of Sec. III): the staple sum of
// one link and exp of a traceless anti-Hermitian 3x3 matrix through the
// Cayley-Hamilton relation Q^3 = c1 Q + c0 (Q = -iA Hermitian traceless,
// c1 = tr(Q^2)/2, c0 = det Q).
#pragma once

#include "common.hpp"

namespace mcg {

// Powers of Q reduce to Q^n = a_n + b_n Q + d_n Q^2 with the real recursion
// a_{n+1} = c0 d_n, b_{n+1} = a_n + c1 d_n, d_{n+1} = b_n (from Q^3 = c1 Q + c0),
// so exp(iQ) = f0 + f1 Q + f2 Q^2 with f_j = sum_n (i^n / n!) {a,b,d}_n.
// The derivatives of the f_j with respect to c0 and c1 follow from the same
// recursion differentiated term by term (used by the adjoint).
template <typename T> struct CHCoef {
  cx<T> f[3];
  cx<T> df0[3];  // d f_j / d c0
  cx<T> df1[3];  // d f_j / d c1
};

template <typename T, int N, bool DERIV>
__device__ __forceinline__ void ch_series(T c0, T c1, CHCoef<T> &o) {
  T a = T(1), b = T(0), d = T(0);
  T a0 = T(0), b0 = T(0), d0 = T(0);  // d/dc0 of a, b, d
  T a1 = T(0), b1 = T(0), d1 = T(0);  // d/dc1 of a, b, d
  T wre = T(1), wim = T(0);
  o.f[0] = cx<T>{T(1), T(0)};
  o.f[1] = o.f[2] = cx<T>{T(0), T(0)};
  if (DERIV) {
#pragma unroll
    for (int j = 0; j < 3; j++) o.df0[j] = o.df1[j] = cx<T>{T(0), T(0)};
  }
#pragma unroll
  for (int n = 1; n <= N; n++) {
    const T an = c0 * d, bn = a + c1 * d, dn = b;
    if (DERIV) {
      const T a0n = c0 * d0 + d, b0n = a0 + c1 * d0, d0n = b0;
      const T a1n = c0 * d1, b1n = a1 + c1 * d1 + d, d1n = b1;
      a0 = a0n; b0 = b0n; d0 = d0n;
      a1 = a1n; b1 = b1n; d1 = d1n;
    }
    a = an;
    b = bn;
    d = dn;
    const T inv = T(1) / T(n);
    const T nre = -wim * inv, nim = wre * inv;  // w <- w * i / n
    wre = nre;
    wim = nim;
    o.f[0] = o.f[0] + cx<T>{wre * a, wim * a};
    o.f[1] = o.f[1] + cx<T>{wre * b, wim * b};
    o.f[2] = o.f[2] + cx<T>{wre * d, wim * d};
    if (DERIV) {
      o.df0[0] = o.df0[0] + cx<T>{wre * a0, wim * a0};
      o.df0[1] = o.df0[1] + cx<T>{wre * b0, wim * b0};
      o.df0[2] = o.df0[2] + cx<T>{wre * d0, wim * d0};
      o.df1[0] = o.df1[0] + cx<T>{wre * a1, wim * a1};
      o.df1[1] = o.df1[1] + cx<T>{wre * b1, wim * b1};
      o.df1[2] = o.df1[2] + cx<T>{wre * d1, wim * d1};
    }
  }
}

// Q = -iA for anti-Hermitian A
template <typename T> __device__ __forceinline__ M3<T> minus_i(const M3<T> &A) {
  M3<T> Q;
#pragma unroll
  for (int k = 0; k < 9; k++) Q.e[k] = cx<T>{A.e[k].im, -A.e[k].re};
  return Q;
}

// c1 = tr(Q^2)/2 and c0 = det Q = tr(Q^3)/3 for traceless Hermitian Q
template <typename T>
__device__ __forceinline__ void ch_invariants(const M3<T> &Q, const M3<T> &Q2, T &c0, T &c1) {
  c1 = T(0.5) * (Q2.e[0].re + Q2.e[4].re + Q2.e[8].re);
  T t3 = T(0);
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) t3 += (Q.e[3 * i + j] * Q2.e[3 * j + i]).re;
  c0 = t3 * T(1.0 / 3.0);
}

template <typename T> struct ExpTerms;
template <> struct ExpTerms<float> { static constexpr int N = 14; };
template <> struct ExpTerms<double> { static constexpr int N = 22; };

// exp(A) for A in su(3).  Q is scaled by 2^-s until the bound sqrt(4 c1/3)
// on its spectral radius is at most 1; the series is summed for the scaled
// matrix and the result squared s times.
template <typename T> __device__ __forceinline__ M3<T> exp_su3(const M3<T> &A) {
  const M3<T> Q = minus_i(A);
  const M3<T> Q2 = mul(Q, Q);
  T c0, c1;
  ch_invariants(Q, Q2, c0, c1);
  int s = 0;
  T r2 = T(4.0 / 3.0) * c1;
  T sc = T(1);
  while (r2 > T(1) && s < 40) {
    r2 *= T(0.25);
    sc *= T(0.5);
    s++;
  }
  const T sc2 = sc * sc;
  CHCoef<T> co;
  ch_series<T, ExpTerms<T>::N, false>(c0 * sc2 * sc, c1 * sc2, co);
  const cx<T> g1 = sc * co.f[1], g2 = sc2 * co.f[2];
  M3<T> E;
#pragma unroll
  for (int k = 0; k < 9; k++) E.e[k] = g1 * Q.e[k] + g2 * Q2.e[k];
  E.e[0] = E.e[0] + co.f[0];
  E.e[4] = E.e[4] + co.f[0];
  E.e[8] = E.e[8] + co.f[0];
  for (int q = 0; q < s; q++) E = mul(E, E);
  return E;
}

// Make the compiler treat coordinates as freshly produced (see staples).
__device__ __forceinline__ void opaque_coords(int c[4]) {
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
  for (int q = 0; q < 4; q++) __asm__ volatile("" : "+v"(c[q]));
#else
  (void)c;
#endif
}

// Make the compiler treat a loaded matrix as produced here: every load into it is complete at this
// point (see staples).
template <typename T> __device__ __forceinline__ void opaque_m3(M3<T> &m) {
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
  for (int k = 0; k < 9; k++) __asm__ volatile("" : "+v"(m.e[k].re), "+v"(m.e[k].im));
#else
  (void)m;
#endif
}

// Plaquette part Cp and rectangle part Cr (OI only) of the staple sum of
// link (c, mu): paths from x to x+mu.  Per nu != mu and per sign of nu: the
// plaquette staple and the rectangles 2x1 ahead, 2x1 behind (long in mu) and
// 1x2 (long in nu).  Rectangles that end on the same link share the last
// product: the 2x1-behind and 1x2 paths of one nu and sign both end on the
// link into x+mu along nu, and every 2x1-ahead path ends on U_mu(x+mu)^dag, so
// their prefixes are summed first and multiplied by that link once.
template <typename T, bool OI>
__device__ __forceinline__ void staples(const Geom &g, const Links<T> &L, const int c[4], int mu,
                                        M3<T> &Cp, M3<T> &Cr) {
  Cp = m_zero<T>();
  Cr = m_zero<T>();
  M3<T> ahead = m_zero<T>();  // OI: sum of the 2x1-ahead prefixes, closed by U_mu(x+mu)^dag at the end
  int cpm[4], cmm[4];
  moved(g, c, mu, +1, cpm);
  moved(g, c, mu, -1, cmm);
  const M3<T> umu_xmm = OI ? L.at(g, cmm, mu) : m_zero<T>();  // U_mu(x-mu)
  if constexpr (!OI) {
    // Stout: the six links of a direction are loaded together and (FP32) held until all six are in,
    // so a wave has six loads in flight instead of three; 142 VGPRs and three waves per SIMD
    // instead of 94 and five, 1.7 % less time.  The sums are taken in the same order.
    for (int nu = 0; nu < 4; nu++) {
      if (nu == mu) continue;
      int b[4] = {c[0], c[1], c[2], c[3]}, bpm[4] = {cpm[0], cpm[1], cpm[2], cpm[3]};
      opaque_coords(b);
      opaque_coords(bpm);
      int cpn[4], cmn[4], cmnpm[4];
      moved(g, b, nu, +1, cpn);
      moved(g, b, nu, -1, cmn);
      moved(g, cmn, mu, +1, cmnpm);
      M3<T> unu_x = L.at(g, b, nu), umu_xpn = L.at(g, cpn, mu), unu_xpm = L.at(g, bpm, nu);  // +nu side
      M3<T> unu_xmn = L.at(g, cmn, nu), umu_xmn = L.at(g, cmn, mu), unu_xmnpm = L.at(g, cmnpm, nu);  // -nu
      if constexpr (sizeof(T) == 4) {
        opaque_m3(unu_x);
        opaque_m3(umu_xpn);
        opaque_m3(unu_xpm);
        opaque_m3(unu_xmn);
        opaque_m3(umu_xmn);
        opaque_m3(unu_xmnpm);
      }
      mac_nd(mul(unu_x, umu_xpn), unu_xpm, Cp);       // U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
      mac(mul_dn(unu_xmn, umu_xmn), unu_xmnpm, Cp);  // U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)
    }
    return;
  }
  for (int nu = 0; nu < 4; nu++) {
    if (nu == mu) continue;
    // Each side of the direction starts from opaque copies of the base coordinates, so the
    // compiler forms its addresses and loads where they are used rather than all at once (a
    // register-pressure hint with no run-time cost); the sums are taken in the same order.
    {  // +nu
      int b[4] = {c[0], c[1], c[2], c[3]}, bpm[4] = {cpm[0], cpm[1], cpm[2], cpm[3]},
          bmm[4] = {cmm[0], cmm[1], cmm[2], cmm[3]};
      opaque_coords(b);
      opaque_coords(bpm);
      opaque_coords(bmm);
      int cpn[4];
      moved(g, b, nu, +1, cpn);
      const M3<T> unu_x = L.at(g, b, nu);       // U_nu(x)
      const M3<T> umu_xpn = L.at(g, cpn, mu);   // U_mu(x+nu)
      const M3<T> unu_xpm = L.at(g, bpm, nu);   // U_nu(x+mu)
      const M3<T> up = mul(unu_x, umu_xpn);     // U_nu(x) U_mu(x+nu)
      mac_nd(up, unu_xpm, Cp);
      if (OI) {
        int cpnpm[4], cp2m[4], cmmpn[4], cp2n[4];
        moved(g, cpn, mu, +1, cpnpm);
        moved(g, bpm, mu, +1, cp2m);
        moved(g, bmm, nu, +1, cmmpn);
        moved(g, cpn, nu, +1, cp2n);
        M3<T> t, end;
        // 2x1 ahead: U_nu(x) U_mu(x+nu) U_mu(x+nu+mu) U_nu(x+2mu)^dag [U_mu(x+mu)^dag]
        t = mul(up, L.at(g, cpnpm, mu));
        mac_nd(t, L.at(g, cp2m, nu), ahead);
        // 2x1 behind: U_mu(x-mu)^dag U_nu(x-mu) U_mu(x-mu+nu) U_mu(x+nu) [U_nu(x+mu)^dag]
        t = mul_dn(umu_xmm, L.at(g, bmm, nu));
        t = mul(t, L.at(g, cmmpn, mu));
        end = mul(t, umu_xpn);
        // 1x2: U_nu(x) U_nu(x+nu) U_mu(x+2nu) U_nu(x+mu+nu)^dag [U_nu(x+mu)^dag]
        t = mul(unu_x, L.at(g, cpn, nu));
        t = mul(t, L.at(g, cp2n, mu));
        mac_nd(t, L.at(g, cpnpm, nu), end);
        mac_nd(end, unu_xpm, Cr);
      }
    }
    {  // -nu
      int b[4] = {c[0], c[1], c[2], c[3]}, bmm[4] = {cmm[0], cmm[1], cmm[2], cmm[3]};
      opaque_coords(b);
      opaque_coords(bmm);
      int cmn[4], cmnpm[4];
      moved(g, b, nu, -1, cmn);
      moved(g, cmn, mu, +1, cmnpm);
      const M3<T> unu_xmn = L.at(g, cmn, nu);      // U_nu(x-nu)
      const M3<T> umu_xmn = L.at(g, cmn, mu);      // U_mu(x-nu)
      const M3<T> unu_xmnpm = L.at(g, cmnpm, nu);  // U_nu(x-nu+mu)
      const M3<T> dn = mul_dn(unu_xmn, umu_xmn);   // U_nu(x-nu)^dag U_mu(x-nu)
      mac(dn, unu_xmnpm, Cp);
      if (OI) {
        int cmnp2m[4], cmmmn[4], cm2n[4], cm2npm[4];
        moved(g, cmnpm, mu, +1, cmnp2m);
        moved(g, bmm, nu, -1, cmmmn);
        moved(g, cmn, nu, -1, cm2n);
        moved(g, cm2n, mu, +1, cm2npm);
        M3<T> t, end;
        // 2x1 ahead: U_nu(x-nu)^dag U_mu(x-nu) U_mu(x-nu+mu) U_nu(x-nu+2mu) [U_mu(x+mu)^dag]
        t = mul(dn, L.at(g, cmnpm, mu));
        mac(t, L.at(g, cmnp2m, nu), ahead);
        // 2x1 behind: U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_mu(x-nu) [U_nu(x-nu+mu)]
        t = dag(mul(L.at(g, cmmmn, nu), umu_xmm));
        t = mul(t, L.at(g, cmmmn, mu));
        end = mul(t, umu_xmn);
        // 1x2: U_nu(x-nu)^dag U_nu(x-2nu)^dag U_mu(x-2nu) U_nu(x-2nu+mu) [U_nu(x-nu+mu)]
        t = dag(mul(L.at(g, cm2n, nu), unu_xmn));
        t = mul(t, L.at(g, cm2n, mu));
        mac(t, L.at(g, cm2npm, nu), end);
        mac(end, unu_xmnpm, Cr);
      }
    }
  }
  if (OI) mac_nd(ahead, L.at(g, cpm, mu), Cr);  // ... U_mu(x+mu)^dag
}

}  // namespace mcg
