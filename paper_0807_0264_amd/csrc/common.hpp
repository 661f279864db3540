// common.hpp -- device-side building blocks of the gfx950 MCG library:
// complex and 3x3 complex matrix arithmetic, lattice geometry of the
// even/odd structure-of-arrays layout, link I/O and deterministic block
// reductions.  Everything is templated on the link precision T (float or
// double); gauge transforms are always double.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcg {

template <typename T> struct V2t;
template <> struct V2t<float> { using type = float2; };
template <> struct V2t<double> { using type = double2; };
template <typename T> using V2 = typename V2t<T>::type;

// ---------------------------------------------------------------- complex
template <typename T> struct cx {
  T re, im;
};

template <typename T> __device__ __forceinline__ cx<T> cmk(T r, T i) { return cx<T>{r, i}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return cx<T>{a.re + b.re, a.im + b.im};
}
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return cx<T>{a.re - b.re, a.im - b.im};
}
template <typename T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) {
  return cx<T>{s * a.re, s * a.im};
}
template <typename T> __device__ __forceinline__ cx<T> conj(cx<T> a) { return cx<T>{a.re, -a.im}; }
// a * conj(b)
template <typename T> __device__ __forceinline__ cx<T> mulc(cx<T> a, cx<T> b) {
  return cx<T>{a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// conj(a) * b
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return cx<T>{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T> __device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }

template <typename To, typename From> __device__ __forceinline__ cx<To> cvt(cx<From> a) {
  return cx<To>{(To)a.re, (To)a.im};
}

// ------------------------------------------------------------ 3x3 matrices
template <typename T> struct M3 {
  cx<T> e[9];
};

template <typename T> __device__ __forceinline__ M3<T> m_zero() {
  M3<T> r;
#pragma unroll
  for (int k = 0; k < 9; k++) r.e[k] = cx<T>{T(0), T(0)};
  return r;
}
template <typename T> __device__ __forceinline__ M3<T> m_ident() {
  M3<T> r = m_zero<T>();
  r.e[0].re = r.e[4].re = r.e[8].re = T(1);
  return r;
}
template <typename To, typename From> __device__ __forceinline__ M3<To> m_cvt(const M3<From> &a) {
  M3<To> r;
#pragma unroll
  for (int k = 0; k < 9; k++) r.e[k] = cvt<To>(a.e[k]);
  return r;
}
// ----------------------------------------------- products in a fixed FMA order
// Every 3x3 product is written as explicit fused multiply-adds in a fixed order: left to the
// compiler, a complex product term becomes a multiply and an FMA and the three terms two more
// adds (16 instructions per element instead of 12), and the contraction it picks can differ from
// one kernel to the next in the last bit.  Written out, the same product gives the same bits
// wherever it is inlined.
template <typename T> __device__ __forceinline__ T fma_t(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return fmaf(a, b, c);
  else return fma(a, b, c);
}
// a0 b0 + a1 b1 + a2 b2
template <typename T>
__device__ __forceinline__ cx<T> dot3_fma(cx<T> a0, cx<T> b0, cx<T> a1, cx<T> b1, cx<T> a2, cx<T> b2) {
  T re = a0.re * b0.re, im = a0.re * b0.im;
  re = fma_t(-a0.im, b0.im, re);
  im = fma_t(a0.im, b0.re, im);
  re = fma_t(a1.re, b1.re, re);
  re = fma_t(-a1.im, b1.im, re);
  im = fma_t(a1.re, b1.im, im);
  im = fma_t(a1.im, b1.re, im);
  re = fma_t(a2.re, b2.re, re);
  re = fma_t(-a2.im, b2.im, re);
  im = fma_t(a2.re, b2.im, im);
  im = fma_t(a2.im, b2.re, im);
  return cx<T>{re, im};
}
// a0 conj(b0) + a1 conj(b1) + a2 conj(b2)
template <typename T>
__device__ __forceinline__ cx<T> dot3c_fma(cx<T> a0, cx<T> b0, cx<T> a1, cx<T> b1, cx<T> a2, cx<T> b2) {
  T re = a0.re * b0.re, im = -(a0.re * b0.im);
  re = fma_t(a0.im, b0.im, re);
  im = fma_t(a0.im, b0.re, im);
  re = fma_t(a1.re, b1.re, re);
  re = fma_t(a1.im, b1.im, re);
  im = fma_t(-a1.re, b1.im, im);
  im = fma_t(a1.im, b1.re, im);
  re = fma_t(a2.re, b2.re, re);
  re = fma_t(a2.im, b2.im, re);
  im = fma_t(-a2.re, b2.im, im);
  im = fma_t(a2.im, b2.re, im);
  return cx<T>{re, im};
}
// conj(a0) b0 + conj(a1) b1 + conj(a2) b2
template <typename T>
__device__ __forceinline__ cx<T> dot3n_fma(cx<T> a0, cx<T> b0, cx<T> a1, cx<T> b1, cx<T> a2, cx<T> b2) {
  T re = a0.re * b0.re, im = a0.re * b0.im;
  re = fma_t(a0.im, b0.im, re);
  im = fma_t(-a0.im, b0.re, im);
  re = fma_t(a1.re, b1.re, re);
  re = fma_t(a1.im, b1.im, re);
  im = fma_t(a1.re, b1.im, im);
  im = fma_t(-a1.im, b1.re, im);
  re = fma_t(a2.re, b2.re, re);
  re = fma_t(a2.im, b2.im, re);
  im = fma_t(a2.re, b2.im, im);
  im = fma_t(-a2.im, b2.re, im);
  return cx<T>{re, im};
}
// a b
template <typename T> __device__ __forceinline__ M3<T> mul(const M3<T> &a, const M3<T> &b) {
  M3<T> c;
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int q = 0; q < 3; q++)
      c.e[3 * r + q] = dot3_fma(a.e[3 * r], b.e[q], a.e[3 * r + 1], b.e[3 + q], a.e[3 * r + 2], b.e[6 + q]);
  return c;
}
// a b^dagger
template <typename T> __device__ __forceinline__ M3<T> mul_nd(const M3<T> &a, const M3<T> &b) {
  M3<T> c;
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int q = 0; q < 3; q++)
      c.e[3 * r + q] = dot3c_fma(a.e[3 * r], b.e[3 * q], a.e[3 * r + 1], b.e[3 * q + 1], a.e[3 * r + 2], b.e[3 * q + 2]);
  return c;
}
// a^dagger b
template <typename T> __device__ __forceinline__ M3<T> mul_dn(const M3<T> &a, const M3<T> &b) {
  M3<T> c;
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int q = 0; q < 3; q++)
      c.e[3 * r + q] = dot3n_fma(a.e[r], b.e[q], a.e[3 + r], b.e[3 + q], a.e[6 + r], b.e[6 + q]);
  return c;
}
// c += a b and c += a b^dagger, each element's FMA chain starting from c
template <typename T>
__device__ __forceinline__ cx<T> dot3_acc(cx<T> c, cx<T> a0, cx<T> b0, cx<T> a1, cx<T> b1, cx<T> a2, cx<T> b2) {
  T re = fma_t(a0.re, b0.re, c.re), im = fma_t(a0.re, b0.im, c.im);
  re = fma_t(-a0.im, b0.im, re);
  im = fma_t(a0.im, b0.re, im);
  re = fma_t(a1.re, b1.re, re);
  re = fma_t(-a1.im, b1.im, re);
  im = fma_t(a1.re, b1.im, im);
  im = fma_t(a1.im, b1.re, im);
  re = fma_t(a2.re, b2.re, re);
  re = fma_t(-a2.im, b2.im, re);
  im = fma_t(a2.re, b2.im, im);
  im = fma_t(a2.im, b2.re, im);
  return cx<T>{re, im};
}
template <typename T>
__device__ __forceinline__ cx<T> dot3c_acc(cx<T> c, cx<T> a0, cx<T> b0, cx<T> a1, cx<T> b1, cx<T> a2, cx<T> b2) {
  T re = fma_t(a0.re, b0.re, c.re), im = fma_t(-a0.re, b0.im, c.im);
  re = fma_t(a0.im, b0.im, re);
  im = fma_t(a0.im, b0.re, im);
  re = fma_t(a1.re, b1.re, re);
  re = fma_t(a1.im, b1.im, re);
  im = fma_t(-a1.re, b1.im, im);
  im = fma_t(a1.im, b1.re, im);
  re = fma_t(a2.re, b2.re, re);
  re = fma_t(a2.im, b2.im, re);
  im = fma_t(-a2.re, b2.im, im);
  im = fma_t(a2.im, b2.re, im);
  return cx<T>{re, im};
}
template <typename T> __device__ __forceinline__ void mac(const M3<T> &a, const M3<T> &b, M3<T> &c) {
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int q = 0; q < 3; q++)
      c.e[3 * r + q] =
          dot3_acc(c.e[3 * r + q], a.e[3 * r], b.e[q], a.e[3 * r + 1], b.e[3 + q], a.e[3 * r + 2], b.e[6 + q]);
}
template <typename T> __device__ __forceinline__ void mac_nd(const M3<T> &a, const M3<T> &b, M3<T> &c) {
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int q = 0; q < 3; q++)
      c.e[3 * r + q] = dot3c_acc(c.e[3 * r + q], a.e[3 * r], b.e[3 * q], a.e[3 * r + 1], b.e[3 * q + 1],
                                 a.e[3 * r + 2], b.e[3 * q + 2]);
}
template <typename T> __device__ __forceinline__ M3<T> dag(const M3<T> &a) {
  M3<T> c;
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) c.e[3 * i + j] = conj(a.e[3 * j + i]);
  return c;
}
template <typename T> __device__ __forceinline__ cx<T> trace(const M3<T> &a) {
  return a.e[0] + a.e[4] + a.e[8];
}
// c += s a (complex s)
template <typename T> __device__ __forceinline__ void axpy(cx<T> s, const M3<T> &a, M3<T> &c) {
#pragma unroll
  for (int k = 0; k < 9; k++) c.e[k] = c.e[k] + s * a.e[k];
}
template <typename T> __device__ __forceinline__ void add_to(const M3<T> &a, M3<T> &c) {
#pragma unroll
  for (int k = 0; k < 9; k++) c.e[k] = c.e[k] + a.e[k];
}
template <typename T> __device__ __forceinline__ M3<T> scale(T s, const M3<T> &a) {
  M3<T> c;
#pragma unroll
  for (int k = 0; k < 9; k++) c.e[k] = s * a.e[k];
  return c;
}
// traceless anti-Hermitian part: (1/2)(M - M^dag) - (1/6) tr(M - M^dag) 1
template <typename T> __device__ __forceinline__ M3<T> ta(const M3<T> &m) {
  M3<T> o;
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) {
      cx<T> a = m.e[3 * i + j], b = m.e[3 * j + i];
      o.e[3 * i + j] = cx<T>{T(0.5) * (a.re - b.re), T(0.5) * (a.im + b.im)};
    }
  // tr(M - M^dag) = 2i Im tr M
  T im3 = (m.e[0].im + m.e[4].im + m.e[8].im) * T(1.0 / 3.0);
  o.e[0].im -= im3;
  o.e[4].im -= im3;
  o.e[8].im -= im3;
  return o;
}
// Re tr(a^dagger b)
template <typename T> __device__ __forceinline__ T rdot(const M3<T> &a, const M3<T> &b) {
  T s = T(0);
#pragma unroll
  for (int k = 0; k < 9; k++) s += a.e[k].re * b.e[k].re + a.e[k].im * b.e[k].im;
  return s;
}
// |tr M|^2 evaluated in double from the stored precision
template <typename T> __device__ __forceinline__ double tr2(const M3<T> &a) {
  cx<T> t = trace(a);
  double r = (double)t.re, i = (double)t.im;
  return r * r + i * i;
}

// Gram-Schmidt on the rows; third row = conj(r0 x r1), so det = +1.
__device__ __forceinline__ void reunit(M3<double> &m) {
  double n0 = norm2(m.e[0]) + norm2(m.e[1]) + norm2(m.e[2]);
  double i0 = 1.0 / sqrt(n0);
#pragma unroll
  for (int k = 0; k < 3; k++) m.e[k] = i0 * m.e[k];
  cx<double> ip = cmul(m.e[0], m.e[3]) + cmul(m.e[1], m.e[4]) + cmul(m.e[2], m.e[5]);
#pragma unroll
  for (int k = 0; k < 3; k++) m.e[3 + k] = m.e[3 + k] - ip * m.e[k];
  double n1 = norm2(m.e[3]) + norm2(m.e[4]) + norm2(m.e[5]);
  double i1 = 1.0 / sqrt(n1);
#pragma unroll
  for (int k = 3; k < 6; k++) m.e[k] = i1 * m.e[k];
  m.e[6] = conj(m.e[1] * m.e[5] - m.e[2] * m.e[4]);
  m.e[7] = conj(m.e[2] * m.e[3] - m.e[0] * m.e[5]);
  m.e[8] = conj(m.e[0] * m.e[4] - m.e[1] * m.e[3]);
}

// ---------------------------------------------------------------- geometry
// Sites are split by parity; within a parity, the half index is h = i >> 1
// with i = x + Lx*(y + Ly*(z + Lz*t)) (Lx is even, so i and i^1 have opposite
// parity and the same h).
struct Geom {
  int L[4];
  int V, Vh, hx;  // sites, sites per parity, Lx / 2
};

__device__ __forceinline__ void coords_of(const Geom &g, int par, int h, int c[4]) {
  int r = h / g.hx;
  int xh = h - r * g.hx;
  int r2 = r / g.L[1];
  int y = r - r2 * g.L[1];
  int t = r2 / g.L[2];
  int z = r2 - t * g.L[2];
  c[0] = 2 * xh + ((par + y + z + t) & 1);
  c[1] = y;
  c[2] = z;
  c[3] = t;
}
// Workgroups are dealt to the eight XCDs in turn (block i to XCD i mod 8).  xcd_range maps block i
// of a range of n tiles so that the blocks of one XCD (equal i mod 8) take a contiguous range of
// tiles, the j-th block of the class (i = class + 8j) the j-th tile of that range, instead of every
// eighth tile: the tiles a site's neighbours lie in, a few tiles away, then mostly belong to the
// same XCD and meet in its L2.  A bijection of [0, n) for every n.
__device__ __forceinline__ int xcd_range(int i, int n) {
  const int x = i & 7, q = n >> 3, r = n & 7;
  return x * q + (x < r ? x : r) + (i >> 3);
}
// Tiles of the gather kernels (smearing and its adjoint): a tile is 128 half-sites of one t-slice
// (S = Vh / Lt half-sites per slice, ceil(S / 128) tiles each).  Tiles come in groups of up to
// eight consecutive t-slices, and inside a group the slice index runs fastest, so the tiles that
// hold a site's t-neighbours are a few tiles away, not a whole slice (at 32^3x64 a slice of links
// is larger than an XCD's L2).  gather_site maps (tile, lane) to the half-site index, or -1 for the
// idle lanes of a slice's last tile; a bijection of [0, gather_tiles) x [0, 128) onto the
// half-sites and the idle lanes.
__host__ __device__ inline int gather_tiles(const Geom &g) { return g.L[3] * ((g.Vh / g.L[3] + 127) / 128); }
__device__ __forceinline__ int gather_site(const Geom &g, int tile, int lane) {
  const int S = g.Vh / g.L[3], span = 8 * ((S + 127) / 128);
  const int gi = tile / span, rem = tile - gi * span;
  const int bt = g.L[3] - 8 * gi < 8 ? g.L[3] - 8 * gi : 8;
  const int ch = rem / bt, t = 8 * gi + (rem - ch * bt);
  const int s = ch * 128 + lane;
  return s < S ? t * S + s : -1;
}
__device__ __forceinline__ int lex_index(const Geom &g, const int c[4]) {
  return c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}
__device__ __forceinline__ int half_index(const Geom &g, const int c[4]) {
  return lex_index(g, c) >> 1;
}
__device__ __forceinline__ int parity_of(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }
// coordinates moved by `step` (|step| < L) along mu, periodic
__device__ __forceinline__ void moved(const Geom &g, const int c[4], int mu, int step, int d[4]) {
#pragma unroll
  for (int k = 0; k < 4; k++) d[k] = c[k];
  int v = c[mu] + step;
  int Lm = g.L[mu];
  v = v >= Lm ? v - Lm : v;
  v = v < 0 ? v + Lm : v;
  d[mu] = v;
}

// ------------------------------------------------------------------ I/O
// Loads and stores address a plane through a wave-uniform base pointer plus a
// 32-bit per-lane byte offset, so the compiler can use the scalar-base form
// of global memory instructions and keeps no 64-bit per-lane addresses live.
template <typename V>
__device__ __forceinline__ V ld_plane(const V *plane, unsigned byte_off) {
  return *(const V *)((const char *)plane + byte_off);
}
template <typename V>
__device__ __forceinline__ void st_plane(V *plane, unsigned byte_off, V v) {
  *(V *)((char *)plane + byte_off) = v;
}
// Streaming loads and stores (non-temporal hint) for data touched once: the
// transform ring, written by a half-sweep and read back by the fold many
// sweeps later, so it does not displace the links in the last-level cache.
// The host build of these sources (the emulation) uses plain accesses.
#if defined(__HIP_DEVICE_COMPILE__)
typedef float mcg_f2v __attribute__((ext_vector_type(2)));
typedef double mcg_d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_plane_stream(const float2 *plane, unsigned byte_off) {
  const mcg_f2v w = __builtin_nontemporal_load((const mcg_f2v *)((const char *)plane + byte_off));
  return make_float2(w.x, w.y);
}
__device__ __forceinline__ double2 ld_plane_stream(const double2 *plane, unsigned byte_off) {
  const mcg_d2v w = __builtin_nontemporal_load((const mcg_d2v *)((const char *)plane + byte_off));
  return make_double2(w.x, w.y);
}
__device__ __forceinline__ void st_plane_stream(float2 *plane, unsigned byte_off, float2 v) {
  mcg_f2v w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, (mcg_f2v *)((char *)plane + byte_off));
}
__device__ __forceinline__ void st_plane_stream(double2 *plane, unsigned byte_off, double2 v) {
  mcg_d2v w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, (mcg_d2v *)((char *)plane + byte_off));
}
#else
template <typename V> __device__ __forceinline__ V ld_plane_stream(const V *plane, unsigned byte_off) {
  return ld_plane(plane, byte_off);
}
template <typename V> __device__ __forceinline__ void st_plane_stream(V *plane, unsigned byte_off, V v) {
  st_plane(plane, byte_off, v);
}
#endif

// complex element (mu, par, k, h) at ((mu*2 + par)*9 + k)*Vh + h
//   = (mu*18 + k)*Vh  [uniform]  +  par*9*Vh + h  [per lane]
template <typename T> struct Links {
  V2<T> *p;
  int Vh;
  __device__ __forceinline__ unsigned off(int par, int h) const {
    return (unsigned)(par * 9 * Vh + h) * (unsigned)sizeof(V2<T>);
  }
  __device__ __forceinline__ M3<T> load_off(int mu, unsigned o) const {
    M3<T> m;
#pragma unroll
    for (int k = 0; k < 9; k++) {
      const V2<T> v = ld_plane(p + (size_t)(mu * 18 + k) * Vh, o);
      m.e[k] = cx<T>{v.x, v.y};
    }
    return m;
  }
  __device__ __forceinline__ void store_off(int mu, unsigned o, const M3<T> &m) const {
#pragma unroll
    for (int k = 0; k < 9; k++) {
      V2<T> v;
      v.x = m.e[k].re;
      v.y = m.e[k].im;
      st_plane(p + (size_t)(mu * 18 + k) * Vh, o, v);
    }
  }
  __device__ __forceinline__ M3<T> load(int mu, int par, int h) const { return load_off(mu, off(par, h)); }
  __device__ __forceinline__ void store(int mu, int par, int h, const M3<T> &m) const {
    store_off(mu, off(par, h), m);
  }
  // link mu at the site with coordinates c
  __device__ __forceinline__ M3<T> at(const Geom &g, const int c[4], int mu) const {
    return load(mu, parity_of(c), half_index(g, c));
  }
};

// complex element (par, k, h) at (par*9 + k)*Vh + h
struct Gauge {
  double2 *p;
  int Vh;
  __device__ __forceinline__ unsigned off(int par, int h) const {
    return (unsigned)(par * 9 * Vh + h) * (unsigned)sizeof(double2);
  }
  __device__ __forceinline__ M3<double> load(int par, int h) const {
    const unsigned o = off(par, h);
    M3<double> m;
#pragma unroll
    for (int k = 0; k < 9; k++) {
      const double2 v = ld_plane(p + (size_t)k * Vh, o);
      m.e[k] = cx<double>{v.x, v.y};
    }
    return m;
  }
  __device__ __forceinline__ void store(int par, int h, const M3<double> &m) const {
    const unsigned o = off(par, h);
#pragma unroll
    for (int k = 0; k < 9; k++) st_plane(p + (size_t)k * Vh, o, make_double2(m.e[k].re, m.e[k].im));
  }
  __device__ __forceinline__ M3<double> load_fixed(int par, int h) const { return load(par, h); }
  // streaming forms (the ring fold: G is not touched again until the next fold)
  __device__ __forceinline__ M3<double> load_fixed_stream(int par, int h) const {
    const unsigned o = off(par, h);
    M3<double> m;
#pragma unroll
    for (int k = 0; k < 9; k++) {
      const double2 v = ld_plane_stream(p + (size_t)k * Vh, o);
      m.e[k] = cx<double>{v.x, v.y};
    }
    return m;
  }
  __device__ __forceinline__ void store_stream(int par, int h, const M3<double> &m) const {
    const unsigned o = off(par, h);
#pragma unroll
    for (int k = 0; k < 9; k++) st_plane_stream(p + (size_t)k * Vh, o, make_double2(m.e[k].re, m.e[k].im));
  }
};

// Make the compiler treat the first two rows of m as freshly produced, so a
// value derived from them (row 2) is recomputed instead of kept live across a
// long stretch of code (a register-pressure hint with no run-time cost).
template <typename T> __device__ __forceinline__ void opaque_rows(M3<T> &m) {
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
  for (int k = 0; k < 6; k++) __asm__ volatile("" : "+v"(m.e[k].re), "+v"(m.e[k].im));
#else
  (void)m;
#endif
}

// ------------------------------------------------- two-row (compressed) I/O
// An SU(3) matrix is fixed by its first two rows: row 2 = conj(row 0 x row 1).
// The fixing iteration keeps its working field and transform in this form:
// 12 reals per matrix instead of 18.
template <typename T> __device__ __forceinline__ void third_row(M3<T> &m) {
  m.e[6] = conj(m.e[1] * m.e[5] - m.e[2] * m.e[4]);
  m.e[7] = conj(m.e[2] * m.e[3] - m.e[0] * m.e[5]);
  m.e[8] = conj(m.e[0] * m.e[4] - m.e[1] * m.e[3]);
}

// complex element (mu, par, k < 6, h) at ((mu*2 + par)*6 + k)*Vh + h
template <typename T> struct Links12 {
  V2<T> *p;
  int Vh;
  __device__ __forceinline__ unsigned off(int par, int h) const {
    return (unsigned)(par * 6 * Vh + h) * (unsigned)sizeof(V2<T>);
  }
  // rows 0 and 1 only (row 2 left unset)
  __device__ __forceinline__ M3<T> load_rows(int mu, unsigned o) const {
    M3<T> m;
#pragma unroll
    for (int k = 0; k < 6; k++) {
      const V2<T> v = ld_plane(p + (size_t)(mu * 12 + k) * Vh, o);
      m.e[k] = cx<T>{v.x, v.y};
    }
    return m;
  }
  __device__ __forceinline__ M3<T> load_off(int mu, unsigned o) const {
    M3<T> m = load_rows(mu, o);
    third_row(m);
    return m;
  }
  __device__ __forceinline__ void store_off(int mu, unsigned o, const M3<T> &m) const {
#pragma unroll
    for (int k = 0; k < 6; k++) {
      V2<T> v;
      v.x = m.e[k].re;
      v.y = m.e[k].im;
      st_plane(p + (size_t)(mu * 12 + k) * Vh, o, v);
    }
  }
  __device__ __forceinline__ M3<T> load(int mu, int par, int h) const { return load_off(mu, off(par, h)); }
  __device__ __forceinline__ void store(int mu, int par, int h, const M3<T> &m) const {
    store_off(mu, off(par, h), m);
  }
};

// ----------------------------------------- products of rows in the fixed FMA order
// rows 0 and 1 of a b and of a b^dagger (row 2 zero); the first needs all of b, the second only
// rows 0 and 1 of a
template <typename T> __device__ __forceinline__ M3<T> mul_fixed_rows(const M3<T> &a, const M3<T> &b) {
  M3<T> c = m_zero<T>();
#pragma unroll
  for (int r = 0; r < 2; r++)
#pragma unroll
    for (int q = 0; q < 3; q++)
      c.e[3 * r + q] = dot3_fma(a.e[3 * r], b.e[q], a.e[3 * r + 1], b.e[3 + q], a.e[3 * r + 2], b.e[6 + q]);
  return c;
}
template <typename T> __device__ __forceinline__ M3<T> mul_nd_fixed_rows(const M3<T> &a, const M3<T> &b) {
  M3<T> c = m_zero<T>();
#pragma unroll
  for (int r = 0; r < 2; r++)
#pragma unroll
    for (int q = 0; q < 3; q++)
      c.e[3 * r + q] = dot3c_fma(a.e[3 * r], b.e[3 * q], a.e[3 * r + 1], b.e[3 * q + 1], a.e[3 * r + 2], b.e[3 * q + 2]);
  return c;
}
// conj(x y - z w), the product terms fused in a fixed order
template <typename T> __device__ __forceinline__ cx<T> cross_fma(cx<T> x, cx<T> y, cx<T> z, cx<T> w) {
  T re = x.re * y.re, im = x.re * y.im;
  re = fma_t(-x.im, y.im, re);
  im = fma_t(x.im, y.re, im);
  re = fma_t(-z.re, w.re, re);
  re = fma_t(z.im, w.im, re);
  im = fma_t(-z.re, w.im, im);
  im = fma_t(-z.im, w.re, im);
  return cx<T>{re, -im};
}
template <typename T> __device__ __forceinline__ void third_row_fixed(M3<T> &m) {
  m.e[6] = cross_fma(m.e[1], m.e[5], m.e[2], m.e[4]);
  m.e[7] = cross_fma(m.e[2], m.e[3], m.e[0], m.e[5]);
  m.e[8] = cross_fma(m.e[0], m.e[4], m.e[1], m.e[3]);
}

// complex element (par, k < 6, h) at (par*6 + k)*Vh + h
struct Gauge12 {
  double2 *p;
  int Vh;
  __device__ __forceinline__ unsigned off(int par, int h) const {
    return (unsigned)(par * 6 * Vh + h) * (unsigned)sizeof(double2);
  }
  __device__ __forceinline__ M3<double> load(int par, int h) const {
    M3<double> m = load_rows(par, h);
    third_row(m);
    return m;
  }
  __device__ __forceinline__ M3<double> load_rows(int par, int h) const {
    const unsigned o = off(par, h);
    M3<double> m;
#pragma unroll
    for (int k = 0; k < 6; k++) {
      const double2 v = ld_plane(p + (size_t)k * Vh, o);
      m.e[k] = cx<double>{v.x, v.y};
    }
    return m;
  }
  // load with row 2 rebuilt by third_row_fixed (for transform updates)
  __device__ __forceinline__ M3<double> load_fixed(int par, int h) const {
    M3<double> m = load_rows(par, h);
    third_row_fixed(m);
    return m;
  }
  // streaming forms (the ring fold: G is not touched again until the next fold)
  __device__ __forceinline__ M3<double> load_fixed_stream(int par, int h) const {
    const unsigned o = off(par, h);
    M3<double> m;
#pragma unroll
    for (int k = 0; k < 6; k++) {
      const double2 v = ld_plane_stream(p + (size_t)k * Vh, o);
      m.e[k] = cx<double>{v.x, v.y};
    }
    third_row_fixed(m);
    return m;
  }
  __device__ __forceinline__ void store_stream(int par, int h, const M3<double> &m) const {
    const unsigned o = off(par, h);
#pragma unroll
    for (int k = 0; k < 6; k++) st_plane_stream(p + (size_t)k * Vh, o, make_double2(m.e[k].re, m.e[k].im));
  }
  __device__ __forceinline__ void store(int par, int h, const M3<double> &m) const {
    const unsigned o = off(par, h);
#pragma unroll
    for (int k = 0; k < 6; k++) st_plane(p + (size_t)k * Vh, o, make_double2(m.e[k].re, m.e[k].im));
  }
};

// the two storage forms of the fixing iteration's working field and transform
template <typename T, bool C12> struct FixStore;
template <typename T> struct FixStore<T, false> {
  using W = Links<T>;
  using G = Gauge;
};
template <typename T> struct FixStore<T, true> {
  using W = Links12<T>;
  using G = Gauge12;
};

// ------------------------------------------------------------- reductions
// Butterfly sum over the 64 lanes of a wavefront (result in every lane): the
// same tree whatever the block size, so per-wave partials written at the
// wave's global index make a reduction independent of the launch shape.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block sum of one double per thread: butterfly within each
// 64-wide wavefront, then the per-wave sums in wave order.  Result valid in
// thread 0.  BS must be a multiple of 64.
template <int BS> __device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[BS / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) part[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < BS / 64; i++) r += part[i];
  }
  __syncthreads();  // part[] may be reused by a later call
  return r;
}
template <int BS> __device__ __forceinline__ double block_min(double v) {
  __shared__ double part[BS / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) part[w] = v;
  __syncthreads();
  double r = v;
  if (threadIdx.x == 0) {
    r = part[0];
#pragma unroll
    for (int i = 1; i < BS / 64; i++) r = fmin(r, part[i]);
  }
  __syncthreads();
  return r;
}
// Fixed-order sum of n partials by one block: thread t adds t, t+BS, ...
// in order, then block_sum.  Result valid in thread 0.
template <int BS, int NL = 8> __device__ __forceinline__ double sum_partials(const double *p, int n) {
  double s = 0.0;
  int i = threadIdx.x;
  // NL loads in flight per step; the additions keep the order i, i+BS, i+2BS, ...
  for (; i + (NL - 1) * BS < n; i += NL * BS) {
    double v[NL];
#pragma unroll
    for (int k = 0; k < NL; k++) v[k] = p[i + k * BS];
#pragma unroll
    for (int k = 0; k < NL; k++) s += v[k];
  }
  for (; i < n; i += BS) s += p[i];
  return block_sum<BS>(s);
}

}  // namespace mcg
