// k_loops.hip -- the centre part of a projected field and its remainder, and
// Wilson loops W(R, T) averaged over all sites (Sec. III.B of arXiv:0807.0264).
//   vortex-only     Z_mu(x) = exp(2 pi i m_mu(x) / 3) 1
//   vortex-removed  Z_mu(x)^dag U^G_mu(x)
//   W(R, T) = < Re tr(loop) / 3 >, the spatial side a path of unit steps
//   (built as a line field by k_line), the time sides straight.

#include "loops_kernels.hpp"

namespace mcg {

template <typename T>
hipError_t launch_vortex_field(const Geom &g, const void *U, const double *G, const int8_t *Z, int mode, void *out,
                               hipStream_t s) {
  k_vortex_field<T><<<(g.Vh + 255) / 256, 256, 0, s>>>(g, (const V2<T> *)U, (const double2 *)G, Z, mode,
                                                      (V2<T> *)out);
  return hipGetLastError();
}

int line_blocks(const Geom &g) { return 2 * ((g.Vh + 255) / 256); }

template <typename T>
hipError_t launch_line(const Geom &g, const void *U, const void *in, const SPathArg &path, const int off[3],
                       void *out, hipStream_t s) {
  SPath p;
  p.n = path.n;
  for (int k = 0; k < 3; k++) p.d[k] = path.d[k];
  for (int k = 0; k < MAX_PATH; k++) p.s[k] = k < path.n ? (signed char)path.s[k] : 0;
  k_line<T><<<line_blocks(g), 256, 0, s>>>(g, (const V2<T> *)U, (const V2<T> *)in, p, off[0], off[1], off[2],
                                           (V2<T> *)out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_wloop(const Geom &g, const void *U, const void *S, const int D[3], int tmax, double *part,
                        double weight, double *res, hipStream_t s) {
  const int nb = line_blocks(g);
  k_wloop<T, 256><<<nb, 256, 0, s>>>(g, (const V2<T> *)U, (const V2<T> *)S, D[0], D[1], D[2], tmax, part);
  k_wloop_final<<<tmax, 256, 0, s>>>(part, nb, weight, res);
  return hipGetLastError();
}

hipError_t launch_zero(double *p, int n, hipStream_t s) {
  k_zero<<<(n + 255) / 256, 256, 0, s>>>(p, n);
  return hipGetLastError();
}

#define MCG_LOOPS_INST(T)                                                                                  \
  template hipError_t launch_vortex_field<T>(const Geom &, const void *, const double *, const int8_t *, int, \
                                             void *, hipStream_t);                                         \
  template hipError_t launch_line<T>(const Geom &, const void *, const void *, const SPathArg &, const int *, \
                                     void *, hipStream_t);                                                 \
  template hipError_t launch_wloop<T>(const Geom &, const void *, const void *, const int *, int, double *,  \
                                      double, double *, hipStream_t);
MCG_LOOPS_INST(float)
MCG_LOOPS_INST(double)

}  // namespace mcg
