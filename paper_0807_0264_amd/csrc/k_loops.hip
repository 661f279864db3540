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
hipError_t launch_lines(const Geom &g, const void *U, const LoopImage<T> *imgs, int nimg, int k, hipStream_t s) {
  k_line<T><<<dim3(line_blocks(g), nimg), 256, 0, s>>>(g, (const V2<T> *)U, imgs, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_wloops(const Geom &g, const void *U, const LoopImage<T> *imgs, int nimg, int k, int tmax,
                         double *part, double *res, hipStream_t s) {
  const int nb = line_blocks(g);
  k_wloop<T, 256><<<dim3(nb, nimg), 256, 0, s>>>(g, (const V2<T> *)U, imgs, k, tmax, part);
  k_wloop_final<T><<<tmax, 256, 0, s>>>(part, nb, nimg, tmax, imgs, res);
  return hipGetLastError();
}

hipError_t launch_zero(double *p, int n, hipStream_t s) {
  k_zero<<<(n + 255) / 256, 256, 0, s>>>(p, n);
  return hipGetLastError();
}

#define MCG_LOOPS_INST(T)                                                                                  \
  template hipError_t launch_vortex_field<T>(const Geom &, const void *, const double *, const int8_t *, int, \
                                             void *, hipStream_t);                                         \
  template hipError_t launch_lines<T>(const Geom &, const void *, const LoopImage<T> *, int, int, hipStream_t); \
  template hipError_t launch_wloops<T>(const Geom &, const void *, const LoopImage<T> *, int, int, int, double *, \
                                       double *, hipStream_t);
MCG_LOOPS_INST(float)
MCG_LOOPS_INST(double)

}  // namespace mcg
