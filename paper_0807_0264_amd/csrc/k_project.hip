// k_project.hip -- centre projection and P-vortex identification
// (Sec. II.A of arXiv:0807.0264).
//   Z_mu(x) = exp(2 pi i m / 3), m maximising Re(t e^{-2 pi i m/3}) with
//   t = tr(G(x) U_mu(x) G(x+mu)^dag) in FP64 (candidates 0, +1, -1; the first
//   wins a tie; t = 0 gives m = 0); margin = pi/3 - |arg(t e^{-2 pi i m/3})|.
//   A plaquette is a P-vortex when (m_mu(x) + m_nu(x+mu) - m_mu(x+nu) - m_nu(x))
//   mod 3 is non-zero.

#include <algorithm>

#include "project_kernels.hpp"

namespace mcg {

template <typename T>
hipError_t launch_center_project(const Geom &g, const void *U, const double *G, int8_t *Z,
                                 double *part, double *min_out, hipStream_t s) {
  const int nb = field_blocks256(g);
  k_center_project<T><<<nb, 256, 0, s>>>(g, (const V2<T> *)U, (const double2 *)G, Z, part);
  k_min_final<<<1, 256, 0, s>>>(part, nb, min_out);
  return hipGetLastError();
}

hipError_t launch_count_vortices(const Geom &g, const int8_t *Z, unsigned long long *counts,
                                 hipStream_t s) {
  // a few blocks per CU, each site visited by one thread of a grid-stride loop
  const int blocks = std::min((g.V + 255) / 256, 2048);
  k_count_vortices<<<blocks, 256, 0, s>>>(g, Z, counts);
  return hipGetLastError();
}

template hipError_t launch_center_project<float>(const Geom &, const void *, const double *, int8_t *,
                                                 double *, double *, hipStream_t);
template hipError_t launch_center_project<double>(const Geom &, const void *, const double *, int8_t *,
                                                  double *, double *, hipStream_t);

}  // namespace mcg
