// k_smear.hip -- one Jacobi step of stout (eps = 1) or over-improved stout
// smearing (Sec. II.B and Sec. III of arXiv:0807.0264):
//   C = rho (wp Cp + wr Cr),  wp = (5 - 2 eps)/3,  wr = -(1 - eps)/12
//   U'_mu(x) = exp(TA(C U_mu(x)^dag)) U_mu(x)
// One thread per link; every new link is computed from the old field, so
// the input and output buffers are distinct.

#include "smear_kernels.hpp"

namespace mcg {

template <typename T>
hipError_t launch_smear_step(const Geom &g, const void *U, void *out, double rho, double eps,
                             hipStream_t s, void *Cst) {
  const double wp = (5.0 - 2.0 * eps) / 3.0, wr = -(1.0 - eps) / 12.0;
  const int grid = 8 * gather_tiles(g);
  if (!out) return hipErrorInvalidValue;
  const V2<T> *u = (const V2<T> *)U;
  V2<T> *o = (V2<T> *)out, *cs = (V2<T> *)Cst;
  const T r = (T)rho, p = (T)wp, q = (T)wr;
  if (eps == 1.0) {
    if (cs) k_smear<T, false, 1><<<grid, 128, 0, s>>>(g, u, o, r, p, q, cs);
    else k_smear<T, false><<<grid, 128, 0, s>>>(g, u, o, r, p, q);
  } else {
    if (cs) k_smear<T, true, 1><<<grid, 128, 0, s>>>(g, u, o, r, p, q, cs);
    else k_smear<T, true><<<grid, 128, 0, s>>>(g, u, o, r, p, q);
  }
  return hipGetLastError();
}

template hipError_t launch_smear_step<float>(const Geom &, const void *, void *, double, double, hipStream_t,
                                             void *);
template hipError_t launch_smear_step<double>(const Geom &, const void *, void *, double, double, hipStream_t,
                                              void *);

}  // namespace mcg
