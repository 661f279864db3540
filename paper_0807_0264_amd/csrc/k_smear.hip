// k_smear.hip -- one Jacobi step of stout (eps = 1) or over-improved stout
// smearing (Sec. II.B and Sec. III of arXiv:0807.0264):
//   C = rho (wp Cp + wr Cr),  wp = (5 - 2 eps)/3,  wr = -(1 - eps)/12
//   U'_mu(x) = exp(TA(C U_mu(x)^dag)) U_mu(x)
// One thread per link; every new link is computed from the old field, so
// the input and output buffers are distinct.
#include "internal.hpp"
#include "smear.hpp"

namespace mcg {

template <typename T, bool OI>
__global__ __launch_bounds__(128) void k_smear(Geom g, const V2<T> *__restrict__ U,
                                               V2<T> *__restrict__ out, T rho, T wp, T wr) {
  const int h = blockIdx.x * 128 + threadIdx.x;
  if (h >= g.Vh) return;
  const int mu = blockIdx.y >> 1, par = blockIdx.y & 1;
  const Links<T> L{const_cast<V2<T> *>(U), g.Vh};
  int c[4];
  coords_of(g, par, h, c);
  M3<T> Cp, Cr;
  staples<T, OI>(g, L, c, mu, Cp, Cr);
  M3<T> C;
#pragma unroll
  for (int k = 0; k < 9; k++) {
    C.e[k] = rho * (wp * Cp.e[k]);
    if (OI) C.e[k] = rho * (wp * Cp.e[k] + wr * Cr.e[k]);
  }
  const M3<T> u = L.load(mu, par, h);
  const M3<T> E = exp_su3(ta(mul_nd(C, u)));
  Links<T>{out, g.Vh}.store(mu, par, h, mul(E, u));
}

template <typename T>
hipError_t launch_smear_step(const Geom &g, const void *U, void *out, double rho, double eps,
                             hipStream_t s) {
  const double wp = (5.0 - 2.0 * eps) / 3.0, wr = -(1.0 - eps) / 12.0;
  dim3 grid((g.Vh + 127) / 128, 8);
  if (eps == 1.0)
    k_smear<T, false><<<grid, 128, 0, s>>>(g, (const V2<T> *)U, (V2<T> *)out, (T)rho, (T)wp, (T)wr);
  else
    k_smear<T, true><<<grid, 128, 0, s>>>(g, (const V2<T> *)U, (V2<T> *)out, (T)rho, (T)wp, (T)wr);
  return hipGetLastError();
}

template hipError_t launch_smear_step<float>(const Geom &, const void *, void *, double, double, hipStream_t);
template hipError_t launch_smear_step<double>(const Geom &, const void *, void *, double, double, hipStream_t);

}  // namespace mcg
