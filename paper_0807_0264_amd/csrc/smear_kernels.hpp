// smear_kernels.hpp -- the smearing-step kernel (launcher in k_smear.hip).
#pragma once

#include "internal.hpp"
#include "smear.hpp"

namespace mcg {

// CS = 1: also store the staple sums Cp (and Cr, OI) of every link in Cst, as two link fields
// [Cp | Cr], for the adjoint's first pass
template <typename T, bool OI, int CS = 0>
__global__ __launch_bounds__(128) void k_smear(Geom g, const V2<T> *__restrict__ U,
                                               V2<T> *__restrict__ out, T rho, T wp, T wr,
                                               V2<T> *__restrict__ Cst = nullptr) {
  // one block per (tile, direction, parity), the tiles as gather_site lays them out; the eight blocks
  // of a tile follow each other and each XCD takes a contiguous range of tiles (xcd_range), so the
  // staple links that the eight share, and those of the neighbouring tiles along z and t, are mostly
  // still in that XCD's L2
  const int w = xcd_range((int)blockIdx.x, (int)gridDim.x);
  const int h = gather_site(g, w >> 3, (int)threadIdx.x);
  if (h < 0) return;
  const int mu = (w & 7) >> 1, par = w & 1;
  const Links<T> L{const_cast<V2<T> *>(U), g.Vh};
  int c[4];
  coords_of(g, par, h, c);
  M3<T> Cp, Cr;
  staples<T, OI>(g, L, c, mu, Cp, Cr);
  if constexpr (CS != 0) {
    Links<T>{Cst, g.Vh}.store(mu, par, h, Cp);
    if (OI) Links<T>{Cst + (size_t)72 * g.Vh, g.Vh}.store(mu, par, h, Cr);
  }
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

}  // namespace mcg
