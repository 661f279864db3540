// k_backward.hip -- launchers of the smeared-field functional's adjoint
// (kernels in backward_kernels.hpp).

#include "backward_kernels.hpp"

namespace mcg {

int adjoint_blocks(const Geom &g) { return 8 * gather_tiles(g); }

template <typename T>
hipError_t launch_loss_seed(const Geom &g, const void *S, const double *G, void *grad, double *part,
                            hipStream_t s) {
  k_loss_seed<T><<<field_blocks256(g), 256, 0, s>>>(g, (const V2<T> *)S, (const double2 *)G, (V2<T> *)grad,
                                                     part);
  return hipGetLastError();
}

hipError_t launch_reduce_parts(const double *part, int nb_seed, int n, int nb, double *out, hipStream_t s) {
  k_reduce_parts<<<3, 1024, 0, s>>>(part, nb_seed, n, nb, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_adjoint(const Geom &g, const void *U, const void *Cst, const void *gOut, void *gU, void *gC,
                               double rho, double eps, double *part, int *flag, hipStream_t s) {
  const double wp = (5.0 - 2.0 * eps) / 3.0, wr = -(1.0 - eps) / 12.0;
  const int grid = adjoint_blocks(g);
  const int nb = grid;
  if (eps == 1.0) {
#define MCG_ADJ_A(OI, ST)                                                                                    \
  k_step_adj_a<T, OI, ST><<<grid, 128, 0, s>>>(g, (const V2<T> *)U, (const V2<T> *)Cst, (const V2<T> *)gOut,   \
                                               (V2<T> *)gU, (V2<T> *)gC, (T)rho, (T)wp, (T)wr, part, flag)
    if (Cst) MCG_ADJ_A(false, true); else MCG_ADJ_A(false, false);
    k_eps_rect<T><<<grid, 128, 0, s>>>(g, (const V2<T> *)U, (const V2<T> *)gC, (T)rho, part + 2 * nb);
    k_step_adj_b<T, false><<<grid, 128, 0, s>>>(g, (const V2<T> *)U, (const V2<T> *)gC, (V2<T> *)gU, (T)rho,
                                                (T)wp, (T)wr);
  } else {
    if (Cst) MCG_ADJ_A(true, true); else MCG_ADJ_A(true, false);
#undef MCG_ADJ_A
    k_step_adj_b<T, true><<<grid, 128, 0, s>>>(g, (const V2<T> *)U, (const V2<T> *)gC, (V2<T> *)gU, (T)rho,
                                               (T)wp, (T)wr);
  }
  return hipGetLastError();
}

template hipError_t launch_loss_seed<float>(const Geom &, const void *, const double *, void *, double *,
                                            hipStream_t);
template hipError_t launch_loss_seed<double>(const Geom &, const void *, const double *, void *, double *,
                                             hipStream_t);
template hipError_t launch_step_adjoint<float>(const Geom &, const void *, const void *, const void *, void *,
                                               void *, double, double, double *, int *, hipStream_t);
template hipError_t launch_step_adjoint<double>(const Geom &, const void *, const void *, const void *, void *,
                                                void *, double, double, double *, int *, hipStream_t);

}  // namespace mcg
