// k_field.hip -- layout conversion (interchange <-> even/odd
// structure-of-arrays), gauge-field utilities, the gauge transform
// U^G_mu(x) = G(x) U_mu(x) G(x+mu)^dag and whole-field sums (the MCG
// functional of Sec. II.A and the plaquette).

#include "field_kernels.hpp"

namespace mcg {

int field_blocks256(const Geom &g) { return (g.Vh + 255) / 256; }

template <typename Tin, typename Tout>
hipError_t launch_pack_links(const Geom &g, const void *src, void *dst, hipStream_t s) {
  k_pack_links<Tin, Tout><<<(4 * g.V + 255) / 256, 256, 0, s>>>(g, (const V2<Tin> *)src, (V2<Tout> *)dst);
  return hipGetLastError();
}
template <typename Tin, typename Tout>
hipError_t launch_unpack_links(const Geom &g, const void *src, void *dst, hipStream_t s) {
  k_unpack_links<Tin, Tout><<<(4 * g.V + 255) / 256, 256, 0, s>>>(g, (const V2<Tin> *)src, (V2<Tout> *)dst);
  return hipGetLastError();
}
hipError_t launch_pack_gauge(const Geom &g, const double *src, double *dst, hipStream_t s) {
  k_pack_gauge<<<(g.V + 255) / 256, 256, 0, s>>>(g, (const double2 *)src, (double2 *)dst, 0);
  return hipGetLastError();
}
hipError_t launch_unpack_gauge(const Geom &g, const double *src, double *dst, hipStream_t s) {
  k_pack_gauge<<<(g.V + 255) / 256, 256, 0, s>>>(g, (const double2 *)src, (double2 *)dst, 1);
  return hipGetLastError();
}
hipError_t launch_gauge_identity(const Geom &g, double *G, hipStream_t s) {
  k_gauge_op<<<field_blocks256(g), 256, 0, s>>>(g, (double2 *)G, 0);
  return hipGetLastError();
}
hipError_t launch_gauge_reunit(const Geom &g, double *G, hipStream_t s) {
  k_gauge_op<<<field_blocks256(g), 256, 0, s>>>(g, (double2 *)G, 1);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_apply_gauge(const Geom &g, const void *U, const double *G, void *out, hipStream_t s) {
  k_apply_gauge<T><<<field_blocks256(g), 256, 0, s>>>(g, (const V2<T> *)U, (const double2 *)G, (V2<T> *)out);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_functional(const Geom &g, const void *U, double *part, double *out, hipStream_t s) {
  const int nb = field_blocks256(g);
  k_field_sum<T><<<nb, 256, 0, s>>>(g, (const V2<T> *)U, part, 0);
  k_final_sum<<<1, 256, 0, s>>>(part, nb, 1.0 / (9.0 * (double)(4 * g.V)), out);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_plaquette(const Geom &g, const void *U, double *part, double *out, hipStream_t s) {
  const int nb = field_blocks256(g);
  k_field_sum<T><<<nb, 256, 0, s>>>(g, (const V2<T> *)U, part, 1);
  k_final_sum<<<1, 256, 0, s>>>(part, nb, 1.0 / (18.0 * (double)g.V), out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_unitarity(const Geom &g, const void *U, int nmu, double *part, double *out, hipStream_t s) {
  const int nb = field_blocks256(g);
  k_unitarity<T><<<nb, 256, 0, s>>>(g, (const V2<T> *)U, nmu, part);
  k_max_final<<<1, 256, 0, s>>>(part, nb, out);
  return hipGetLastError();
}

template hipError_t launch_unitarity<float>(const Geom &, const void *, int, double *, double *, hipStream_t);
template hipError_t launch_unitarity<double>(const Geom &, const void *, int, double *, double *, hipStream_t);
template hipError_t launch_pack_links<double, double>(const Geom &, const void *, void *, hipStream_t);
template hipError_t launch_pack_links<double, float>(const Geom &, const void *, void *, hipStream_t);
template hipError_t launch_pack_links<float, float>(const Geom &, const void *, void *, hipStream_t);
template hipError_t launch_pack_links<float, double>(const Geom &, const void *, void *, hipStream_t);
template hipError_t launch_unpack_links<double, double>(const Geom &, const void *, void *, hipStream_t);
template hipError_t launch_unpack_links<double, float>(const Geom &, const void *, void *, hipStream_t);
template hipError_t launch_unpack_links<float, float>(const Geom &, const void *, void *, hipStream_t);
template hipError_t launch_unpack_links<float, double>(const Geom &, const void *, void *, hipStream_t);
template hipError_t launch_apply_gauge<float>(const Geom &, const void *, const double *, void *, hipStream_t);
template hipError_t launch_apply_gauge<double>(const Geom &, const void *, const double *, void *, hipStream_t);
template hipError_t launch_functional<float>(const Geom &, const void *, double *, double *, hipStream_t);
template hipError_t launch_functional<double>(const Geom &, const void *, double *, double *, hipStream_t);
template hipError_t launch_plaquette<float>(const Geom &, const void *, double *, double *, hipStream_t);
template hipError_t launch_plaquette<double>(const Geom &, const void *, double *, double *, hipStream_t);

}  // namespace mcg
