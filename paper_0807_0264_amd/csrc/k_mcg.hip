// k_mcg.hip -- MCG fixing kernels (Sec. II.A of arXiv:0807.0264): the
// checkerboard half-sweep, re-derivation of the working field, G
// re-unitarisation, the stationarity residual, and the single-block
// bookkeeping kernels that keep each field's stop test on the device.
//
// Every kernel takes a table of LatDesc (one per field) and finds its field
// from blockIdx.x, so one launch serves a batch of fields of unequal sizes
// and the single-field path is the batch of one.  Per-field partial sums
// are reduced in a fixed order, so a field gives the same bits alone or in
// a batch.

#include "mcg_kernels.hpp"

namespace mcg {

// ---------------------------------------------------------- launchers
#define MCG_BS_SWITCH(bs, CALL) \
  switch (bs) {                 \
  case 64: { constexpr int BS = 64; CALL; } break;   \
  case 128: { constexpr int BS = 128; CALL; } break; \
  case 256: { constexpr int BS = 256; CALL; } break; \
  default: return hipErrorInvalidValue;              \
  }

// variant v: block size {64, 128, 256}[v % 3], waves per SIMD 1 + v / 3;
// c12: working field and transform stored as two rows
template <typename T>
hipError_t launch_halfsweep(int variant, bool c12, const void *D, int B, int blocks, int par, double omega,
                            bool withR, bool gated, hipStream_t s, int slab, int hits, int exact, int rev,
                            int gslot, int pend, int keep) {
  const LatDesc<T> *dd = (const LatDesc<T> *)D;
  const int bs = variant_block(variant), g = gated ? 1 : 0;
  // the paired form needs the two-row working field and a slot for the first half's g (with the
  // FP32 ring, that half-sweep's own ring slot)
  if ((pend >= 0 || keep) && !c12) return hipErrorInvalidValue;
  if (keep && (pend < 0 || withR || (gslot >= 0 && gslot != pend))) return hipErrorInvalidValue;
  if (hits > 1 || exact) {  // one instantiation: 256-thread blocks (the caller's descriptors use variant 2)
    if (bs != 256) return hipErrorInvalidValue;
#define MCG_HM(WR, C, E) \
  k_halfsweep<T, 256, WR, 1, C, true, E><<<blocks, 256, 0, s>>>(dd, B, par, (T)omega, g, slab, rev, gslot, pend, hits)
    {
      if (keep) {  // the first half of a paired sweep: the links stay, g goes to slot pend
#define MCG_HK(E) \
  k_halfsweep<T, 256, false, 1, true, true, E, KEEP><<<blocks, 256, 0, s>>>(dd, B, par, (T)omega, g, slab, rev, gslot, pend, hits)
        if (exact) MCG_HK(true); else MCG_HK(false);
#undef MCG_HK
        return hipGetLastError();
      }
      if (pend >= 0) {  // the second half: the pending g applied as the links are loaded
#define MCG_HP(WR, E) \
  k_halfsweep<T, 256, WR, 1, true, true, E, PEND><<<blocks, 256, 0, s>>>(dd, B, par, (T)omega, g, slab, rev, gslot, pend, hits)
        if (exact) {
          if (withR) MCG_HP(true, true); else MCG_HP(false, true);
        } else {
          if (withR) MCG_HP(true, false); else MCG_HP(false, false);
        }
#undef MCG_HP
        return hipGetLastError();
      }
    }
    if (exact) {
      if (c12) {
        if (withR) MCG_HM(true, true, true); else MCG_HM(false, true, true);
      } else {
        if (withR) MCG_HM(true, false, true); else MCG_HM(false, false, true);
      }
    } else {
      if (c12) {
        if (withR) MCG_HM(true, true, false); else MCG_HM(false, true, false);
      } else {
        if (withR) MCG_HM(true, false, false); else MCG_HM(false, false, false);
      }
    }
#undef MCG_HM
    return hipGetLastError();
  }
#define MCG_HS(WR, OCC, C)                                                                         \
  MCG_BS_SWITCH(bs, (k_halfsweep<T, BS, WR, OCC, C><<<blocks, BS, 0, s>>>(dd, B, par, (T)omega, g, slab, rev, gslot, pend)))
#define MCG_HK(OCC) \
  MCG_BS_SWITCH(bs, (k_halfsweep<T, BS, false, OCC, true, false, false, KEEP><<<blocks, BS, 0, s>>>(dd, B, par, (T)omega, g, slab, rev, gslot, pend)))
#define MCG_HP(WR, OCC) \
  MCG_BS_SWITCH(bs, (k_halfsweep<T, BS, WR, OCC, true, false, false, PEND><<<blocks, BS, 0, s>>>(dd, B, par, (T)omega, g, slab, rev, gslot, pend)))
  {
    // no link products: FP32 three waves per SIMD without spills (variants 0-2), four with a few
    // (3-5); FP64 as the variant says
    constexpr int K1 = sizeof(T) == 4 ? 3 : 1, K2 = sizeof(T) == 4 ? 4 : 2;
    if (keep) {
      if (variant / 3 == 0) { MCG_HK(K1); } else { MCG_HK(K2); }
      return hipGetLastError();
    }
    if (pend >= 0) {
      if (variant / 3 == 0) {
        if (withR) { MCG_HP(true, 1); } else { MCG_HP(false, 1); }
      } else {
        if (withR) { MCG_HP(true, 2); } else { MCG_HP(false, 2); }
      }
      return hipGetLastError();
    }
  }
#undef MCG_HK
#undef MCG_HP
  if (c12) {
    if (variant / 3 == 0) {
      if (withR) { MCG_HS(true, 1, true); } else { MCG_HS(false, 1, true); }
    } else {
      if (withR) { MCG_HS(true, 2, true); } else { MCG_HS(false, 2, true); }
    }
  } else {
    if (variant / 3 == 0) {
      if (withR) { MCG_HS(true, 1, false); } else { MCG_HS(false, 1, false); }
    } else {
      if (withR) { MCG_HS(true, 2, false); } else { MCG_HS(false, 2, false); }
    }
  }
#undef MCG_HS
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rederive(int bs, bool c12, const void *D, int B, int blocks, bool gated, hipStream_t s) {
  const LatDesc<T> *dd = (const LatDesc<T> *)D;
  if (c12) {
    MCG_BS_SWITCH(bs, (k_rederive<T, BS, true><<<blocks, BS, 0, s>>>(dd, B, gated ? 1 : 0)));
  } else {
    MCG_BS_SWITCH(bs, (k_rederive<T, BS, false><<<blocks, BS, 0, s>>>(dd, B, gated ? 1 : 0)));
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fold(int bs, bool c12, const void *D, int B, int blocks, int nfix, hipStream_t s) {
  const LatDesc<T> *dd = (const LatDesc<T> *)D;
  if (c12) {
    MCG_BS_SWITCH(bs, (k_fold<T, BS, true><<<blocks, BS, 0, s>>>(dd, B, nfix)));
  } else {
    MCG_BS_SWITCH(bs, (k_fold<T, BS, false><<<blocks, BS, 0, s>>>(dd, B, nfix)));
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_reunit(int bs, bool c12, const void *D, int B, int blocks, bool gated, hipStream_t s) {
  const LatDesc<T> *dd = (const LatDesc<T> *)D;
  if (c12) {
    MCG_BS_SWITCH(bs, (k_reunit<T, BS, true><<<blocks, BS, 0, s>>>(dd, B, gated ? 1 : 0)));
  } else {
    MCG_BS_SWITCH(bs, (k_reunit<T, BS, false><<<blocks, BS, 0, s>>>(dd, B, gated ? 1 : 0)));
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_theta(int bs, bool c12, const void *D, int B, int blocks, hipStream_t s) {
  const LatDesc<T> *dd = (const LatDesc<T> *)D;
  if (c12) {
    MCG_BS_SWITCH(bs, (k_theta<T, BS, true><<<blocks, BS, 0, s>>>(dd, B)));
  } else {
    MCG_BS_SWITCH(bs, (k_theta<T, BS, false><<<blocks, BS, 0, s>>>(dd, B)));
  }
  return hipGetLastError();
}

template <typename T> hipError_t launch_book(const void *D, int B, int what, hipStream_t s) {
  k_book<T><<<B, 1024, 0, s>>>((const LatDesc<T> *)D, what);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_links_form(const Geom &g, const void *src, void *dst, bool to12, hipStream_t s) {
  dim3 grid((g.Vh + 255) / 256, 8);
  k_links_form<T><<<grid, 256, 0, s>>>(g, (const V2<T> *)src, (V2<T> *)dst, to12 ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_gauge_form(const Geom &g, const double *src, double *dst, bool to12, hipStream_t s) {
  dim3 grid((g.Vh + 255) / 256, 2);
  k_gauge_form<<<grid, 256, 0, s>>>(g, (const double2 *)src, (double2 *)dst, to12 ? 1 : 0);
  return hipGetLastError();
}

#define MCG_INST(T)                                                                                  \
  template hipError_t launch_halfsweep<T>(int, bool, const void *, int, int, int, double, bool, bool,  \
                                          hipStream_t, int, int, int, int, int, int, int);           \
  template hipError_t launch_fold<T>(int, bool, const void *, int, int, int, hipStream_t);            \
  template hipError_t launch_rederive<T>(int, bool, const void *, int, int, bool, hipStream_t);       \
  template hipError_t launch_reunit<T>(int, bool, const void *, int, int, bool, hipStream_t);         \
  template hipError_t launch_theta<T>(int, bool, const void *, int, int, hipStream_t);                \
  template hipError_t launch_book<T>(const void *, int, int, hipStream_t);                            \
  template hipError_t launch_links_form<T>(const Geom &, const void *, void *, bool, hipStream_t);
MCG_INST(float)
MCG_INST(double)

}  // namespace mcg
