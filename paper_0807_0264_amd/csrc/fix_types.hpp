// fix_types.hpp -- structures shared by the host driver and the fixing
// kernels: the per-field device state of the sweep loop and the descriptor
// of one field inside a (possibly batched) launch.
#pragma once

#include <stdint.h>

#include "common.hpp"

namespace mcg {

// Device-resident state of one field's fixing loop.  Written only by the
// single-block bookkeeping kernels (init / reset / check / final).
struct FixState {
  double R_prev;   // R before the current sweep
  double R_last;   // R after the last sweep
  double dR;       // R_last - R_prev of the last sweep
  double R_final;  // R after the final re-unitarisation
  double theta;    // stationarity residual of the final field
  double tol;
  int32_t k;       // sweeps done in this call
  int32_t max_k;   // sweeps allowed in this call
  int32_t done;    // 1 once converged or out of sweeps: every gated kernel exits at once
  int32_t status;  // 0 converged, 1 not converged
  int32_t stop_every;   // the stop test only after sweeps whose global number is a multiple of it
  int32_t start_sweep;  // global number of the sweep before this call's first
  int32_t kfold;        // sweeps whose transforms have been folded into G (k - kfold still in the ring)
};

constexpr int MAX_SLABS = 16;

// One field in a launch.  Blocks [blk0, blk0 + nblk) of a batched grid work
// on this field; block j covers half indices [j*BS, (j+1)*BS).  A half-sweep
// may instead run slab by slab: the field's blocks split into nslab
// contiguous chunks, chunk s = [s*nblk/nslab, (s+1)*nblk/nslab) (all blocks
// in chunk 0 when nslab = 1), and the launch for slab s maps its grid blocks
// [sblk0[s], sblk0[s] + size of chunk s) onto that chunk.
template <typename T> struct LatDesc {
  Geom g;
  int blk0, nblk;
  int nslab;
  int sblk0[MAX_SLABS];
  V2<T> *W;        // working field U^G (updated in place)
  const V2<T> *U;  // the field being fixed (read only)
  double2 *G;      // gauge transform (FP64)
  FixState *st;
  double *part;    // npart = nblk * BS / 64 partial sums, one per 64-site wavefront
  int npart;
  double *traj;    // device copy of the R trajectory (max_k + 1) or null
  // ring of per-half-sweep transforms (FP32 fields) or null: slot q holds rows 0 and 1 of the g of
  // every site of parity q & 1, complex element (q, k < 6, h) at (q*6 + k)*Vh + h; for FP64 fields
  // with paired sweeps, slot 0 alone: the even g handed to the odd half-sweep
  V2<T> *gring;
};

}  // namespace mcg
