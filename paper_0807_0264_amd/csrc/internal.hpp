// internal.hpp -- host-side declarations of the kernel launchers (one per
// .hip translation unit).  All launchers enqueue on the given stream and
// return the launch status; `D` points to a device table of LatDesc<T>.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace mcg {

// k_mcg.hip -- fixing (bs = block size of the half-index grid; the
// half-sweep takes a variant = block size and occupancy, see variant_block)
constexpr int NUM_VARIANTS = 6;
inline int variant_block(int v) { return v % 3 == 0 ? 64 : (v % 3 == 1 ? 128 : 256); }
template <typename T>
// slab < 0: the whole of every field (blocks = total); slab >= 0: that slab's chunks (blocks = their total)
// hits > 1 (re-linearisation hits) or exact (exact subgroup maximisation) requires variant 2
// (256-thread blocks); rev: bit 0 tiles in reverse order within each residue class of the grid
// index mod 8, bit 1 contiguous tile ranges per XCD within each field (same results, other
// visiting order); gslot >= 0: g goes to that slot of each field's transform ring instead of into
// G (k_fold); paired sweeps (two-row form): keep = 1 leaves the links as they are (the first
// half-sweep of a sweep) and writes g to slot pend of d.gring (with the ring, pend = gslot), and
// pend >= 0 without keep names the slot whose g the links still wait for (the second half-sweep
// applies it as it loads them); for FP32 the first half runs 3 + variant / 3 waves per SIMD (it
// has no link products), the second 1 + variant / 3 like a plain half-sweep
hipError_t launch_halfsweep(int variant, bool c12, const void *D, int B, int blocks, int par, double omega,
                            bool withR, bool gated, hipStream_t s, int slab = -1, int hits = 1, int exact = 0,
                            int rev = 0, int gslot = -1, int pend = -1, int keep = 0);
// fold the ring's transforms into G (nfix: the count for fields without a FixState)
template <typename T>
hipError_t launch_fold(int bs, bool c12, const void *D, int B, int blocks, int nfix, hipStream_t s);
template <typename T>
hipError_t launch_rederive(int bs, bool c12, const void *D, int B, int blocks, bool gated, hipStream_t s);
template <typename T>
hipError_t launch_reunit(int bs, bool c12, const void *D, int B, int blocks, bool gated, hipStream_t s);
template <typename T>
hipError_t launch_theta(int bs, bool c12, const void *D, int B, int blocks, hipStream_t s);
template <typename T> hipError_t launch_book(const void *D, int B, int what, hipStream_t s);
// full (18 reals) <-> two-row (12 reals) forms of a link field / gauge field
template <typename T>
hipError_t launch_links_form(const Geom &g, const void *src, void *dst, bool to12, hipStream_t s);
hipError_t launch_gauge_form(const Geom &g, const double *src, double *dst, bool to12, hipStream_t s);
enum { BOOK_INIT = 0, BOOK_RESET = 1, BOOK_CHECK = 2, BOOK_FINAL = 3, BOOK_THETA = 4, BOOK_FOLD = 5 };
// most sweeps whose transforms an FP32 fix keeps in its ring before folding them into G
constexpr int GRING_SWEEPS = 25;
// ring length of a fix that re-unitarises every `re` sweeps: the fewest folds per block of re
// sweeps, spread evenly (re = 50: folds after sweeps 25 and 50 of each block)
inline int gring_sweeps(int re) {
  const int folds = (re + GRING_SWEEPS - 1) / GRING_SWEEPS;
  return (re + folds - 1) / folds;
}

// k_field.hip -- layout conversion and whole-field measurements
template <typename Tin, typename Tout>
hipError_t launch_pack_links(const Geom &g, const void *src, void *dst, hipStream_t s);
template <typename Tin, typename Tout>
hipError_t launch_unpack_links(const Geom &g, const void *src, void *dst, hipStream_t s);
hipError_t launch_pack_gauge(const Geom &g, const double *src, double *dst, hipStream_t s);
hipError_t launch_unpack_gauge(const Geom &g, const double *src, double *dst, hipStream_t s);
hipError_t launch_gauge_identity(const Geom &g, double *G, hipStream_t s);
hipError_t launch_gauge_reunit(const Geom &g, double *G, hipStream_t s);
template <typename T>
hipError_t launch_apply_gauge(const Geom &g, const void *U, const double *G, void *out, hipStream_t s);
// per-block partial sums into `part` (ceil(Vh/256) entries), then final sum into *out
template <typename T>
hipError_t launch_functional(const Geom &g, const void *U, double *part, double *out, hipStream_t s);
template <typename T>
hipError_t launch_plaquette(const Geom &g, const void *U, double *part, double *out, hipStream_t s);
int field_blocks256(const Geom &g);

// k_smear.hip -- one stout / over-improved stout step U -> out.  With Cst, the staple sums of every
// link are stored there too (field_bytes each: Cp, then Cr for eps != 1)
template <typename T>
hipError_t launch_smear_step(const Geom &g, const void *U, void *out, double rho, double eps,
                             hipStream_t s, void *Cst = nullptr);

// k_project.hip -- centre projection and vortex counting
template <typename T>
hipError_t launch_center_project(const Geom &g, const void *U, const double *G, int8_t *Z,
                                 double *part, double *min_out, hipStream_t s);
hipError_t launch_count_vortices(const Geom &g, const int8_t *Z, unsigned long long *counts,
                                 hipStream_t s);

// max_ij |(M M^dag - 1)_ij| over all matrices (nmu per site; NaN -> inf) into *out (device)
template <typename T>
hipError_t launch_unitarity(const Geom &g, const void *U, int nmu, double *part, double *out, hipStream_t s);

// k_loops.hip -- vortex-only / vortex-removed fields and Wilson loops.
// A spatial path for the line kernel: n unit steps +-(axis+1), displacement d.
constexpr int MAX_PATH = 32;
// a spatial step sequence: steps +-(axis + 1), axis < 3
struct SPath {
  int n;
  int d[3];  // displacement of the whole path
  signed char s[MAX_PATH];
};
// One image of a spatial path in a batched Wilson-loop launch: its steps, its weight in the
// average, and its two line fields (line k is built into a if k is odd, else into b, from the other).
template <typename T> struct LoopImage {
  SPath path;
  double weight;
  V2<T> *a, *b;
};
// images per batched Wilson-loop launch (each holds two line fields)
constexpr int LOOP_IMAGES_PER_LAUNCH = 16;
template <typename T>
hipError_t launch_vortex_field(const Geom &g, const void *U, const double *G, const int8_t *Z, int mode, void *out,
                               hipStream_t s);
int line_blocks(const Geom &g);
// for every image (device array of nimg <= LOOP_IMAGES_PER_LAUNCH): line k = line k - 1 times the
// path's links from x + (k - 1) d (line 0: 1); a line field holds 9 V complex of T
template <typename T>
hipError_t launch_lines(const Geom &g, const void *U, const LoopImage<T> *imgs, int nimg, int k, hipStream_t s);
// res[t] += sum over the images of weight * sum_x Re tr(loop with spatial line k of the image,
// displacement k d, time extent t + 1), t < tmax; part holds nimg * tmax * line_blocks(g) doubles
template <typename T>
hipError_t launch_wloops(const Geom &g, const void *U, const LoopImage<T> *imgs, int nimg, int k, int tmax,
                         double *part, double *res, hipStream_t s);
hipError_t launch_zero(double *p, int n, hipStream_t s);

// k_backward.hip -- adjoint of one smearing step and the loss seed.
// Seed: per-block sums of |tr W|^2 into part (field_blocks256 entries).
// Step (U12: scratch for U's links as two rows, the path factors of the gather):
// per-block (dL/drho, dL/deps) pairs into part[0 .. 2 nb) and, for
// eps = 1, the rectangle part of dL/deps into part[2 nb .. 3 nb), with
// nb = adjoint_blocks(g); *flag is set if an exponent lies outside the
// range of the unscaled series.
int adjoint_blocks(const Geom &g);
// out[0..2] = the loss, dL/drho and dL/deps from the partials of launch_loss_seed (nb_seed block
// sums) and of n launch_step_adjoint calls (3 nb entries each, as they lay them out), each summed in
// a fixed order on the device
hipError_t launch_reduce_parts(const double *part, int nb_seed, int n, int nb, double *out, hipStream_t s);
template <typename T>
hipError_t launch_loss_seed(const Geom &g, const void *S, const double *G, void *grad, double *part,
                            hipStream_t s);
// Cst: the staple sums of U as launch_smear_step stores them, or null (the first pass forms them)
template <typename T>
hipError_t launch_step_adjoint(const Geom &g, const void *U, const void *Cst, const void *gOut, void *gU, void *gC,
                               double rho, double eps, double *part, int *flag, hipStream_t s);

}  // namespace mcg
