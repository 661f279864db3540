// mcg_api.cpp -- the C ABI declared in include/mcg.h: context and scratch
// management, argument checks, precision dispatch, the sweep driver of the
// fixing iteration (direct launches for a single field, a captured hipGraph
// per block of sweeps for batches) and the block-size autotuner.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "fix_types.hpp"
#include "internal.hpp"
#include "mcg.h"

using namespace mcg;

namespace {

struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
};

}  // namespace

struct mcg_ctx {
  int device = 0;
  std::string err;
  hipStream_t cap_stream = nullptr;  // stream used only to capture graphs
  DevBuf part, scalars, counts, states, desc, tmpfield, grad_a, grad_b, gC, ckpt, bw_part, w12, g12;
  DevBuf line_a, line_b, wl_part, wl_res, wl_img;  // Wilson loops: line fields, partial sums, results, images
  std::vector<DevBuf> W, G12, fpart, traj, gring;
  std::vector<DevBuf> smeared;  // mcg_precondition_batch: the smeared fields
  DevBuf pc_part, pc_counts;    // mcg_precondition_batch: margin partials and vortex counters
  void *h_pinned = nullptr;
  size_t h_pinned_cap = 0;
  bool c12 = true;  // fixing keeps W and G as two rows (MCG_OPT_TWO_ROW)
  int nslab = 1;    // half-sweeps run slab by slab when > 1 (MCG_OPT_SLABS)
  int hits = 1;     // re-linearisation hits per site visit (MCG_OPT_HITS)
  bool exact = false;  // exact maximisation over each SU(2) subgroup (MCG_OPT_EXACT)
  int order = 2;       // 1: odd half-sweeps visit the tiles in reverse order; 2: and each XCD a contiguous range (MCG_OPT_ORDER)
  bool defer_g = true;  // FP32 fixes keep each half-sweep's g in a ring, folded into G later (MCG_OPT_DEFER_G)
  int paired = 1;  // 1: FP32 (ring) sweeps paired, 2: FP64 too (MCG_OPT_PAIRED)
  bool check = false;       // validate input links and transforms (MCG_OPT_CHECK)
  size_t scratch_limit = 0;  // bytes of device scratch the context may hold, 0 = no limit
  size_t scratch_used = 0;
  int stop_every = 1;  // stop test only after sweeps numbered by multiples of this (MCG_OPT_STOP_EVERY)
  int variant[2][2] = {{2, 2}, {2, 2}};  // half-sweep variant per [precision][two-row form]
  // launch variant and schedule chosen by mcg_tune_batch, per batch shape (tune_key); used by the
  // fixes of that shape until an explicit variant or schedule option is set
  std::map<std::string, mcg_tune_choice> tuned;
  double *noalloc = nullptr;  // this device's address of the allocation-free entry point's scratch
  std::string noalloc_err;    // why it is missing, if it is
};

// Scratch of the allocation-free centre projection (mcg_center_project_noalloc): the per-block
// minima of the centre-phase margin, one per 256 half sites, then the final minimum.  Every GPU the
// library runs on holds its own copy until the process ends.  In host code `scratch` names a
// host-side stand-in: the kernels get this device's address of it, looked up once per device.
constexpr int NOALLOC_PARTS = 65536;  // ceil(V / 512) <= 65536: lattices of up to 2^25 sites
static __device__ __align__(256) double scratch[NOALLOC_PARTS + 32];

namespace {

std::mutex noalloc_mu;
std::vector<double *> noalloc_ptr;  // per device, filled on the first context of that device

// With `device` current: this device's address of `scratch` (cached), or the runtime's error.
hipError_t noalloc_scratch(int device, double **out) {
  std::lock_guard<std::mutex> lk(noalloc_mu);
  if ((int)noalloc_ptr.size() <= device) noalloc_ptr.resize(device + 1, nullptr);
  if (!noalloc_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e;
    }
    noalloc_ptr[device] = (double *)p;
  }
  *out = noalloc_ptr[device];
  return hipSuccess;
}

}  // namespace

namespace {

// A ROCTX range around one call of the ABI (smear, fix, fix_batch, projection, counting, backward,
// Wilson loops), and nested ones around the phases of the batched pipeline and the backward, so
// that a trace groups the kernels of a call under its name.
struct Range {
  explicit Range(const char *name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range &) = delete;
  Range &operator=(const Range &) = delete;
};

mcg_status fail(mcg_ctx *ctx, mcg_status s, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return s;
}

#define HIPCHK(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(ctx, MCG_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),   \
                  __FILE__, __LINE__);                                                    \
  } while (0)

mcg_status ensure(mcg_ctx *ctx, DevBuf &b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return MCG_OK;
  if (ctx->scratch_limit && ctx->scratch_used - b.cap + bytes > ctx->scratch_limit)
    return fail(ctx, MCG_ENOMEM, "context scratch limit of %zu bytes reached (%zu held, %zu more requested)",
                ctx->scratch_limit, ctx->scratch_used, bytes - b.cap);
  if (b.p) {
    hipError_t e = hipFree(b.p);
    ctx->scratch_used -= b.cap;
    b.p = nullptr;
    b.cap = 0;
    if (e != hipSuccess) return fail(ctx, MCG_EHIP, "hipFree: %s", hipGetErrorString(e));
  }
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(ctx, MCG_ENOMEM, "device allocation of %zu bytes failed", bytes);
  }
  b.cap = bytes;
  ctx->scratch_used += bytes;
  return MCG_OK;
}

mcg_status ensure_pinned(mcg_ctx *ctx, size_t bytes) {
  if (ctx->h_pinned_cap >= bytes) return MCG_OK;
  if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
  ctx->h_pinned = nullptr;
  ctx->h_pinned_cap = 0;
  if (hipHostMalloc(&ctx->h_pinned, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, MCG_ENOMEM, "pinned host allocation of %zu bytes failed", bytes);
  }
  ctx->h_pinned_cap = bytes;
  return MCG_OK;
}

bool dims_valid(const mcg_dims &d) {
  int64_t V = 1;
  for (int k = 0; k < 4; k++) {
    if (d.L[k] < 2 || (d.L[k] & 1)) return false;
    V *= d.L[k];
  }
  // Loads address a (mu, k) plane by a wave-uniform base pointer plus a 32-bit byte offset of up to
  // (9 V/2 + V/2) * 16 = 80 V (FP64 elements, both parities), so 80 V < 2^32: V < 53,687,092.
  return 80 * V < (int64_t(1) << 32);
}

Geom geom_of(const mcg_dims &d) {
  Geom g;
  for (int k = 0; k < 4; k++) g.L[k] = d.L[k];
  g.V = d.L[0] * d.L[1] * d.L[2] * d.L[3];
  g.Vh = g.V / 2;
  g.hx = d.L[0] / 2;
  return g;
}

bool same_dims(const mcg_dims &a, const mcg_dims &b) {
  return a.L[0] == b.L[0] && a.L[1] == b.L[1] && a.L[2] == b.L[2] && a.L[3] == b.L[3];
}

mcg_status check_field(mcg_ctx *ctx, const mcg_field *f, const char *name) {
  if (!f) return fail(ctx, MCG_EINVAL, "%s is NULL", name);
  if (!dims_valid(f->d))
    return fail(ctx, MCG_EINVAL, "%s: extents (%d,%d,%d,%d) must be even, >= 2, with V < 53687092", name,
                f->d.L[0], f->d.L[1], f->d.L[2], f->d.L[3]);
  if (f->prec != MCG_F64 && f->prec != MCG_F32) return fail(ctx, MCG_EINVAL, "%s: bad precision %d", name, f->prec);
  if (!f->ptr) return fail(ctx, MCG_EINVAL, "%s: NULL data pointer", name);
  return MCG_OK;
}

mcg_status check_gauge(mcg_ctx *ctx, const mcg_gauge *G, const mcg_dims &d, const char *name) {
  if (!G || !G->ptr) return fail(ctx, MCG_EINVAL, "%s is NULL", name);
  if (!same_dims(G->d, d)) return fail(ctx, MCG_EINVAL, "%s: extents differ from the field's", name);
  return MCG_OK;
}

size_t field_bytes(const mcg_dims &d, int prec) {
  if (!dims_valid(d)) return 0;
  // 4 links x 9 complex entries x 2 reals per site
  size_t V = (size_t)d.L[0] * d.L[1] * d.L[2] * d.L[3];
  return V * 72 * (prec == MCG_F64 ? sizeof(double) : sizeof(float));
}

int nblocks(const Geom &g, int bs) { return (g.Vh + bs - 1) / bs; }

// working-field and transform bytes of the fixing iteration in the chosen form
size_t work_field_bytes(const mcg_dims &d, int prec, bool c12) {
  return c12 ? field_bytes(d, prec) / 3 * 2 : field_bytes(d, prec);
}
size_t gauge_form_bytes(const mcg_dims &d, bool c12) {
  const size_t V = (size_t)d.L[0] * d.L[1] * d.L[2] * d.L[3];
  return V * (c12 ? 6 : 9) * 2 * sizeof(double);
}
// the transform ring of an FP32 fix holding C sweeps: 2C slots of Vh two-row FP32 matrices
size_t gring_bytes(const Geom &g, int C) { return (size_t)2 * C * 6 * g.Vh * sizeof(V2<float>); }

// Reserve the rings of fields 0..B-1.  The ring is optional: when it does not fit (device memory or
// the context's scratch limit), the call updates G in place instead, with the same results, and the
// context's last error is left as it was.
bool reserve_rings(mcg_ctx *ctx, int B, const mcg_field *U, int C) {
  const std::string err = ctx->err;
  for (int b = 0; b < B; b++)
    if (ensure(ctx, ctx->gring[b], gring_bytes(geom_of(U[b].d), C)) != MCG_OK) {
      ctx->err = err;
      return false;
    }
  return true;
}

// ------------------------------------------------------------ fixing driver
// Largest |(M M^dag - 1)_ij| over U's links (and G's matrices when G is given), NaN as inf; host
// results, synchronises the stream.
mcg_status unitarity(mcg_ctx *ctx, const mcg_field *U, const mcg_gauge *G, double *devU, double *devG,
                     hipStream_t s) {
  const mcg_dims &d = U ? U->d : G->d;
  const Geom g = geom_of(d);
  mcg_status st;
  if ((st = ensure(ctx, ctx->part, sizeof(double) * field_blocks256(g))) || (st = ensure(ctx, ctx->scalars, 64)))
    return st;
  double *dv = (double *)ctx->scalars.p + 4;
  if (U) {
    if (U->prec == MCG_F64)
      HIPCHK(launch_unitarity<double>(g, U->ptr, 4, (double *)ctx->part.p, dv, s));
    else
      HIPCHK(launch_unitarity<float>(g, U->ptr, 4, (double *)ctx->part.p, dv, s));
  }
  if (G) HIPCHK(launch_unitarity<double>(g, G->ptr, 1, (double *)ctx->part.p, dv + 1, s));
  double h[2] = {0.0, 0.0};
  HIPCHK(hipMemcpyAsync(h, dv, sizeof h, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (devU) *devU = U ? h[0] : 0.0;
  if (devG) *devG = G ? h[1] : 0.0;
  return MCG_OK;
}

// In check mode: MCG_EINPUT unless every link of U (nullable) is unitary to 1e-6 (FP32) or 1e-10
// (FP64) and every matrix of G (nullable) to 1e-10, with no NaN.
mcg_status check_inputs(mcg_ctx *ctx, const mcg_field *U, const mcg_gauge *G, hipStream_t s) {
  if (!ctx->check || (!U && !G)) return MCG_OK;
  double du = 0.0, dg = 0.0;
  mcg_status st = unitarity(ctx, U, G, &du, &dg, s);
  if (st) return st;
  const double tu = U && U->prec == MCG_F32 ? 1e-6 : 1e-10;
  if (U && !(du <= tu)) return fail(ctx, MCG_EINPUT, "U is not unitary: max |U U^dag - 1| = %g (limit %g)", du, tu);
  if (G && !(dg <= 1e-10))
    return fail(ctx, MCG_EINPUT, "G is not unitary: max |G G^dag - 1| = %g (limit 1e-10)", dg);
  return MCG_OK;
}

// Slab plan of a launch table: a field is split into n chunks of its blocks (LatDesc) when every
// chunk holds at least two time slices' worth of half sites.  Every neighbour of a site then lies
// in the same chunk or the next one on either side (cyclically): spatial neighbours differ by less
// than one slice in the half index, time neighbours by exactly one slice.  grid[s] = blocks of the
// launch for slab s.  Returns n, or 1 when no field is split (whole-field launches).
template <typename T> int plan_slabs(LatDesc<T> *D, int B, int n, int bs, int grid[MAX_SLABS]) {
  n = std::max(1, std::min(n, MAX_SLABS));
  bool any = false;
  for (int b = 0; b < B; b++) {
    const int64_t vs = (int64_t)D[b].g.L[0] * D[b].g.L[1] * D[b].g.L[2];
    const bool split = n > 1 && ((int64_t)(D[b].nblk / n) - 1) * bs >= vs;
    D[b].nslab = split ? n : 1;
    any = any || split;
  }
  for (int k = 0; k < MAX_SLABS; k++) grid[k] = 0;
  if (!any) return 1;
  for (int k = 0; k < n; k++) {
    int tot = 0;
    for (int b = 0; b < B; b++) {
      D[b].sblk0[k] = tot;
      const int nb = D[b].nblk, ns = D[b].nslab;
      tot += ns > 1 ? ((k + 1) * nb) / ns - (k * nb) / ns : (k == 0 ? nb : 0);
    }
    grid[k] = tot;
  }
  return n;
}

// the tile-order argument of a half-sweep of parity par: bit 0 reverse, bit 1 contiguous XCD ranges
static int tile_order(int order, int par) { return order == 0 ? 0 : (order == 2 ? 2 : 0) | (par == 1 ? 1 : 0); }

// The launch variant and schedule of the fixing sweeps of a batch: what mcg_tune_batch chose for
// this batch shape (precision, storage form, transform ring, update variant, the fields' extents in
// order), else the context's variant and options.  Re-linearisation hits and exact steps run with
// 256-thread blocks (variant 2).  Every choice gives the same bits.
struct Sched {
  int variant, order, paired, nslab;
};
std::string tune_key(const mcg_ctx *ctx, int B, const mcg_field *U) {
  std::string k = std::to_string(U[0].prec) + (ctx->c12 ? "/rows" : "/full") + (ctx->defer_g ? "/ring" : "/G") +
                  "/hits" + std::to_string(ctx->hits) + (ctx->exact ? "/exact" : "");
  for (int b = 0; b < B; b++) {
    k += ":";
    for (int j = 0; j < 4; j++) k += (j ? "x" : "") + std::to_string(U[b].d.L[j]);
  }
  return k;
}
Sched schedule_of(const mcg_ctx *ctx, int B, const mcg_field *U) {
  Sched r{ctx->variant[U[0].prec][ctx->c12], ctx->order, ctx->paired, ctx->nslab};
  const auto it = ctx->tuned.find(tune_key(ctx, B, U));
  if (it != ctx->tuned.end()) r = Sched{it->second.variant, it->second.order, it->second.paired, it->second.slabs};
  if (ctx->hits > 1 || ctx->exact) r.variant = 2;
  return r;
}

template <typename T> struct FixRun {
  mcg_ctx *ctx;
  hipStream_t s;
  int B, variant, bs, total_blocks;
  bool c12;
  void *dD;  // device LatDesc table
  double omega;
  int nslab = 1;
  int grid[MAX_SLABS] = {};
  bool gated = true;
  int hits = 1;
  int exact = 0;
  int order = 0;
  // Deferred transform: with C > 0 every half-sweep writes its g into ring slot
  // 2 * since_fold + parity instead of updating G, and fold() applies the ring to G before
  // anything reads G (re-unitarisation, the end of the call) and whenever C sweeps are in it.
  int C = 0;
  int since_fold = 0;
  bool stateful = true;  // fields carry a FixState (the fold count comes from it)
  // Paired sweeps (two-row form with the FP32 ring, or FP64 with a one-slot handoff `hand`): the
  // even half-sweep leaves the links and records g (in its ring slot, or in the handoff slot 0),
  // the odd one applies it to the links it loads.
  bool paired = false;
  bool hand = false;

  mcg_status pass(int par, bool wr, int slab) {
    const int blocks = slab < 0 ? total_blocks : grid[slab];
    const int slot = C ? 2 * since_fold + par : -1;
    const bool pr = paired && c12 && (C || hand);
    int pend = -1, keep = 0;
    if (pr) {
      keep = par == 0 ? 1 : 0;
      pend = C ? (par == 0 ? slot : slot - 1) : 0;
    }
    if (blocks > 0)
      HIPCHK(launch_halfsweep<T>(variant, c12, dD, B, blocks, par, omega, wr, gated, s, slab, hits, exact,
                                 tile_order(order, par), slot, pend, keep));
    return MCG_OK;
  }
  // Launched whatever since_fold says on the host: a field's own count decides what is folded,
  // so a captured block that starts with a fold is right on every replay.
  mcg_status fold() {
    if (!C) return MCG_OK;
    HIPCHK(launch_fold<T>(bs, c12, dD, B, total_blocks, since_fold, s));
    if (stateful) HIPCHK(launch_book<T>(dD, B, BOOK_FOLD, s));
    since_fold = 0;
    return MCG_OK;
  }
  mcg_status advance() {
    if (C && ++since_fold == C) return fold();
    return MCG_OK;
  }
  // Even then odd half-sweep.  Slab by slab (n > 1), in the order E0 E1 [E(k) O(k-1)] for
  // k = 2..n-1, O(n-1) O0: odd slab k runs once even slabs k-1, k, k+1 are done, and no even slab
  // runs after an odd slab next to it, so the result is that of the two whole half-sweeps, while
  // the data of a slab is re-read soon after it was written.
  mcg_status halfsweeps(bool wr) {
    mcg_status st;
    if (nslab <= 1) {
      if ((st = pass(0, false, -1)) || (st = pass(1, wr, -1))) return st;
      return MCG_OK;
    }
    if ((st = pass(0, false, 0)) || (st = pass(0, false, 1))) return st;
    for (int k = 2; k < nslab; k++)
      if ((st = pass(0, false, k)) || (st = pass(1, wr, k - 1))) return st;
    if ((st = pass(1, wr, nslab - 1)) || (st = pass(1, wr, 0))) return st;
    return MCG_OK;
  }
  mcg_status sweep(bool reunit_first) {
    mcg_status st;
    if (reunit_first) {
      if ((st = fold())) return st;
      HIPCHK(launch_reunit<T>(bs, c12, dD, B, total_blocks, true, s));
      HIPCHK(launch_rederive<T>(bs, c12, dD, B, total_blocks, true, s));
      HIPCHK(launch_book<T>(dD, B, BOOK_RESET, s));
    }
    if ((st = halfsweeps(true))) return st;
    HIPCHK(launch_book<T>(dD, B, BOOK_CHECK, s));
    return advance();
  }
};

template <typename T>
mcg_status fix_impl(mcg_ctx *ctx, int B, const mcg_field *U, mcg_gauge *G, const mcg_fix_opts *opts,
                    mcg_fix_result *res, hipStream_t s, bool batch) {
  const int prec = std::is_same<T, double>::value ? MCG_F64 : MCG_F32;
  if (B < 1) return fail(ctx, MCG_EINVAL, "batch size %d < 1", B);
  if (!U || !G || !opts || !res) return fail(ctx, MCG_EINVAL, "NULL argument");
  const double omega = opts[0].omega;
  const int re = opts[0].reunit_every, s0 = opts[0].start_sweep;
  const int check_every = std::max(1, opts[0].check_every);
  int kmax = 0;
  for (int b = 0; b < B; b++) {
    mcg_status st = check_field(ctx, &U[b], "U");
    if (st) return st;
    if (U[b].prec != prec) return fail(ctx, MCG_EINVAL, "field %d: precision differs within the batch", b);
    if ((st = check_gauge(ctx, &G[b], U[b].d, "G"))) return st;
    const mcg_fix_opts &o = opts[b];
    if (o.max_sweeps < 0) return fail(ctx, MCG_EINVAL, "max_sweeps < 0");
    if (o.reunit_every < 1) return fail(ctx, MCG_EINVAL, "reunit_every < 1");
    if (!(o.omega >= 0.0 && o.omega <= 2.0)) return fail(ctx, MCG_EINVAL, "omega must lie in [0, 2]");
    if (std::isnan(o.tol)) return fail(ctx, MCG_EINVAL, "tol is NaN");
    if (o.omega != omega || o.reunit_every != re || o.start_sweep != s0)
      return fail(ctx, MCG_EINVAL, "omega, reunit_every and start_sweep must agree across the batch");
    kmax = std::max(kmax, o.max_sweeps);
    for (int c = 0; c < b; c++)
      if (U[c].ptr == U[b].ptr && G[c].ptr == G[b].ptr)
        return fail(ctx, MCG_EINVAL, "fields %d and %d share U and G", c, b);
    if ((st = check_inputs(ctx, &U[b], &G[b], s))) return st;
  }
  const bool c12 = ctx->c12;
  const Sched sc = schedule_of(ctx, B, U);
  const int variant = sc.variant, bs = variant_block(variant);
  if ((int)ctx->W.size() < B) {
    ctx->W.resize(B);
    ctx->G12.resize(B);
    ctx->fpart.resize(B);
    ctx->traj.resize(B);
    ctx->gring.resize(B);
  }
  bool ring = prec == MCG_F32 && ctx->defer_g;
  mcg_status st;
  if ((st = ensure(ctx, ctx->states, sizeof(FixState) * B))) return st;
  if ((st = ensure(ctx, ctx->desc, sizeof(LatDesc<T>) * B))) return st;
  if ((st = ensure_pinned(ctx, (sizeof(LatDesc<T>) + sizeof(FixState)) * B + 64))) return st;
  LatDesc<T> *hD = (LatDesc<T> *)ctx->h_pinned;
  FixState *hS = (FixState *)(hD + B);
  int total = 0;
  for (int b = 0; b < B; b++) {
    const Geom g = geom_of(U[b].d);
    const int nb = nblocks(g, bs);
    if ((st = ensure(ctx, ctx->W[b], work_field_bytes(U[b].d, prec, c12)))) return st;
    if (c12 && (st = ensure(ctx, ctx->G12[b], gauge_form_bytes(U[b].d, true)))) return st;
    if ((st = ensure(ctx, ctx->fpart[b], sizeof(double) * nb * (bs / 64)))) return st;
    const bool want_traj = opts[b].traj != nullptr;
    if (want_traj && (st = ensure(ctx, ctx->traj[b], sizeof(double) * (opts[b].max_sweeps + 1)))) return st;
    LatDesc<T> d;
    d.g = g;
    d.blk0 = total;
    d.nblk = nb;
    d.W = (V2<T> *)ctx->W[b].p;
    d.U = (const V2<T> *)U[b].ptr;
    d.G = c12 ? (double2 *)ctx->G12[b].p : (double2 *)G[b].ptr;
    d.st = (FixState *)ctx->states.p + b;
    d.part = (double *)ctx->fpart[b].p;
    d.npart = nb * (bs / 64);
    d.traj = want_traj ? (double *)ctx->traj[b].p : nullptr;
    d.gring = nullptr;
    hD[b] = d;
    FixState f;
    memset(&f, 0, sizeof f);
    f.tol = opts[b].tol;
    f.max_k = opts[b].max_sweeps;
    f.stop_every = ctx->stop_every;
    f.start_sweep = s0;
    hS[b] = f;
    total += nb;
  }
  // the ring (or FP64's handoff slot for paired sweeps) last, after everything the fix cannot do
  // without
  if (ring) ring = reserve_rings(ctx, B, U, gring_sweeps(re));
  bool hand = prec == MCG_F64 && c12 && sc.paired == 2;
  if (hand) hand = reserve_rings(ctx, B, U, 1);
  for (int b = 0; b < B && (ring || hand); b++) hD[b].gring = (V2<T> *)ctx->gring[b].p;
  FixRun<T> run{ctx, s, B, variant, bs, total, c12, ctx->desc.p, omega};
  run.nslab = plan_slabs(hD, B, sc.nslab, bs, run.grid);
  run.hits = ctx->hits;
  run.exact = ctx->exact ? 1 : 0;
  run.order = sc.order;
  run.C = ring ? gring_sweeps(re) : 0;
  run.paired = sc.paired != 0;
  run.hand = hand;
  HIPCHK(hipMemcpyAsync(ctx->desc.p, hD, sizeof(LatDesc<T>) * B, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ctx->states.p, hS, sizeof(FixState) * B, hipMemcpyHostToDevice, s));
  // the pinned staging area is reused below: wait for these copies first
  HIPCHK(hipStreamSynchronize(s));

  if (c12)
    for (int b = 0; b < B; b++)
      HIPCHK(launch_gauge_form(geom_of(U[b].d), G[b].ptr, (double *)ctx->G12[b].p, true, s));
  HIPCHK(launch_rederive<T>(bs, c12, run.dD, B, total, false, s));
  HIPCHK(launch_book<T>(run.dD, B, BOOK_INIT, s));

  auto all_done = [&](bool &done) -> mcg_status {
    HIPCHK(hipMemcpyAsync(hS, ctx->states.p, sizeof(FixState) * B, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    done = true;
    for (int b = 0; b < B; b++) done = done && hS[b].done;
    return MCG_OK;
  };
  auto due = [&](int k) { return k > 1 && (s0 + k - 1) % re == 0; };

  int issued = 0;
  bool done = kmax == 0;
  if (!batch) {
    while (!done && issued < kmax) {
      const int chunk = std::min(check_every, kmax - issued);
      for (int j = 0; j < chunk; j++) {
        ++issued;
        if ((st = run.sweep(due(issued)))) return st;
      }
      if ((st = all_done(done))) return st;
    }
  } else {
    // sweeps up to the next re-unitarisation boundary go directly ...
    while (!done && issued < kmax && !(issued > 0 && due(issued + 1))) {
      ++issued;
      if ((st = run.sweep(due(issued)))) return st;
      if (issued % check_every == 0 && (st = all_done(done))) return st;
    }
    if (!done && (st = all_done(done))) return st;
    // ... then whole blocks [re-unitarise, re sweeps] replay one captured graph
    if (!done && issued < kmax && kmax - issued >= re) {
      if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
      FixRun<T> cap = run;
      cap.s = ctx->cap_stream;
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
      mcg_status cst = MCG_OK;
      for (int j = 0; j < re && cst == MCG_OK; j++) cst = cap.sweep(j == 0);
      hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
      if (cst) {
        if (graph) (void)hipGraphDestroy(graph);
        return cst;
      }
      if (e != hipSuccess) return fail(ctx, MCG_EHIP, "graph capture failed: %s", hipGetErrorString(e));
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(ctx, MCG_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
      }
      while (!done && kmax - issued >= re) {
        e = hipGraphLaunch(exec, s);
        if (e != hipSuccess) break;
        issued += re;
        mcg_status q = all_done(done);
        if (q) {
          (void)hipGraphExecDestroy(exec);
          (void)hipGraphDestroy(graph);
          return q;
        }
      }
      (void)hipGraphExecDestroy(exec);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return fail(ctx, MCG_EHIP, "graph launch failed: %s", hipGetErrorString(e));
      run.since_fold = cap.since_fold;  // every replay leaves the ring as the captured block did
    }
    while (!done && issued < kmax) {
      ++issued;
      if ((st = run.sweep(due(issued)))) return st;
      if (issued % check_every == 0 && (st = all_done(done))) return st;
    }
  }
  // final re-unitarisation, R and the stationarity residual
  if ((st = run.fold())) return st;
  HIPCHK(launch_reunit<T>(bs, c12, run.dD, B, total, false, s));
  HIPCHK(launch_rederive<T>(bs, c12, run.dD, B, total, false, s));
  HIPCHK(launch_book<T>(run.dD, B, BOOK_FINAL, s));
  HIPCHK(launch_theta<T>(bs, c12, run.dD, B, total, s));
  HIPCHK(launch_book<T>(run.dD, B, BOOK_THETA, s));
  if (c12)
    for (int b = 0; b < B; b++)
      HIPCHK(launch_gauge_form(geom_of(U[b].d), (const double *)ctx->G12[b].p, G[b].ptr, false, s));
  HIPCHK(hipMemcpyAsync(hS, ctx->states.p, sizeof(FixState) * B, hipMemcpyDeviceToHost, s));
  for (int b = 0; b < B; b++)
    if (opts[b].traj && ctx->traj[b].p)
      HIPCHK(hipMemcpyAsync(opts[b].traj, ctx->traj[b].p, sizeof(double) * (opts[b].max_sweeps + 1),
                            hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  mcg_status worst = MCG_OK;
  for (int b = 0; b < B; b++) {
    mcg_fix_result &r = res[b];
    r.R = hS[b].R_final;
    r.dR = hS[b].dR;
    r.theta = hS[b].theta;
    r.sweeps = hS[b].k;
    r.blocks50 = (hS[b].k + 49) / 50;
    r.status = hS[b].status ? MCG_WNOTCONV : MCG_OK;
    r.pad_ = 0;
    if (r.status) worst = MCG_WNOTCONV;
  }
  return worst;
}

// ------------------------------------------------------- the whole path of a batch
// Sec. II.B for B fields at once: smear every field (n steps), fix the smeared fields together
// from G (batched, graph-captured blocks), fix the original fields together from the smeared
// fields' transforms, then project every fixed field onto Z3 and count its P-vortices.  The
// projections and counts of all fields are queued together and read back with one
// synchronisation; the fixes synchronise once per block of sweeps to read their stop flags.
template <typename T>
static mcg_status precondition_impl(mcg_ctx *ctx, int B, const mcg_field *U, double rho, double eps, int n,
                                    const mcg_fix_opts *opts, mcg_gauge *G, int8_t *const *Z,
                                    mcg_precond_result *res, hipStream_t s) {
  mcg_status st;
  size_t maxbytes = 0;
  for (int b = 0; b < B; b++) maxbytes = std::max(maxbytes, field_bytes(U[b].d, U[b].prec));
  if ((int)ctx->smeared.size() < B) ctx->smeared.resize(B);
  std::vector<mcg_field> S(U, U + B);
  // ROCTX ranges mark each phase on the host: the fixes synchronise on their stop flags, so their
  // ranges follow the device; the smearing steps are only queued within theirs
  if (n > 0) {
    const Range range_("smear");
    for (int b = 0; b < B; b++) {
      if ((st = ensure(ctx, ctx->smeared[b], field_bytes(U[b].d, U[b].prec)))) return st;
      S[b].ptr = ctx->smeared[b].p;
    }
    if (n > 1 && (st = ensure(ctx, ctx->tmpfield, maxbytes))) return st;
    for (int b = 0; b < B; b++) {
      const Geom g = geom_of(U[b].d);
      const void *src = U[b].ptr;
      for (int k = 0; k < n; k++) {  // ping-pong so that the last step writes S[b]
        void *dst = ((n - 1 - k) % 2 == 0) ? S[b].ptr : ctx->tmpfield.p;
        HIPCHK(launch_smear_step<T>(g, src, dst, rho, eps, s));
        src = dst;
      }
    }
  }
  std::vector<mcg_fix_result> rs(B), rf(B);
  mcg_status s1, s2;
  {
    const Range range_("fix smeared fields");
    s1 = fix_impl<T>(ctx, B, S.data(), G, opts, rs.data(), s, true);
  }
  if (s1 < 0) return s1;
  {
    const Range range_("fix carried back");
    s2 = fix_impl<T>(ctx, B, U, G, opts, rf.data(), s, true);
  }
  if (s2 < 0) return s2;
  // every field's projection and count, then one copy back
  const Range range_("project and count");
  std::vector<size_t> p0(B + 1, 0);
  for (int b = 0; b < B; b++) p0[b + 1] = p0[b] + (size_t)field_blocks256(geom_of(U[b].d));
  if ((st = ensure(ctx, ctx->pc_part, sizeof(double) * (p0[B] + B))) ||
      (st = ensure(ctx, ctx->pc_counts, sizeof(unsigned long long) * 12 * B)) ||
      (st = ensure_pinned(ctx, sizeof(double) * B + sizeof(unsigned long long) * 12 * B)))
    return st;
  double *part = (double *)ctx->pc_part.p, *mins = part + p0[B];
  unsigned long long *counts = (unsigned long long *)ctx->pc_counts.p;
  HIPCHK(launch_zero((double *)counts, 12 * B, s));  // a fill kernel, not a memset: graph-safe
  for (int b = 0; b < B; b++) {
    const Geom g = geom_of(U[b].d);
    HIPCHK(launch_center_project<T>(g, U[b].ptr, G[b].ptr, Z[b], part + p0[b], mins + b, s));
    HIPCHK(launch_count_vortices(g, Z[b], counts + 12 * b, s));
  }
  double *hmin = (double *)ctx->h_pinned;
  unsigned long long *hcnt = (unsigned long long *)(hmin + B);
  HIPCHK(hipMemcpyAsync(hmin, mins, sizeof(double) * B, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hcnt, counts, sizeof(unsigned long long) * 12 * B, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int b = 0; b < B; b++) {
    mcg_precond_result &r = res[b];
    memset(&r, 0, sizeof r);
    r.smeared = rs[b];
    r.fixed = rf[b];
    r.min_margin = hmin[b];
    const unsigned long long *c = hcnt + 12 * b;
    for (int p = 0; p < 6; p++) {
      r.per_plane[p] = (int64_t)(c[2 * p] + c[2 * p + 1]);
      r.per_charge[0] += (int64_t)c[2 * p];
      r.per_charge[1] += (int64_t)c[2 * p + 1];
      r.vortices += r.per_plane[p];
    }
  }
  return s1 == MCG_WNOTCONV || s2 == MCG_WNOTCONV ? MCG_WNOTCONV : MCG_OK;
}

// ----------------------------------------------------------------- backward
// L = R(S_n(U)^G*): forward with a checkpoint every c steps, seed grad_S_n,
// then per segment (last first) recompute the c fields from the checkpoint
// and apply the step adjoints in reverse.  Partial sums of L, dL/drho and
// dL/deps stay on the device and are reduced there at the end in a fixed
// order; three scalars and a flag come back.
template <typename T>
mcg_status backward_impl(mcg_ctx *ctx, const mcg_field *U, double rho, double eps, int n, const mcg_gauge *Gstar,
                         int ckpt_every, mcg_field *gradU, double *loss, double *dRho, double *dEps,
                         hipStream_t s) {
  const Geom g = geom_of(U->d);
  const size_t fb = field_bytes(U->d, U->prec);
  const int c = (ckpt_every <= 0 || ckpt_every > n) ? std::max(n, 1) : ckpt_every;
  const int nck = n > 0 ? (n + c - 1) / c : 0;
  // fields: nck checkpoints, c-1 segment slots, 2 forward temporaries, 2 gradients, grad_C, the
  // staple sums (Cp, and Cr for eps != 1) of the first c-1 steps of a segment, and those of every
  // segment's last step, which the forward pass stores.  If that does not fit, the sums are not
  // kept and the adjoint's first pass forms the staples itself (the same results, more time).
  const int ncs = eps == 1.0 ? 1 : 2;
  const size_t nbase = (size_t)nck + (size_t)(c - 1) + 5;
  const size_t nfields = nbase + (size_t)(c - 1) * ncs + (size_t)nck * ncs;
  mcg_status st;
  bool stored = true;
  {
    const std::string err = ctx->err;
    if (ensure(ctx, ctx->ckpt, fb * nfields) != MCG_OK) {
      ctx->err = err;
      stored = false;
      if ((st = ensure(ctx, ctx->ckpt, fb * nbase))) return st;
    }
  }
  const int nb_seed = field_blocks256(g), nb_step = adjoint_blocks(g);
  const size_t nparts = (size_t)nb_seed + (size_t)std::max(n, 1) * 3 * nb_step;
  if ((st = ensure(ctx, ctx->bw_part, sizeof(double) * nparts + 64))) return st;
  char *base = (char *)ctx->ckpt.p;
  auto slot = [&](size_t i) { return (void *)(base + i * fb); };
  void *tmp0 = slot(nck + c - 1), *tmp1 = slot(nck + c), *gA = slot(nck + c + 1), *gB = slot(nck + c + 2),
       *gC = slot(nck + c + 3);
  auto csum = [&](int j) -> void * {  // step j < c-1 of a segment
    return stored ? slot((size_t)nck + c + 4 + (size_t)j * ncs) : nullptr;
  };
  auto clast = [&](int seg) -> void * {  // a segment's last step
    return stored ? slot((size_t)nck + c + 4 + (size_t)(c - 1) * ncs + (size_t)seg * ncs) : nullptr;
  };
  double *part = (double *)ctx->bw_part.p;
  double *red = part + nparts;      // the three reduced scalars ...
  int *flag = (int *)(red + 3);     // ... and the adjoint's range flag, copied back together
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), s));
  HIPCHK(hipMemsetAsync(part, 0, sizeof(double) * nparts, s));

  // forward, keeping every c-th field and the staple sums of each segment's last step; the last
  // segment's fields and staple sums go straight to the slots its recomputation would fill, so the
  // adjoint starts on it without recomputing
  const void *cur = U->ptr;
  const int k0_last = (nck - 1) * c;  // first step of the last segment
  {
    const Range range_("backward: forward smearing");
    for (int k = 0; k < n; k++) {
      if (k % c == 0) HIPCHK(hipMemcpyAsync(slot(k / c), cur, fb, hipMemcpyDeviceToDevice, s));
      const bool in_last = k >= k0_last && k < n - 1;
      void *nxt = in_last ? slot((size_t)nck + (k - k0_last)) : (cur == tmp0 ? tmp1 : tmp0);
      const bool last = k % c == c - 1 || k == n - 1;
      void *cs = last ? clast(k / c) : in_last ? csum(k - k0_last) : nullptr;
      HIPCHK(launch_smear_step<T>(g, cur, nxt, rho, eps, s, cs));
      cur = nxt;
    }
  }
  HIPCHK(launch_loss_seed<T>(g, cur, Gstar->ptr, gA, part, s));
  void *gin = gA, *gout = gB;
  const Range range_("backward: adjoint segments");
  for (int seg = nck - 1; seg >= 0; seg--) {
    const int k0 = seg * c, len = std::min(c, n - k0);
    // the segment's fields again from its checkpoint, keeping the staple sums that each smearing
    // step forms (the last step's were kept by the forward pass), which the first pass of the
    // adjoint reads
    std::vector<const void *> fields(len);
    fields[0] = slot(seg);
    for (int j = 1; j < len; j++) {
      void *dst = slot(nck + j - 1);
      if (seg < nck - 1) HIPCHK(launch_smear_step<T>(g, fields[j - 1], dst, rho, eps, s, csum(j - 1)));
      fields[j] = dst;
    }
    for (int j = len - 1; j >= 0; j--) {
      const int k = k0 + j;
      double *p = part + nb_seed + (size_t)k * 3 * nb_step;
      HIPCHK(launch_step_adjoint<T>(g, fields[j], j == len - 1 ? clast(seg) : csum(j), gin, gout, gC, rho, eps,
                                    p, flag, s));
      std::swap(gin, gout);
    }
  }
  HIPCHK(hipMemcpyAsync(gradU->ptr, gin, fb, hipMemcpyDeviceToDevice, s));
  HIPCHK(launch_reduce_parts(part, nb_seed, n, nb_step, red, s));
  double h[4];
  HIPCHK(hipMemcpyAsync(h, red, 3 * sizeof(double) + sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int hflag;
  std::memcpy(&hflag, &h[3], sizeof(int));
  if (hflag)
    return fail(ctx, MCG_EINPUT, "a smearing exponent exceeds the range of the adjoint's series "
                                 "(spectral radius of C U^dag above 4)");
  *loss = h[0] / (9.0 * (double)(4 * g.V));
  *dRho = h[1];
  *dEps = h[2];
  return MCG_OK;
}

}  // namespace

// ======================================================================= ABI
extern "C" {

const char *mcg_status_string(mcg_status s) {
  switch (s) {
  case MCG_OK: return "ok";
  case MCG_WNOTCONV: return "not converged within max_sweeps";
  case MCG_EINVAL: return "invalid argument";
  case MCG_ENOMEM: return "out of device memory";
  case MCG_EHIP: return "HIP runtime error";
  case MCG_EINPUT: return "input outside the supported range";
  default: return "unknown status";
  }
}

const char *mcg_last_error(const mcg_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

mcg_status mcg_create(mcg_ctx **out, int32_t device) {
  if (!out) return MCG_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return MCG_EHIP;
  }
  if (hipSetDevice(device) != hipSuccess) return MCG_EHIP;
  mcg_ctx *ctx = new mcg_ctx();
  ctx->device = device;
  // the allocation-free entry point's scratch on this device; without it only that call fails
  const hipError_t e = noalloc_scratch(device, &ctx->noalloc);
  if (e != hipSuccess) ctx->noalloc_err = hipGetErrorString(e);
  *out = ctx;
  return MCG_OK;
}

mcg_status mcg_destroy(mcg_ctx *ctx) {
  if (!ctx) return MCG_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  DevBuf *bufs[] = {&ctx->part, &ctx->scalars, &ctx->counts, &ctx->states, &ctx->desc, &ctx->tmpfield,
                    &ctx->grad_a, &ctx->grad_b, &ctx->gC, &ctx->ckpt, &ctx->bw_part, &ctx->w12, &ctx->g12,
                    &ctx->line_a, &ctx->line_b, &ctx->wl_part, &ctx->wl_res, &ctx->wl_img};
  for (DevBuf *b : bufs)
    if (b->p) (void)hipFree(b->p);
  for (DevBuf *b : {&ctx->pc_part, &ctx->pc_counts})
    if (b->p) (void)hipFree(b->p);
  for (auto *v : {&ctx->W, &ctx->G12, &ctx->fpart, &ctx->traj, &ctx->gring, &ctx->smeared})
    for (DevBuf &b : *v)
      if (b.p) (void)hipFree(b.p);
  if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
  return MCG_OK;
}

size_t mcg_field_bytes(mcg_dims d, int32_t prec) {
  if (prec != MCG_F64 && prec != MCG_F32) return 0;
  return field_bytes(d, prec);
}

size_t mcg_gauge_bytes(mcg_dims d) {
  if (!dims_valid(d)) return 0;
  return (size_t)d.L[0] * d.L[1] * d.L[2] * d.L[3] * 9 * 2 * sizeof(double);
}

mcg_status mcg_pack_links(mcg_ctx *ctx, const void *src, int32_t src_prec, mcg_field *dst, void *stream) {
  if (!ctx) return MCG_EINVAL;
  mcg_status st = check_field(ctx, dst, "dst");
  if (st) return st;
  if (!src || (src_prec != MCG_F64 && src_prec != MCG_F32)) return fail(ctx, MCG_EINVAL, "bad source");
  const Geom g = geom_of(dst->d);
  hipStream_t s = (hipStream_t)stream;
  if (src_prec == MCG_F64 && dst->prec == MCG_F64) HIPCHK((launch_pack_links<double, double>(g, src, dst->ptr, s)));
  if (src_prec == MCG_F64 && dst->prec == MCG_F32) HIPCHK((launch_pack_links<double, float>(g, src, dst->ptr, s)));
  if (src_prec == MCG_F32 && dst->prec == MCG_F32) HIPCHK((launch_pack_links<float, float>(g, src, dst->ptr, s)));
  if (src_prec == MCG_F32 && dst->prec == MCG_F64) HIPCHK((launch_pack_links<float, double>(g, src, dst->ptr, s)));
  return MCG_OK;
}

mcg_status mcg_unpack_links(mcg_ctx *ctx, const mcg_field *src, void *dst, int32_t dst_prec, void *stream) {
  if (!ctx) return MCG_EINVAL;
  mcg_status st = check_field(ctx, src, "src");
  if (st) return st;
  if (!dst || (dst_prec != MCG_F64 && dst_prec != MCG_F32)) return fail(ctx, MCG_EINVAL, "bad destination");
  const Geom g = geom_of(src->d);
  hipStream_t s = (hipStream_t)stream;
  if (src->prec == MCG_F64 && dst_prec == MCG_F64) HIPCHK((launch_unpack_links<double, double>(g, src->ptr, dst, s)));
  if (src->prec == MCG_F64 && dst_prec == MCG_F32) HIPCHK((launch_unpack_links<double, float>(g, src->ptr, dst, s)));
  if (src->prec == MCG_F32 && dst_prec == MCG_F32) HIPCHK((launch_unpack_links<float, float>(g, src->ptr, dst, s)));
  if (src->prec == MCG_F32 && dst_prec == MCG_F64) HIPCHK((launch_unpack_links<float, double>(g, src->ptr, dst, s)));
  return MCG_OK;
}

mcg_status mcg_pack_gauge(mcg_ctx *ctx, const double *src, mcg_gauge *dst, void *stream) {
  if (!ctx) return MCG_EINVAL;
  if (!src || !dst || !dst->ptr || !dims_valid(dst->d)) return fail(ctx, MCG_EINVAL, "bad gauge arguments");
  HIPCHK(launch_pack_gauge(geom_of(dst->d), src, dst->ptr, (hipStream_t)stream));
  return MCG_OK;
}

mcg_status mcg_unpack_gauge(mcg_ctx *ctx, const mcg_gauge *src, double *dst, void *stream) {
  if (!ctx) return MCG_EINVAL;
  if (!src || !dst || !src->ptr || !dims_valid(src->d)) return fail(ctx, MCG_EINVAL, "bad gauge arguments");
  HIPCHK(launch_unpack_gauge(geom_of(src->d), src->ptr, dst, (hipStream_t)stream));
  return MCG_OK;
}

mcg_status mcg_gauge_identity(mcg_ctx *ctx, mcg_gauge *G, void *stream) {
  if (!ctx) return MCG_EINVAL;
  if (!G || !G->ptr || !dims_valid(G->d)) return fail(ctx, MCG_EINVAL, "bad gauge argument");
  HIPCHK(launch_gauge_identity(geom_of(G->d), G->ptr, (hipStream_t)stream));
  return MCG_OK;
}

mcg_status mcg_gauge_reunit(mcg_ctx *ctx, mcg_gauge *G, void *stream) {
  if (!ctx) return MCG_EINVAL;
  if (!G || !G->ptr || !dims_valid(G->d)) return fail(ctx, MCG_EINVAL, "bad gauge argument");
  HIPCHK(launch_gauge_reunit(geom_of(G->d), G->ptr, (hipStream_t)stream));
  return MCG_OK;
}

mcg_status mcg_unitarity(mcg_ctx *ctx, const mcg_field *U, const mcg_gauge *G, double *dev_U, double *dev_G,
                         void *stream) {
  if (!ctx) return MCG_EINVAL;
  mcg_status st;
  if (!U && !G) return fail(ctx, MCG_EINVAL, "U and G are both NULL");
  if (U && (st = check_field(ctx, U, "U"))) return st;
  if (G && !U && !dims_valid(G->d)) return fail(ctx, MCG_EINVAL, "G: bad extents");
  if (G && (st = check_gauge(ctx, G, U ? U->d : G->d, "G"))) return st;
  return unitarity(ctx, U, G, dev_U, dev_G, (hipStream_t)stream);
}

mcg_status mcg_smear(mcg_ctx *ctx, const mcg_field *U, mcg_field *out, double rho, double eps, int32_t n,
                     void *stream) {
  const Range range_("mcg_smear");
  if (!ctx) return MCG_EINVAL;
  mcg_status st;
  if ((st = check_field(ctx, U, "U")) || (st = check_field(ctx, out, "out"))) return st;
  if (!same_dims(U->d, out->d) || U->prec != out->prec)
    return fail(ctx, MCG_EINVAL, "U and out differ in extents or precision");
  if (U->ptr == out->ptr) return fail(ctx, MCG_EINVAL, "U and out must not alias");
  if (n < 0 || std::isnan(rho) || std::isnan(eps)) return fail(ctx, MCG_EINVAL, "bad smearing parameters");
  hipStream_t s = (hipStream_t)stream;
  if ((st = check_inputs(ctx, U, nullptr, s))) return st;
  const size_t bytes = field_bytes(U->d, U->prec);
  if (n == 0) {
    HIPCHK(hipMemcpyAsync(out->ptr, U->ptr, bytes, hipMemcpyDeviceToDevice, s));
    return MCG_OK;
  }
  if (n > 1 && (st = ensure(ctx, ctx->tmpfield, bytes))) return st;
  const Geom g = geom_of(U->d);
  // ping-pong so that the last step writes `out`
  const void *src = U->ptr;
  for (int k = 0; k < n; k++) {
    void *dst = ((n - 1 - k) % 2 == 0) ? out->ptr : ctx->tmpfield.p;
    if (U->prec == MCG_F64)
      HIPCHK(launch_smear_step<double>(g, src, dst, rho, eps, s));
    else
      HIPCHK(launch_smear_step<float>(g, src, dst, rho, eps, s));
    src = dst;
  }
  return MCG_OK;
}

mcg_status mcg_apply_gauge(mcg_ctx *ctx, const mcg_field *U, const mcg_gauge *G, mcg_field *out,
                           void *stream) {
  if (!ctx) return MCG_EINVAL;
  mcg_status st;
  if ((st = check_field(ctx, U, "U")) || (st = check_field(ctx, out, "out")) ||
      (st = check_gauge(ctx, G, U->d, "G")))
    return st;
  if (!same_dims(U->d, out->d) || U->prec != out->prec)
    return fail(ctx, MCG_EINVAL, "U and out differ in extents or precision");
  if ((st = check_inputs(ctx, U, G, (hipStream_t)stream))) return st;
  const Geom g = geom_of(U->d);
  if (U->prec == MCG_F64)
    HIPCHK(launch_apply_gauge<double>(g, U->ptr, G->ptr, out->ptr, (hipStream_t)stream));
  else
    HIPCHK(launch_apply_gauge<float>(g, U->ptr, G->ptr, out->ptr, (hipStream_t)stream));
  return MCG_OK;
}

static mcg_status field_scalar(mcg_ctx *ctx, const mcg_field *U, double *out, void *stream, int what) {
  if (!ctx) return MCG_EINVAL;
  mcg_status st;
  if ((st = check_field(ctx, U, "U"))) return st;
  if (!out) return fail(ctx, MCG_EINVAL, "NULL output");
  const Geom g = geom_of(U->d);
  if ((st = ensure(ctx, ctx->part, sizeof(double) * field_blocks256(g))) ||
      (st = ensure(ctx, ctx->scalars, 64)))
    return st;
  hipStream_t s = (hipStream_t)stream;
  double *dres = (double *)ctx->scalars.p;
  if (what == 0) {
    if (U->prec == MCG_F64) HIPCHK(launch_functional<double>(g, U->ptr, (double *)ctx->part.p, dres, s));
    else HIPCHK(launch_functional<float>(g, U->ptr, (double *)ctx->part.p, dres, s));
  } else {
    if (U->prec == MCG_F64) HIPCHK(launch_plaquette<double>(g, U->ptr, (double *)ctx->part.p, dres, s));
    else HIPCHK(launch_plaquette<float>(g, U->ptr, (double *)ctx->part.p, dres, s));
  }
  HIPCHK(hipMemcpyAsync(out, dres, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return MCG_OK;
}

mcg_status mcg_functional(mcg_ctx *ctx, const mcg_field *U, double *R, void *stream) {
  return field_scalar(ctx, U, R, stream, 0);
}

mcg_status mcg_plaquette(mcg_ctx *ctx, const mcg_field *U, double *P, void *stream) {
  return field_scalar(ctx, U, P, stream, 1);
}

}  // extern "C"

template <typename T>
static mcg_status theta_impl(mcg_ctx *ctx, const mcg_field *W, double *theta, hipStream_t s) {
  const Geom g = geom_of(W->d);
  const int bs = 256, nb = nblocks(g, bs);
  mcg_status st;
  if ((st = ensure(ctx, ctx->part, sizeof(double) * nb)) || (st = ensure(ctx, ctx->states, sizeof(FixState))) ||
      (st = ensure(ctx, ctx->desc, sizeof(LatDesc<T>))) ||
      (st = ensure_pinned(ctx, sizeof(LatDesc<T>) + sizeof(FixState))))
    return st;
  LatDesc<T> *hD = (LatDesc<T> *)ctx->h_pinned;
  memset(hD, 0, sizeof(LatDesc<T>));
  hD->g = g;
  hD->blk0 = 0;
  hD->nblk = nb;
  hD->W = (V2<T> *)W->ptr;
  hD->st = (FixState *)ctx->states.p;
  hD->part = (double *)ctx->part.p;
  HIPCHK(hipMemcpyAsync(ctx->desc.p, hD, sizeof(LatDesc<T>), hipMemcpyHostToDevice, s));
  HIPCHK(launch_theta<T>(bs, false, ctx->desc.p, 1, nb, s));
  HIPCHK(launch_book<T>(ctx->desc.p, 1, BOOK_THETA, s));
  FixState *hS = (FixState *)(hD + 1);
  HIPCHK(hipMemcpyAsync(hS, ctx->states.p, sizeof(FixState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *theta = hS->theta;
  return MCG_OK;
}

extern "C" {


mcg_status mcg_theta(mcg_ctx *ctx, const mcg_field *W, double *theta, void *stream) {
  if (!ctx) return MCG_EINVAL;
  mcg_status st;
  if ((st = check_field(ctx, W, "W"))) return st;
  if (!theta) return fail(ctx, MCG_EINVAL, "NULL output");
  return W->prec == MCG_F64 ? theta_impl<double>(ctx, W, theta, (hipStream_t)stream)
                            : theta_impl<float>(ctx, W, theta, (hipStream_t)stream);
}

}  // extern "C"

// parity >= 0: one half-sweep of that parity on the caller's (full-form)
// fields.  parity < 0: n sweeps (0, 1, 0, 1, ...) in the context's storage
// form; in the two-row form W and G are converted into context scratch,
// swept, and converted back.  ms: the summed duration of the half-sweep
// launches alone (HIP events around each sweep's pair; synchronises).
template <typename T>
static mcg_status halfsweep_impl(mcg_ctx *ctx, mcg_field *W, mcg_gauge *G, int parity, double omega,
                                 hipStream_t s, int n = 1, double *ms = nullptr) {
  const Geom g = geom_of(W->d);
  const bool c12 = parity < 0 && ctx->c12;
  const int variant = (ctx->hits > 1 || ctx->exact) ? 2 : ctx->variant[W->prec][c12],
            nb = nblocks(g, variant_block(variant));
  mcg_status st;
  if ((st = ensure(ctx, ctx->desc, sizeof(LatDesc<T>))) || (st = ensure_pinned(ctx, sizeof(LatDesc<T>))))
    return st;
  if (c12 && ((st = ensure(ctx, ctx->w12, work_field_bytes(W->d, W->prec, true))) ||
              (st = ensure(ctx, ctx->g12, gauge_form_bytes(W->d, true)))))
    return st;
  bool ring = parity < 0 && W->prec == MCG_F32 && ctx->defer_g;
  bool hand = parity < 0 && W->prec == MCG_F64 && c12 && ctx->paired == 2;
  if (ring || hand) {
    if (ctx->gring.empty()) ctx->gring.resize(1);
    if (ring) ring = reserve_rings(ctx, 1, W, GRING_SWEEPS);
    if (hand) hand = reserve_rings(ctx, 1, W, 1);
  }
  // the pinned staging area may still feed an earlier copy on this stream
  HIPCHK(hipStreamSynchronize(s));
  LatDesc<T> *hD = (LatDesc<T> *)ctx->h_pinned;
  memset(hD, 0, sizeof(LatDesc<T>));
  hD->gring = (ring || hand) ? (V2<T> *)ctx->gring[0].p : nullptr;
  hD->g = g;
  hD->nblk = nb;
  hD->nslab = 1;
  hD->W = c12 ? (V2<T> *)ctx->w12.p : (V2<T> *)W->ptr;
  hD->G = c12 ? (double2 *)ctx->g12.p : (double2 *)G->ptr;
  FixRun<T> run{ctx, s, 1, variant, variant_block(variant), nb, c12, ctx->desc.p, omega};
  run.gated = false;
  run.hits = ctx->hits;
  run.exact = ctx->exact ? 1 : 0;
  run.order = ctx->order;
  run.C = ring ? GRING_SWEEPS : 0;
  run.paired = ctx->paired != 0;
  run.hand = hand;
  run.stateful = false;
  if (parity < 0) run.nslab = plan_slabs(hD, 1, ctx->nslab, variant_block(variant), run.grid);
  HIPCHK(hipMemcpyAsync(ctx->desc.p, hD, sizeof(LatDesc<T>), hipMemcpyHostToDevice, s));
  if (parity >= 0) {
    HIPCHK(launch_halfsweep<T>(variant, false, ctx->desc.p, 1, nb, parity, omega, false, false, s, -1, ctx->hits,
                               ctx->exact ? 1 : 0, tile_order(ctx->order, parity)));
    return MCG_OK;
  }
  if (c12) {
    HIPCHK(launch_links_form<T>(g, W->ptr, ctx->w12.p, true, s));
    HIPCHK(launch_gauge_form(g, G->ptr, (double *)ctx->g12.p, true, s));
  }
  if (!ms) {
    for (int k = 0; k < n; k++)
      if ((st = run.halfsweeps(false)) || (st = run.advance())) return st;
  } else {
    std::vector<hipEvent_t> ev((size_t)2 * n, nullptr);
    hipError_t e = hipSuccess;
    st = MCG_OK;
    for (int k = 0; k < n && e == hipSuccess && st == MCG_OK; k++) {
      e = hipEventCreate(&ev[2 * k]);
      if (e == hipSuccess) e = hipEventCreate(&ev[2 * k + 1]);
      if (e == hipSuccess) e = hipEventRecord(ev[2 * k], s);
      if (e == hipSuccess) st = run.halfsweeps(false);
      if (e == hipSuccess && st == MCG_OK) e = hipEventRecord(ev[2 * k + 1], s);
      if (e == hipSuccess && st == MCG_OK) st = run.advance();
    }
    if (e == hipSuccess && st == MCG_OK) e = hipEventSynchronize(ev[2 * n - 1]);
    double total = 0.0;
    for (int k = 0; k < n && e == hipSuccess && st == MCG_OK; k++) {
      float t = 0.f;
      e = hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]);
      total += t;
    }
    for (hipEvent_t x : ev)
      if (x) (void)hipEventDestroy(x);
    if (st) return st;
    if (e != hipSuccess) return fail(ctx, MCG_EHIP, "timing events: %s", hipGetErrorString(e));
    *ms = total;
  }
  if ((st = run.fold())) return st;
  if (c12) {
    HIPCHK(launch_links_form<T>(g, ctx->w12.p, W->ptr, false, s));
    HIPCHK(launch_gauge_form(g, (const double *)ctx->g12.p, G->ptr, false, s));
  }
  return MCG_OK;
}

extern "C" {

mcg_status mcg_halfsweep(mcg_ctx *ctx, mcg_field *W, mcg_gauge *G, int32_t parity, double omega, void *stream) {
  if (!ctx) return MCG_EINVAL;
  mcg_status st;
  if ((st = check_field(ctx, W, "W")) || (st = check_gauge(ctx, G, W->d, "G"))) return st;
  if (parity != 0 && parity != 1) return fail(ctx, MCG_EINVAL, "parity must be 0 or 1");
  if (!(omega >= 0.0 && omega <= 2.0)) return fail(ctx, MCG_EINVAL, "omega must lie in [0, 2]");
  return W->prec == MCG_F64 ? halfsweep_impl<double>(ctx, W, G, parity, omega, (hipStream_t)stream)
                            : halfsweep_impl<float>(ctx, W, G, parity, omega, (hipStream_t)stream);
}

}  // extern "C"

// ---------------------------------------------------------------- autotuner
template <typename T>
static mcg_status autotune_impl(mcg_ctx *ctx, int B, const mcg_field *U, int32_t *best, double *ms, hipStream_t s) {
  const bool c12 = ctx->c12;
  const int prec = U[0].prec;
  // time the half-sweep the fixes run: with the transform ring (FP32) g goes to ring slots 0 and 1
  bool ring = prec == MCG_F32 && ctx->defer_g;
  mcg_status st;
  if ((int)ctx->W.size() < B) {
    ctx->W.resize(B);
    ctx->G12.resize(B);
    ctx->fpart.resize(B);
    ctx->traj.resize(B);
    ctx->gring.resize(B);
  }
  if ((st = ensure(ctx, ctx->desc, sizeof(LatDesc<T>) * B)) || (st = ensure_pinned(ctx, sizeof(LatDesc<T>) * B)))
    return st;
  // each field's working copy in the storage form and an identity transform, in the fix's scratch;
  // every buffer is reserved before the first kernel is queued (a grown buffer is freed and
  // reallocated, which must not happen under queued work)
  size_t gfull = 0;
  for (int b = 0; b < B; b++) {
    if ((st = ensure(ctx, ctx->W[b], work_field_bytes(U[b].d, prec, c12))) ||
        (st = ensure(ctx, ctx->G12[b], gauge_form_bytes(U[b].d, c12))))
      return st;
    gfull = std::max(gfull, mcg_gauge_bytes(U[b].d));
  }
  if (c12 && (st = ensure(ctx, ctx->grad_a, gfull))) return st;
  if (ring) ring = reserve_rings(ctx, B, U, 1);
  bool hand = prec == MCG_F64 && c12 && ctx->paired == 2;  // FP64 paired sweeps: the even g's handoff slot
  if (hand) hand = reserve_rings(ctx, B, U, 1);
  const bool pr = (ring || hand) && c12 && ctx->paired != 0;  // paired sweeps, as the fixes run them
  for (int b = 0; b < B; b++) {
    const Geom g = geom_of(U[b].d);
    if (c12) {
      HIPCHK(launch_gauge_identity(g, (double *)ctx->grad_a.p, s));
      HIPCHK(launch_gauge_form(g, (const double *)ctx->grad_a.p, (double *)ctx->G12[b].p, true, s));
      HIPCHK(launch_links_form<T>(g, U[b].ptr, ctx->W[b].p, true, s));
    } else {
      HIPCHK(launch_gauge_identity(g, (double *)ctx->G12[b].p, s));
      HIPCHK(hipMemcpyAsync(ctx->W[b].p, U[b].ptr, field_bytes(U[b].d, prec), hipMemcpyDeviceToDevice, s));
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  LatDesc<T> *hD = (LatDesc<T> *)ctx->h_pinned;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // Three passes over the variants, interleaved so that a slow moment of the device does not
  // count against one variant only; each variant is ranked by the median of its three timings.
  // Every launch covers the whole batch, as the fix's half-sweeps do.
  constexpr int PASSES = 3;
  double per[PASSES][NUM_VARIANTS] = {};
  mcg_status rc = MCG_OK;
  for (int pass = 0; pass < PASSES && rc == MCG_OK; pass++)
    for (int v = 0; v < NUM_VARIANTS && rc == MCG_OK; v++) {
      int total = 0;
      for (int b = 0; b < B; b++) {
        LatDesc<T> d;
        memset(&d, 0, sizeof d);
        d.g = geom_of(U[b].d);
        d.blk0 = total;
        d.nblk = nblocks(d.g, variant_block(v));
        d.nslab = 1;
        d.W = (V2<T> *)ctx->W[b].p;
        d.G = (double2 *)ctx->G12[b].p;
        d.gring = (ring || hand) ? (V2<T> *)ctx->gring[b].p : nullptr;
        hD[b] = d;
        total += d.nblk;
      }
      hipError_t e = hipMemcpyAsync(ctx->desc.p, hD, sizeof(LatDesc<T>) * B, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      for (int k = 0; k < 4 && e == hipSuccess; k++)
        e = launch_halfsweep<T>(v, c12, ctx->desc.p, B, total, k & 1, 1.7, false, false, s, -1, 1, 0,
                                tile_order(ctx->order, k & 1), ring ? (k & 1) : -1, pr ? 0 : -1,
                                pr && !(k & 1) ? 1 : 0);
      if (e == hipSuccess) e = hipEventRecord(e0, s);
      const int reps = 8;
      for (int k = 0; k < reps && e == hipSuccess; k++)
        e = launch_halfsweep<T>(v, c12, ctx->desc.p, B, total, k & 1, 1.7, false, false, s, -1, 1, 0,
                                tile_order(ctx->order, k & 1), ring ? (k & 1) : -1, pr ? 0 : -1,
                                pr && !(k & 1) ? 1 : 0);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float t = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      if (e != hipSuccess) {
        rc = fail(ctx, MCG_EHIP, "autotune variant %d: %s", v, hipGetErrorString(e));
        break;
      }
      per[pass][v] = (double)t / reps;
    }
  double tbest = 1e300;
  int vbest = ctx->variant[prec][c12];
  for (int v = 0; v < NUM_VARIANTS && rc == MCG_OK; v++) {
    double a = per[0][v], b = per[1][v], c = per[2][v];
    const double med = std::max(std::min(a, b), std::min(std::max(a, b), c));
    if (ms) ms[v] = med;
    if (med < tbest) {
      tbest = med;
      vbest = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  ctx->variant[prec][c12] = vbest;
  if (best) *best = vbest;
  return MCG_OK;
}

// Launch variant and schedule of the fixing sweeps, tuned on the batch itself: whole sweeps (both
// half-sweeps) over all B fields, on working copies of U with G = 1, in the context's storage form
// and with the transform ring (one sweep's slots) or FP64 handoff slot that fixes would use.  The
// search runs in three stages -- every variant under the context's current schedule, every
// schedule (tile order x paired sweeps x slabs) under the best variant, every variant under the
// best schedule -- each stage in three interleaved passes, points ranked by their median.  The
// schedule changes only the order in which independent sites are visited and where g waits, so
// every point gives the same bits.
template <typename T>
static mcg_status tune_impl(mcg_ctx *ctx, int B, const mcg_field *U, mcg_tune_choice *out, hipStream_t s) {
  const bool c12 = ctx->c12;
  const int prec = U[0].prec;
  if (ctx->hits > 1 || ctx->exact)
    return fail(ctx, MCG_EINVAL, "mcg_tune_batch: re-linearisation hits and exact steps run one fixed variant");
  bool ring = prec == MCG_F32 && ctx->defer_g;
  mcg_status st;
  if ((int)ctx->W.size() < B) {
    ctx->W.resize(B);
    ctx->G12.resize(B);
    ctx->fpart.resize(B);
    ctx->traj.resize(B);
    ctx->gring.resize(B);
  }
  if ((st = ensure(ctx, ctx->desc, sizeof(LatDesc<T>) * B)) || (st = ensure_pinned(ctx, sizeof(LatDesc<T>) * B)))
    return st;
  size_t gfull = 0;
  for (int b = 0; b < B; b++) {
    if ((st = ensure(ctx, ctx->W[b], work_field_bytes(U[b].d, prec, c12))) ||
        (st = ensure(ctx, ctx->G12[b], gauge_form_bytes(U[b].d, c12))))
      return st;
    gfull = std::max(gfull, mcg_gauge_bytes(U[b].d));
  }
  if (c12 && (st = ensure(ctx, ctx->grad_a, gfull))) return st;
  if (ring) ring = reserve_rings(ctx, B, U, 1);
  // FP64 paired sweeps need the handoff slot; without it (memory) they are not tried
  bool hand = prec == MCG_F64 && c12;
  if (hand) hand = reserve_rings(ctx, B, U, 1);
  for (int b = 0; b < B; b++) {
    const Geom g = geom_of(U[b].d);
    if (c12) {
      HIPCHK(launch_gauge_identity(g, (double *)ctx->grad_a.p, s));
      HIPCHK(launch_gauge_form(g, (const double *)ctx->grad_a.p, (double *)ctx->G12[b].p, true, s));
      HIPCHK(launch_links_form<T>(g, U[b].ptr, ctx->W[b].p, true, s));
    } else {
      HIPCHK(launch_gauge_identity(g, (double *)ctx->G12[b].p, s));
      HIPCHK(hipMemcpyAsync(ctx->W[b].p, U[b].ptr, field_bytes(U[b].d, prec), hipMemcpyDeviceToDevice, s));
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  LatDesc<T> *hD = (LatDesc<T> *)ctx->h_pinned;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // one point: WARM sweeps, then REPS timed sweeps; ms per sweep
  constexpr int WARM = 1, REPS = 4;
  auto time_point = [&](const Sched &p, double &ms) -> mcg_status {
    const int bs = variant_block(p.variant);
    int total = 0;
    for (int b = 0; b < B; b++) {
      LatDesc<T> d;
      memset(&d, 0, sizeof d);
      d.g = geom_of(U[b].d);
      d.blk0 = total;
      d.nblk = nblocks(d.g, bs);
      d.nslab = 1;
      d.W = (V2<T> *)ctx->W[b].p;
      d.G = (double2 *)ctx->G12[b].p;
      d.gring = (ring || hand) ? (V2<T> *)ctx->gring[b].p : nullptr;
      hD[b] = d;
      total += d.nblk;
    }
    FixRun<T> run{ctx, s, B, p.variant, bs, total, c12, ctx->desc.p, 1.7};
    run.gated = false;
    run.stateful = false;
    run.order = p.order;
    run.C = ring ? 1 : 0;  // g to ring slots 0 and 1; no fold is timed
    run.paired = p.paired != 0;
    run.hand = hand && p.paired == 2;
    run.nslab = plan_slabs(hD, B, p.nslab, bs, run.grid);
    HIPCHK(hipMemcpyAsync(ctx->desc.p, hD, sizeof(LatDesc<T>) * B, hipMemcpyHostToDevice, s));
    mcg_status q = MCG_OK;
    for (int k = 0; k < WARM + REPS && q == MCG_OK; k++) {
      if (k == WARM) HIPCHK(hipEventRecord(e0, s));
      q = run.halfsweeps(false);
      run.since_fold = 0;
    }
    if (q) return q;
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));  // also frees the pinned staging area for the next point
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    ms = (double)t / REPS;
    return MCG_OK;
  };
  auto stage = [&](std::vector<Sched> &pts, std::vector<double> &med) -> mcg_status {
    std::vector<double> t(3 * pts.size());
    for (int pass = 0; pass < 3; pass++)
      for (size_t i = 0; i < pts.size(); i++) {
        const mcg_status q = time_point(pts[i], t[3 * i + pass]);
        if (q) return q;
      }
    med.resize(pts.size());
    for (size_t i = 0; i < pts.size(); i++) {
      const double a = t[3 * i], b = t[3 * i + 1], c = t[3 * i + 2];
      med[i] = std::max(std::min(a, b), std::min(std::max(a, b), c));
    }
    return MCG_OK;
  };
  auto argmin = [](const std::vector<double> &v) { return (int)(std::min_element(v.begin(), v.end()) - v.begin()); };
  // the paired values fixes of this precision and form can run
  std::vector<int> pairings{0};
  if (c12 && ring) pairings.push_back(1);
  if (c12 && hand) pairings.push_back(2);
  // the schedule fixes of this batch would run now (for FP32, paired value 2 means paired too)
  Sched base = schedule_of(ctx, B, U);
  if (prec == MCG_F32 && base.paired == 2) base.paired = 1;
  if (std::find(pairings.begin(), pairings.end(), base.paired) == pairings.end()) base.paired = 0;
  std::vector<Sched> pts;
  std::vector<double> med;
  mcg_status rc = MCG_OK;
  for (int v = 0; v < NUM_VARIANTS; v++) pts.push_back(Sched{v, base.order, base.paired, base.nslab});
  if (!(rc = stage(pts, med))) {
    const int v1 = argmin(med);
    pts.clear();
    for (int o = 0; o <= 2; o++)
      for (int pr : pairings)
        for (int n : {1, 2, 4}) pts.push_back(Sched{v1, o, pr, n});
    if (!(rc = stage(pts, med))) {
      const Sched sb = pts[argmin(med)];
      pts.clear();
      for (int v = 0; v < NUM_VARIANTS; v++) pts.push_back(Sched{v, sb.order, sb.paired, sb.nslab});
      // the schedule the batch would run untuned, timed in the same passes as the candidates, is
      // kept unless one of them is more than 1 % faster (the rest is timing noise)
      int ib = -1;
      for (size_t i = 0; i < pts.size(); i++)
        if (pts[i].variant == base.variant && pts[i].order == base.order && pts[i].paired == base.paired &&
            pts[i].nslab == base.nslab)
          ib = (int)i;
      if (ib < 0) {
        ib = (int)pts.size();
        pts.push_back(base);
      }
      if (!(rc = stage(pts, med))) {
        int i = argmin(med);
        if (!(med[i] < 0.99 * med[ib])) i = ib;
        mcg_tune_choice c;
        memset(&c, 0, sizeof c);
        c.variant = pts[i].variant;
        c.order = pts[i].order;
        c.paired = pts[i].paired;
        c.slabs = pts[i].nslab;
        c.ms_per_sweep = med[i];
        c.ms_default = med[ib];
        ctx->tuned[tune_key(ctx, B, U)] = c;
        if (out) *out = c;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

extern "C" {

mcg_status mcg_autotune(mcg_ctx *ctx, const mcg_field *U, int32_t *best_variant, double *ms_per_halfsweep,
                        void *stream) {
  return mcg_autotune_batch(ctx, 1, U, best_variant, ms_per_halfsweep, stream);
}

mcg_status mcg_autotune_batch(mcg_ctx *ctx, int32_t B, const mcg_field *U, int32_t *best_variant,
                              double *ms_per_halfsweep, void *stream) {
  const Range range_("mcg_autotune_batch");
  if (!ctx) return MCG_EINVAL;
  if (B < 1) return fail(ctx, MCG_EINVAL, "batch size %d < 1", B);
  if (!U) return fail(ctx, MCG_EINVAL, "NULL argument");
  mcg_status st;
  for (int b = 0; b < B; b++) {
    if ((st = check_field(ctx, &U[b], "U"))) return st;
    if (U[b].prec != U[0].prec) return fail(ctx, MCG_EINVAL, "field %d: precision differs within the batch", b);
  }
  return U[0].prec == MCG_F64
             ? autotune_impl<double>(ctx, B, U, best_variant, ms_per_halfsweep, (hipStream_t)stream)
             : autotune_impl<float>(ctx, B, U, best_variant, ms_per_halfsweep, (hipStream_t)stream);
}

mcg_status mcg_tune_batch(mcg_ctx *ctx, int32_t B, const mcg_field *U, mcg_tune_choice *best, void *stream) {
  const Range range_("mcg_tune_batch");
  if (!ctx) return MCG_EINVAL;
  if (B < 1 || !U) return fail(ctx, MCG_EINVAL, "empty batch");
  mcg_status st;
  for (int b = 0; b < B; b++) {
    if ((st = check_field(ctx, &U[b], "U"))) return st;
    if (U[b].prec != U[0].prec) return fail(ctx, MCG_EINVAL, "field %d: precision differs within the batch", b);
  }
  hipStream_t s = (hipStream_t)stream;
  return U[0].prec == MCG_F64 ? tune_impl<double>(ctx, B, U, best, s) : tune_impl<float>(ctx, B, U, best, s);
}

mcg_status mcg_clear_tuning(mcg_ctx *ctx) {
  if (!ctx) return MCG_EINVAL;
  ctx->tuned.clear();
  return MCG_OK;
}

mcg_status mcg_set_variant(mcg_ctx *ctx, int32_t prec, int32_t variant) {
  if (!ctx) return MCG_EINVAL;
  ctx->tuned.clear();  // an explicit variant overrides what was tuned
  if ((prec != MCG_F64 && prec != MCG_F32) || variant < 0 || variant >= NUM_VARIANTS)
    return fail(ctx, MCG_EINVAL, "bad precision or variant");
  ctx->variant[prec][ctx->c12] = variant;
  return MCG_OK;
}

mcg_status mcg_get_variant(mcg_ctx *ctx, int32_t prec, int32_t *variant) {
  if (!ctx) return MCG_EINVAL;
  if ((prec != MCG_F64 && prec != MCG_F32) || !variant) return fail(ctx, MCG_EINVAL, "bad arguments");
  *variant = ctx->variant[prec][ctx->c12];
  return MCG_OK;
}

mcg_status mcg_set_option(mcg_ctx *ctx, int32_t option, int32_t value) {
  if (!ctx) return MCG_EINVAL;
  if (option == MCG_OPT_TWO_ROW) {
    if (value != 0 && value != 1) return fail(ctx, MCG_EINVAL, "MCG_OPT_TWO_ROW takes 0 or 1");
    ctx->c12 = value != 0;
    return MCG_OK;
  }
  if (option == MCG_OPT_SLABS) {
    if (value < 1 || value > MAX_SLABS) return fail(ctx, MCG_EINVAL, "MCG_OPT_SLABS takes 1..%d", MAX_SLABS);
    ctx->tuned.clear();  // an explicit schedule overrides what was tuned
    ctx->nslab = value;
    return MCG_OK;
  }
  if (option == MCG_OPT_EXACT) {
    if (value != 0 && value != 1) return fail(ctx, MCG_EINVAL, "MCG_OPT_EXACT takes 0 or 1");
    ctx->exact = value != 0;
    return MCG_OK;
  }
  if (option == MCG_OPT_ORDER) {
    if (value < 0 || value > 2) return fail(ctx, MCG_EINVAL, "MCG_OPT_ORDER takes 0, 1 or 2");
    ctx->tuned.clear();  // an explicit schedule overrides what was tuned
    ctx->order = value;
    return MCG_OK;
  }
  if (option == MCG_OPT_DEFER_G) {
    if (value != 0 && value != 1) return fail(ctx, MCG_EINVAL, "MCG_OPT_DEFER_G takes 0 or 1");
    ctx->defer_g = value != 0;
    return MCG_OK;
  }
  if (option == MCG_OPT_PAIRED) {
    if (value < 0 || value > 2) return fail(ctx, MCG_EINVAL, "MCG_OPT_PAIRED takes 0, 1 or 2");
    ctx->tuned.clear();  // an explicit schedule overrides what was tuned
    ctx->paired = value;
    return MCG_OK;
  }
  if (option == MCG_OPT_CHECK) {
    if (value != 0 && value != 1) return fail(ctx, MCG_EINVAL, "MCG_OPT_CHECK takes 0 or 1");
    ctx->check = value != 0;
    return MCG_OK;
  }
  if (option == MCG_OPT_SCRATCH_LIMIT_MIB) {
    if (value < 0) return fail(ctx, MCG_EINVAL, "MCG_OPT_SCRATCH_LIMIT_MIB takes >= 0");
    ctx->scratch_limit = (size_t)value << 20;
    return MCG_OK;
  }
  if (option == MCG_OPT_HITS) {
    if (value < 1 || value > 16) return fail(ctx, MCG_EINVAL, "MCG_OPT_HITS takes 1..16");
    ctx->hits = value;
    return MCG_OK;
  }
  if (option == MCG_OPT_STOP_EVERY) {
    if (value < 1 || value > 1000000) return fail(ctx, MCG_EINVAL, "MCG_OPT_STOP_EVERY takes 1..1000000");
    ctx->stop_every = value;
    return MCG_OK;
  }
  return fail(ctx, MCG_EINVAL, "unknown option %d", option);
}

mcg_status mcg_get_option(mcg_ctx *ctx, int32_t option, int32_t *value) {
  if (!ctx) return MCG_EINVAL;
  if (!value) return fail(ctx, MCG_EINVAL, "NULL output");
  if (option == MCG_OPT_TWO_ROW) {
    *value = ctx->c12 ? 1 : 0;
    return MCG_OK;
  }
  if (option == MCG_OPT_SLABS) {
    *value = ctx->nslab;
    return MCG_OK;
  }
  if (option == MCG_OPT_HITS) {
    *value = ctx->hits;
    return MCG_OK;
  }
  if (option == MCG_OPT_CHECK) {
    *value = ctx->check ? 1 : 0;
    return MCG_OK;
  }
  if (option == MCG_OPT_EXACT) {
    *value = ctx->exact ? 1 : 0;
    return MCG_OK;
  }
  if (option == MCG_OPT_ORDER) {
    *value = ctx->order;
    return MCG_OK;
  }
  if (option == MCG_OPT_DEFER_G) {
    *value = ctx->defer_g ? 1 : 0;
    return MCG_OK;
  }
  if (option == MCG_OPT_PAIRED) {
    *value = ctx->paired;
    return MCG_OK;
  }
  if (option == MCG_OPT_SCRATCH_LIMIT_MIB) {
    *value = (int32_t)(ctx->scratch_limit >> 20);
    return MCG_OK;
  }
  if (option == MCG_OPT_STOP_EVERY) {
    *value = ctx->stop_every;
    return MCG_OK;
  }
  return fail(ctx, MCG_EINVAL, "unknown option %d", option);
}

mcg_status mcg_sweeps_timed(mcg_ctx *ctx, mcg_field *W, mcg_gauge *G, int32_t n, double omega,
                            double *ms_halfsweeps, void *stream) {
  const Range range_("mcg_sweeps_timed");
  if (!ctx) return MCG_EINVAL;
  mcg_status st;
  if ((st = check_field(ctx, W, "W")) || (st = check_gauge(ctx, G, W->d, "G"))) return st;
  if (n < 1) return fail(ctx, MCG_EINVAL, "n < 1");
  if (!ms_halfsweeps) return fail(ctx, MCG_EINVAL, "NULL output");
  if (!(omega >= 0.0 && omega <= 2.0)) return fail(ctx, MCG_EINVAL, "omega must lie in [0, 2]");
  return W->prec == MCG_F64
             ? halfsweep_impl<double>(ctx, W, G, -1, omega, (hipStream_t)stream, n, ms_halfsweeps)
             : halfsweep_impl<float>(ctx, W, G, -1, omega, (hipStream_t)stream, n, ms_halfsweeps);
}

mcg_status mcg_sweeps(mcg_ctx *ctx, mcg_field *W, mcg_gauge *G, int32_t n, double omega, void *stream) {
  const Range range_("mcg_sweeps");
  if (!ctx) return MCG_EINVAL;
  mcg_status st;
  if ((st = check_field(ctx, W, "W")) || (st = check_gauge(ctx, G, W->d, "G"))) return st;
  if (n < 0) return fail(ctx, MCG_EINVAL, "n < 0");
  if (!(omega >= 0.0 && omega <= 2.0)) return fail(ctx, MCG_EINVAL, "omega must lie in [0, 2]");
  if (n == 0) return MCG_OK;
  return W->prec == MCG_F64 ? halfsweep_impl<double>(ctx, W, G, -1, omega, (hipStream_t)stream, n)
                            : halfsweep_impl<float>(ctx, W, G, -1, omega, (hipStream_t)stream, n);
}

mcg_status mcg_fix(mcg_ctx *ctx, const mcg_field *U, mcg_gauge *G, const mcg_fix_opts *opts,
                   mcg_fix_result *res, void *stream) {
  const Range range_("mcg_fix");
  if (!ctx) return MCG_EINVAL;
  if (!U) return fail(ctx, MCG_EINVAL, "U is NULL");
  hipStream_t s = (hipStream_t)stream;
  return U->prec == MCG_F64 ? fix_impl<double>(ctx, 1, U, G, opts, res, s, false)
                            : fix_impl<float>(ctx, 1, U, G, opts, res, s, false);
}

mcg_status mcg_fix_batch(mcg_ctx *ctx, int32_t B, const mcg_field *U, mcg_gauge *G,
                         const mcg_fix_opts *opts, mcg_fix_result *res, void *stream) {
  const Range range_("mcg_fix_batch");
  if (!ctx) return MCG_EINVAL;
  if (!U || B < 1) return fail(ctx, MCG_EINVAL, "empty batch");
  hipStream_t s = (hipStream_t)stream;
  return U[0].prec == MCG_F64 ? fix_impl<double>(ctx, B, U, G, opts, res, s, true)
                              : fix_impl<float>(ctx, B, U, G, opts, res, s, true);
}

mcg_status mcg_precondition_batch(mcg_ctx *ctx, int32_t B, const mcg_field *U, double rho, double eps,
                                  int32_t n, const mcg_fix_opts *opts, mcg_gauge *G, int8_t *const *Z,
                                  mcg_precond_result *res, void *stream) {
  const Range range_("mcg_precondition_batch");
  if (!ctx) return MCG_EINVAL;
  if (!U || B < 1) return fail(ctx, MCG_EINVAL, "empty batch");
  if (!G || !opts || !Z || !res) return fail(ctx, MCG_EINVAL, "NULL argument");
  if (n < 0 || std::isnan(rho) || std::isnan(eps)) return fail(ctx, MCG_EINVAL, "bad smearing parameters");
  mcg_status st;
  hipStream_t s = (hipStream_t)stream;
  for (int b = 0; b < B; b++) {
    if ((st = check_field(ctx, &U[b], "U"))) return st;
    if (U[b].prec != U[0].prec) return fail(ctx, MCG_EINVAL, "field %d: precision differs within the batch", b);
    if (!Z[b]) return fail(ctx, MCG_EINVAL, "Z[%d] is NULL", b);
    if ((st = check_inputs(ctx, &U[b], nullptr, s))) return st;
  }
  return U[0].prec == MCG_F64 ? precondition_impl<double>(ctx, B, U, rho, eps, n, opts, G, Z, res, s)
                              : precondition_impl<float>(ctx, B, U, rho, eps, n, opts, G, Z, res, s);
}

mcg_status mcg_center_project(mcg_ctx *ctx, const mcg_field *U, const mcg_gauge *G, int8_t *Z,
                              double *min_margin, void *stream) {
  const Range range_("mcg_center_project");
  if (!ctx) return MCG_EINVAL;
  mcg_status st;
  if ((st = check_field(ctx, U, "U"))) return st;
  if (G && (st = check_gauge(ctx, G, U->d, "G"))) return st;
  if (!Z) return fail(ctx, MCG_EINVAL, "Z is NULL");
  if ((st = check_inputs(ctx, U, G, (hipStream_t)stream))) return st;
  const Geom g = geom_of(U->d);
  if ((st = ensure(ctx, ctx->part, sizeof(double) * field_blocks256(g))) ||
      (st = ensure(ctx, ctx->scalars, 64)))
    return st;
  hipStream_t s = (hipStream_t)stream;
  const double *gp = G ? G->ptr : nullptr;
  double *dmin = (double *)ctx->scalars.p + 1;
  if (U->prec == MCG_F64)
    HIPCHK(launch_center_project<double>(g, U->ptr, gp, Z, (double *)ctx->part.p, dmin, s));
  else
    HIPCHK(launch_center_project<float>(g, U->ptr, gp, Z, (double *)ctx->part.p, dmin, s));
  if (min_margin) {
    HIPCHK(hipMemcpyAsync(min_margin, dmin, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return MCG_OK;
}

mcg_status mcg_center_project_noalloc(mcg_ctx *ctx, const mcg_field *U, const mcg_gauge *G, int8_t *Z,
                                      double *min_margin, void *stream) {
  const Range range_("mcg_center_project_noalloc");
  if (!ctx) return MCG_EINVAL;
  mcg_status st;
  if ((st = check_field(ctx, U, "U"))) return st;
  if (G && (st = check_gauge(ctx, G, U->d, "G"))) return st;
  if (!Z) return fail(ctx, MCG_EINVAL, "Z is NULL");
  const Geom g = geom_of(U->d);
  const int nb = field_blocks256(g);
  if (nb > NOALLOC_PARTS)
    return fail(ctx, MCG_EINVAL,
                "mcg_center_project_noalloc: %d sites exceed its limit of %d (2^25); use mcg_center_project",
                g.V, 512 * NOALLOC_PARTS);
  if (!ctx->noalloc)
    return fail(ctx, MCG_EHIP, "mcg_center_project_noalloc: no device address of its scratch: %s",
                ctx->noalloc_err.c_str());
  hipStream_t s = (hipStream_t)stream;
  const double *gp = G ? G->ptr : nullptr;
  double *part = ctx->noalloc, *dmin = ctx->noalloc + NOALLOC_PARTS;
  if (U->prec == MCG_F64)
    HIPCHK(launch_center_project<double>(g, U->ptr, gp, Z, part, dmin, s));
  else
    HIPCHK(launch_center_project<float>(g, U->ptr, gp, Z, part, dmin, s));
  if (min_margin) {
    HIPCHK(hipMemcpyAsync(min_margin, dmin, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return MCG_OK;
}

mcg_status mcg_count_vortices(mcg_ctx *ctx, const int8_t *Z, mcg_dims d, int64_t *total, int64_t *per_plane,
                              int64_t *per_charge, void *stream) {
  const Range range_("mcg_count_vortices");
  if (!ctx) return MCG_EINVAL;
  if (!Z || !total) return fail(ctx, MCG_EINVAL, "NULL argument");
  if (!dims_valid(d)) return fail(ctx, MCG_EINVAL, "bad extents");
  mcg_status st;
  if ((st = ensure(ctx, ctx->counts, 12 * sizeof(unsigned long long)))) return st;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipMemsetAsync(ctx->counts.p, 0, 12 * sizeof(unsigned long long), s));
  HIPCHK(launch_count_vortices(geom_of(d), Z, (unsigned long long *)ctx->counts.p, s));
  unsigned long long h[12];
  HIPCHK(hipMemcpyAsync(h, ctx->counts.p, sizeof h, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  int64_t tot = 0;
  for (int p = 0; p < 6; p++) {
    const int64_t a = (int64_t)h[2 * p], b = (int64_t)h[2 * p + 1];
    if (per_plane) per_plane[p] = a + b;
    tot += a + b;
  }
  if (per_charge) {
    per_charge[0] = per_charge[1] = 0;
    for (int p = 0; p < 6; p++) {
      per_charge[0] += (int64_t)h[2 * p];
      per_charge[1] += (int64_t)h[2 * p + 1];
    }
  }
  *total = tot;
  return MCG_OK;
}

mcg_status mcg_vortex_field(mcg_ctx *ctx, const mcg_field *U, const mcg_gauge *G, const int8_t *Z, int32_t mode,
                            mcg_field *out, void *stream) {
  const Range range_("mcg_vortex_field");
  if (!ctx) return MCG_EINVAL;
  mcg_status st;
  if ((st = check_field(ctx, U, "U")) || (st = check_field(ctx, out, "out"))) return st;
  if (G && (st = check_gauge(ctx, G, U->d, "G"))) return st;
  if (!same_dims(U->d, out->d) || U->prec != out->prec)
    return fail(ctx, MCG_EINVAL, "U and out differ in extents or precision");
  if (!Z) return fail(ctx, MCG_EINVAL, "Z is NULL");
  if (mode != MCG_VORTEX_ONLY && mode != MCG_VORTEX_REMOVED) return fail(ctx, MCG_EINVAL, "bad mode %d", mode);
  if ((st = check_inputs(ctx, U, G, (hipStream_t)stream))) return st;
  const Geom g = geom_of(U->d);
  const double *gp = G ? G->ptr : nullptr;
  hipStream_t s = (hipStream_t)stream;
  if (U->prec == MCG_F64)
    HIPCHK(launch_vortex_field<double>(g, U->ptr, gp, Z, mode, out->ptr, s));
  else
    HIPCHK(launch_vortex_field<float>(g, U->ptr, gp, Z, mode, out->ptr, s));
  return MCG_OK;
}

}  // extern "C"

namespace {

// unit steps +-(axis+1) of the staircase from 0 to v: each step along the axis with steps left
// whose (taken + 1/2) / |v_axis| is smallest, the lower axis on a tie (compared exactly as
// (2 taken_a + 1) |v_b| < (2 taken_b + 1) |v_a|)
std::vector<int> staircase_steps(const int v[3]) {
  int taken[3] = {0, 0, 0}, n = std::abs(v[0]) + std::abs(v[1]) + std::abs(v[2]);
  std::vector<int> st;
  for (int q = 0; q < n; q++) {
    int best = -1;
    for (int a = 0; a < 3; a++) {
      if (taken[a] >= std::abs(v[a])) continue;
      if (best < 0 || (int64_t)(2 * taken[a] + 1) * std::abs(v[best]) <
                          (int64_t)(2 * taken[best] + 1) * std::abs(v[a]))
        best = a;
    }
    taken[best]++;
    st.push_back(v[best] > 0 ? best + 1 : -(best + 1));
  }
  return st;
}

// distinct images of a step sequence under the 48 signed axis permutations, each with the
// number of images it stands for: an image whose reversed, negated sequence (the same loop
// traversed from its other corner, equal in translation-averaged Re tr) is already listed is
// merged into that entry
std::vector<std::pair<std::vector<int>, int>> path_images(const std::vector<int> &base) {
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  std::vector<std::vector<int>> all;
  for (const auto &p : perms)
    for (int sg = 0; sg < 8; sg++) {
      std::vector<int> img;
      for (int st : base) {
        const int a = std::abs(st) - 1, sign = (st > 0 ? 1 : -1) * ((sg >> a) & 1 ? -1 : 1);
        img.push_back(sign * (p[a] + 1));
      }
      all.push_back(img);
    }
  std::sort(all.begin(), all.end());
  all.erase(std::unique(all.begin(), all.end()), all.end());
  std::vector<std::pair<std::vector<int>, int>> out;
  for (const auto &img : all) {
    std::vector<int> rn(img.rbegin(), img.rend());
    for (int &x : rn) x = -x;
    bool merged = false;
    for (auto &e : out)
      if (e.first == rn) {
        e.second++;
        merged = true;
        break;
      }
    if (!merged) out.push_back({img, 1});
  }
  return out;
}

template <typename T>
mcg_status wilson_impl(mcg_ctx *ctx, const mcg_field *U, int nvec, const int32_t *vec, int rmax, int tmax,
                       double *W, hipStream_t s) {
  const Geom g = geom_of(U->d);
  const size_t line_bytes = (size_t)g.V * 9 * 2 * sizeof(T);
  const int nres = nvec * rmax * tmax;
  // images per launch: up to LOOP_IMAGES_PER_LAUNCH, as many as keep their line fields within 4 GiB
  const int ni = (int)std::max<size_t>(
      1, std::min<size_t>(LOOP_IMAGES_PER_LAUNCH, ((size_t)4 << 30) / (2 * line_bytes)));
  mcg_status st;
  if ((st = ensure(ctx, ctx->line_a, line_bytes * ni)) || (st = ensure(ctx, ctx->line_b, line_bytes * ni)) ||
      (st = ensure(ctx, ctx->wl_part, sizeof(double) * (size_t)ni * tmax * line_blocks(g))) ||
      (st = ensure(ctx, ctx->wl_res, sizeof(double) * (size_t)nres)) ||
      (st = ensure(ctx, ctx->wl_img, sizeof(LoopImage<T>) * ni)) ||
      (st = ensure_pinned(ctx, sizeof(LoopImage<T>) * ni)))
    return st;
  double *res = (double *)ctx->wl_res.p;
  LoopImage<T> *hI = (LoopImage<T> *)ctx->h_pinned;
  const LoopImage<T> *dI = (const LoopImage<T> *)ctx->wl_img.p;
  HIPCHK(launch_zero(res, nres, s));
  for (int i = 0; i < nvec; i++) {
    const int v[3] = {vec[3 * i], vec[3 * i + 1], vec[3 * i + 2]};
    const auto imgs = path_images(staircase_steps(v));
    int nimg = 0;
    for (const auto &e : imgs) nimg += e.second;
    for (size_t c0 = 0; c0 < imgs.size(); c0 += ni) {
      const int n = (int)std::min<size_t>(ni, imgs.size() - c0);
      // the staging area and the descriptor table may still feed the previous chunk's launches
      HIPCHK(hipStreamSynchronize(s));
      for (int j = 0; j < n; j++) {
        const auto &e = imgs[c0 + j];
        LoopImage<T> d;
        memset(&d, 0, sizeof d);
        d.path.n = (int)e.first.size();
        for (int q = 0; q < d.path.n; q++) {
          d.path.s[q] = (signed char)e.first[q];
          d.path.d[std::abs(e.first[q]) - 1] += e.first[q] > 0 ? 1 : -1;
        }
        // Re tr / 3, averaged over sites and images
        d.weight = (double)e.second / (3.0 * (double)nimg * (double)g.V);
        d.a = (V2<T> *)((char *)ctx->line_a.p + (size_t)j * line_bytes);
        d.b = (V2<T> *)((char *)ctx->line_b.p + (size_t)j * line_bytes);
        hI[j] = d;
      }
      HIPCHK(hipMemcpyAsync(ctx->wl_img.p, hI, sizeof(LoopImage<T>) * n, hipMemcpyHostToDevice, s));
      for (int k = 1; k <= rmax; k++) {
        HIPCHK(launch_lines<T>(g, U->ptr, dI, n, k, s));
        HIPCHK(launch_wloops<T>(g, U->ptr, dI, n, k, tmax, (double *)ctx->wl_part.p,
                                res + (size_t)(i * rmax + k - 1) * tmax, s));
      }
    }
  }
  HIPCHK(hipMemcpyAsync(W, res, sizeof(double) * nres, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return MCG_OK;
}

}  // namespace

extern "C" {

mcg_status mcg_wilson_loops(mcg_ctx *ctx, const mcg_field *U, int32_t nvec, const int32_t *vec, int32_t rmax,
                            int32_t tmax, double *W, void *stream) {
  const Range range_("mcg_wilson_loops");
  if (!ctx) return MCG_EINVAL;
  mcg_status st;
  if ((st = check_field(ctx, U, "U"))) return st;
  if (nvec < 1 || !vec || !W) return fail(ctx, MCG_EINVAL, "need nvec >= 1, vec and W");
  if (rmax < 1 || tmax < 1) return fail(ctx, MCG_EINVAL, "rmax and tmax must be >= 1");
  if (tmax > U->d.L[3]) return fail(ctx, MCG_EINVAL, "tmax %d exceeds L[3] = %d", tmax, U->d.L[3]);
  const int lmin = std::min(U->d.L[0], std::min(U->d.L[1], U->d.L[2]));
  if ((int64_t)nvec * rmax * tmax > (int64_t(1) << 24)) return fail(ctx, MCG_EINVAL, "too many loops requested");
  for (int i = 0; i < nvec; i++) {
    int n1 = 0, mx = 0;
    for (int j = 0; j < 3; j++) {
      const int a = std::abs(vec[3 * i + j]);
      if (a > 8) return fail(ctx, MCG_EINVAL, "vector %d: components must lie in [-8, 8]", i);
      n1 += a;
      mx = std::max(mx, a);
    }
    if (n1 == 0 || n1 > 24) return fail(ctx, MCG_EINVAL, "vector %d: need 0 < |v|_1 <= 24", i);
    if ((int64_t)rmax * mx > lmin)
      return fail(ctx, MCG_EINVAL, "vector %d: rmax * max|v_j| = %lld exceeds the smallest spatial extent %d", i,
                  (long long)rmax * mx, lmin);
  }
  if ((st = check_inputs(ctx, U, nullptr, (hipStream_t)stream))) return st;
  return U->prec == MCG_F64 ? wilson_impl<double>(ctx, U, nvec, vec, rmax, tmax, W, (hipStream_t)stream)
                            : wilson_impl<float>(ctx, U, nvec, vec, rmax, tmax, W, (hipStream_t)stream);
}

mcg_status mcg_smear_mcg_backward(mcg_ctx *ctx, const mcg_field *U, double rho, double eps, int32_t n,
                                  const mcg_gauge *Gstar, int32_t ckpt_every, mcg_field *gradU, double *loss,
                                  double *dRho, double *dEps, void *stream) {
  const Range range_("mcg_smear_mcg_backward");
  if (!ctx) return MCG_EINVAL;
  mcg_status st;
  if ((st = check_field(ctx, U, "U")) || (st = check_field(ctx, gradU, "gradU")) ||
      (st = check_gauge(ctx, Gstar, U->d, "Gstar")))
    return st;
  if (!same_dims(U->d, gradU->d) || U->prec != gradU->prec)
    return fail(ctx, MCG_EINVAL, "U and gradU differ in extents or precision");
  if (U->ptr == gradU->ptr) return fail(ctx, MCG_EINVAL, "U and gradU must not alias");
  if (n < 0 || std::isnan(rho) || std::isnan(eps)) return fail(ctx, MCG_EINVAL, "bad smearing parameters");
  if (!loss || !dRho || !dEps) return fail(ctx, MCG_EINVAL, "NULL output");
  if ((st = check_inputs(ctx, U, Gstar, (hipStream_t)stream))) return st;
  return U->prec == MCG_F64
             ? backward_impl<double>(ctx, U, rho, eps, n, Gstar, ckpt_every, gradU, loss, dRho, dEps,
                                     (hipStream_t)stream)
             : backward_impl<float>(ctx, U, rho, eps, n, Gstar, ckpt_every, gradU, loss, dRho, dEps,
                                    (hipStream_t)stream);
}

}  // extern "C"
