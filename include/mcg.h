/*
 * mcg.h -- C ABI of the gfx950 (MI355X) library for stout-preconditioned
 * Maximal Center Gauge fixing in SU(3) (O Cais et al., arXiv:0807.0264).
 *
 * The calls follow the paper's statement of the method:
 *   smear(U, rho, eps, n)        Sec. II.B and Sec. III (stout, over-improved stout)
 *   mcg_fix(U) -> (G, R)         Sec. II.A (maximise V_U[G] by local updates)
 *   apply_gauge(U, G)            Sec. II.A/B (U^G; preconditioning transform)
 *   center_project(U, G) -> Z    Sec. II.A (nearest centre element of tr U^G)
 *   count_vortices(Z)            Sec. II.A (non-trivial plaquettes of Z)
 *
 * Conventions
 *   - Extents L = (Lx, Ly, Lz, Lt), each even and >= 2, with at most
 *     53,687,091 sites (80 V < 2^32: device loads use 32-bit byte offsets
 *     within a field), else MCG_EINVAL; periodic; site index
 *     i = x + Lx*(y + Ly*(z + Lz*t)); parity (x+y+z+t) mod 2; half index
 *     h = i >> 1 (the site's index among the V/2 sites of its parity).
 *   - Gauge transform: U^G_mu(x) = G(x) U_mu(x) G(x+mu)^dagger.
 *   - Functional: R = V_U = (1/(9 N_l)) sum_{x,mu} |tr U_mu(x)|^2, N_l = 4V.
 *   - Centre phase: m in {-1,0,1} maximising Re(t e^{-2 pi i m/3}) with
 *     t = tr U^G_mu(x) evaluated in FP64; candidates tried in the order
 *     0, +1, -1 (first wins a tie); t = 0 gives m = 0.
 *
 * Memory (all device pointers, caller-owned, never freed by the library)
 *   mcg_field  links in the internal structure-of-arrays layout: complex
 *              element (mu, parity, k = 3*row + col, h) at complex offset
 *              ((mu*2 + parity)*9 + k)*(V/2) + h; each complex is two reals
 *              (re, im) of the field's precision (MCG_F64: double,
 *              MCG_F32: float).  Size: mcg_field_bytes().
 *   mcg_gauge  per-site SU(3) transform, always FP64: complex element
 *              (parity, k, h) at complex offset (parity*9 + k)*(V/2) + h.
 *              Size: mcg_gauge_bytes().
 *   Z          int8 centre integers, element (mu, i) at mu*V + i.
 *   Interchange arrays (mcg_pack_* / mcg_unpack_*): complex [Lt][Lz][Ly][Lx][4][3][3]
 *              (links) or [Lt][Lz][Ly][Lx][3][3] (gauge), row-major 3x3.
 *
 * Streams: `stream` is a hipStream_t (NULL = default stream).  Calls enqueue
 * work on it and return without waiting, except those that return host
 * scalars (functional, plaquette, theta, fix, fix_batch, center_project's
 * min_margin, count_vortices, the backward's scalars), which synchronise
 * that stream before returning.
 *
 * Errors: every call returns an mcg_status.  Negative values are errors
 * (outputs undefined, the context stays usable); MCG_WNOTCONV is a warning
 * with valid outputs.  mcg_last_error() gives the message of the context's
 * last error.  No call aborts the process.
 *
 * Threads: a context may be used by one host thread at a time.  Calls on
 * one context that overlap on the GPU (different streams) share the
 * context's scratch buffers and race; use one context per stream.
 */
#ifndef MCG_H
#define MCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mcg_status;
enum {
  MCG_OK = 0,
  MCG_WNOTCONV = 1, /* max_sweeps reached; G and R valid and resumable */
  MCG_EINVAL = -1,  /* bad argument: odd/small extent, null pointer, dims mismatch, aliasing */
  MCG_ENOMEM = -2,  /* scratch allocation failed */
  MCG_EHIP = -3,    /* a HIP runtime call failed */
  MCG_EINPUT = -4   /* input outside the method's range (e.g. smearing step too large) */
};

enum { MCG_F64 = 0, MCG_F32 = 1 };

typedef struct {
  int32_t L[4]; /* Lx (fastest), Ly, Lz, Lt */
} mcg_dims;

typedef struct {
  mcg_dims d;
  int32_t prec; /* MCG_F64 or MCG_F32 */
  int32_t pad_;
  void *ptr;    /* device, mcg_field_bytes(d, prec) bytes */
} mcg_field;

typedef struct {
  mcg_dims d;
  double *ptr; /* device, mcg_gauge_bytes(d) bytes */
} mcg_gauge;

/* Options of the fixing iteration (Sec. II.A; readings in the comments).
 * A sweep is one update of every even site followed by one of every odd
 * site ("iteration" of the paper; it counts work in blocks of 50). */
typedef struct {
  double tol;            /* stop after the first sweep s with R_s - R_{s-1} < tol */
  double omega;          /* over-relaxation of each SU(2) subgroup step, in [0, 2] */
  int32_t max_sweeps;    /* sweeps allowed in this call (>= 0) */
  int32_t reunit_every;  /* re-unitarise G and re-derive W = U^G before every sweep s
                            with (s-1) % reunit_every == 0, except the first of a call */
  int32_t start_sweep;   /* global number of sweeps already done (resume) */
  int32_t check_every;   /* host polls the device stop flag every this many sweeps (>= 1) */
  double *traj;          /* nullable HOST array of max_sweeps+1 doubles: R before the
                            first sweep and after each sweep done */
} mcg_fix_opts;

typedef struct {
  double R;        /* R(U^G) after the final re-unitarisation of G */
  double dR;       /* last R_s - R_{s-1} */
  double theta;    /* stationarity residual (1/V) sum_x |TA X(x)|_F^2, X the local
                      linearisation sum_k conj(tr M_k) M_k over the 8 links at x */
  int32_t sweeps;  /* sweeps done in this call */
  int32_t blocks50;/* ceil(sweeps / 50) */
  int32_t status;  /* MCG_OK or MCG_WNOTCONV */
  int32_t pad_;
} mcg_fix_result;

typedef struct mcg_ctx mcg_ctx;

/* ---- context ------------------------------------------------------------ */
/* Create a context on HIP device `device`; it owns scratch buffers, graphs
 * and the autotune table.  Returns MCG_EHIP if the device is unusable. */
mcg_status mcg_create(mcg_ctx **ctx, int32_t device);
mcg_status mcg_destroy(mcg_ctx *ctx);
const char *mcg_status_string(mcg_status s);
const char *mcg_last_error(const mcg_ctx *ctx);

/* Bytes of an internal link field / gauge field; 0 for invalid dims. */
size_t mcg_field_bytes(mcg_dims d, int32_t prec);
size_t mcg_gauge_bytes(mcg_dims d);

/* ---- layout conversion ---------------------------------------------------- */
/* src: device interchange links of precision src_prec -> dst (any precision;
 * FP64 -> FP32 rounds to nearest). */
mcg_status mcg_pack_links(mcg_ctx *ctx, const void *src, int32_t src_prec,
                          mcg_field *dst, void *stream);
mcg_status mcg_unpack_links(mcg_ctx *ctx, const mcg_field *src, void *dst,
                            int32_t dst_prec, void *stream);
/* src/dst: device interchange gauge field, complex double */
mcg_status mcg_pack_gauge(mcg_ctx *ctx, const double *src, mcg_gauge *dst, void *stream);
mcg_status mcg_unpack_gauge(mcg_ctx *ctx, const mcg_gauge *src, double *dst, void *stream);
/* G(x) = 1 everywhere */
mcg_status mcg_gauge_identity(mcg_ctx *ctx, mcg_gauge *G, void *stream);
/* Re-unitarise every G(x) (Gram-Schmidt on rows, third row conj(r0 x r1)). */
mcg_status mcg_gauge_reunit(mcg_ctx *ctx, mcg_gauge *G, void *stream);

/* ---- input validation --------------------------------------------------------------- */
/* Largest |(M M^dagger - 1)_ij| over the links of U and over the matrices of
 * G (either may be NULL; host outputs dev_U / dev_G nullable, +inf when an
 * entry is NaN).  A field fresh from unitary data reads ~1e-7 in FP32 and
 * ~1e-15 in FP64.  Synchronises the stream. */
mcg_status mcg_unitarity(mcg_ctx *ctx, const mcg_field *U, const mcg_gauge *G, double *dev_U, double *dev_G,
                         void *stream);

/* ---- smearing (Sec. II.B; parameters of Sec. III) -------------------------- */
/* n Jacobi steps U' = exp(TA(C U^dagger)) U with the staple sum
 *   C = rho sum_{nu != mu} [ (5-2eps)/3 (2 plaquette staples)
 *                          - (1-eps)/12 (6 rectangle staples) ]
 * (eps = 1: stout; eps < 1: over-improved stout).  TA(M) is the traceless
 * anti-Hermitian part.  n == 0 copies U.  U and out must have equal dims and
 * precision and must not alias.  MCG_EINPUT if some exponent is too large for
 * the series used (spectral radius of C U^dagger above 6). */
mcg_status mcg_smear(mcg_ctx *ctx, const mcg_field *U, mcg_field *out, double rho,
                     double eps, int32_t n, void *stream);

/* ---- gauge transform and functional (Sec. II.A) ------------------------------- */
/* out = U^G (same precision as U; computed in FP64, rounded once). out may alias U. */
mcg_status mcg_apply_gauge(mcg_ctx *ctx, const mcg_field *U, const mcg_gauge *G,
                           mcg_field *out, void *stream);
/* *R = V_U[1] of the field as given (host scalar; FP64 accumulation). */
mcg_status mcg_functional(mcg_ctx *ctx, const mcg_field *U, double *R, void *stream);
/* *P = (1/(18V)) sum_{x, mu<nu} Re tr U_P (host scalar), a gauge invariant. */
mcg_status mcg_plaquette(mcg_ctx *ctx, const mcg_field *U, double *P, void *stream);
/* *theta = stationarity residual of the field as given (host scalar). */
mcg_status mcg_theta(mcg_ctx *ctx, const mcg_field *W, double *theta, void *stream);

/* ---- MCG fixing (Sec. II.A; preconditioning of Sec. II.B) ---------------------- */
/* One half-sweep in place: every site x of `parity` gets the local update g
 * (three SU(2)-subgroup steps maximising the linearised functional
 * Re tr(g X), X = sum_k conj(tr M_k) M_k over the eight links M_k at x, each
 * step over-relaxed with omega), then W_mu(x) <- g W_mu(x),
 * W_mu(x-mu) <- W_mu(x-mu) g^dagger, G(x) <- g G(x).  W and G must not alias. */
mcg_status mcg_halfsweep(mcg_ctx *ctx, mcg_field *W, mcg_gauge *G, int32_t parity,
                         double omega, void *stream);
/* n raw sweeps in place: n times (every even site, then every odd site) as
 * in mcg_halfsweep, launched back to back with no stop test, no R and no
 * re-unitarisation (the fixed-work loop used to measure throughput).  In the
 * two-row storage form (MCG_OPT_TWO_ROW) W and G are converted into context
 * scratch before the sweeps and back after them. */
mcg_status mcg_sweeps(mcg_ctx *ctx, mcg_field *W, mcg_gauge *G, int32_t n, double omega,
                      void *stream);
/* mcg_sweeps (n >= 1) that also returns in *ms_halfsweeps (host) the summed
 * duration of the half-sweep launches alone, from HIP events recorded on
 * `stream` before and after each sweep's two half-sweeps: the folds of the
 * transform ring (MCG_OPT_DEFER_G) and the storage-form conversions fall
 * outside.  Synchronises the stream. */
mcg_status mcg_sweeps_timed(mcg_ctx *ctx, mcg_field *W, mcg_gauge *G, int32_t n, double omega,
                            double *ms_halfsweeps, void *stream);
/* Fix U to MCG.  G holds the start transform on entry (mcg_gauge_identity for
 * plain fixing; the smeared field's transform for the preconditioned re-fix)
 * and the total transform on exit; U is not modified.  The working field
 * W = U^G lives in context scratch.  Returns MCG_OK or MCG_WNOTCONV. */
mcg_status mcg_fix(mcg_ctx *ctx, const mcg_field *U, mcg_gauge *G, const mcg_fix_opts *opts,
                   mcg_fix_result *res, void *stream);
/* Fix B independent fields (Gribov copies and/or lattices of unequal sizes,
 * one precision) concurrently: each half-sweep is ONE launch over all the
 * fields, and the sweep loop runs as a captured hipGraph replayed per block
 * of reunit_every sweeps, with per-field stop flags on the device.  opts is
 * an array of B entries (tol and max_sweeps may differ; omega, reunit_every
 * and start_sweep must agree).  Each field's result equals, bit for bit, the
 * result of mcg_fix on it alone.  U[b] and G[b] as in mcg_fix. */
mcg_status mcg_fix_batch(mcg_ctx *ctx, int32_t B, const mcg_field *U, mcg_gauge *G,
                         const mcg_fix_opts *opts, mcg_fix_result *res, void *stream);

/* The whole preconditioned path of Sec. II.B for a batch of B fields (one
 * precision; Gribov copies and/or lattices of unequal sizes): n smearing steps
 * of every field (rho, eps as in mcg_smear; the smeared fields live in
 * context scratch), one mcg_fix_batch of the smeared fields from G, one of
 * the original fields from the transforms that gave, then the centre
 * projection of every fixed field (Z[b]: caller-owned device array [4][V] as
 * in mcg_center_project) and its P-vortex count.  G[b]: the start transform
 * on entry (mcg_gauge_identity for plain fixing), the total on exit.  opts as
 * in mcg_fix_batch, used by both fixes.  res (host, B entries): both fixes'
 * results, the minimum centre-phase margin and the counts of mcg_count_vortices.
 * Each field's results equal, bit for bit, those of the same calls made one by
 * one; the host synchronises once per block of sweeps of each fix (stop flags)
 * and once at the end.  Returns MCG_WNOTCONV if either fix of any field ran
 * out of sweeps. */
typedef struct {
  mcg_fix_result smeared;  /* fix of the smeared field ("smeared maximum" of Table I) */
  mcg_fix_result fixed;    /* fix of the original field from the smeared field's transform */
  double min_margin;       /* as mcg_center_project */
  int64_t vortices;        /* P-vortex plaquettes, as mcg_count_vortices */
  int64_t per_plane[6];
  int64_t per_charge[2];
} mcg_precond_result;
mcg_status mcg_precondition_batch(mcg_ctx *ctx, int32_t B, const mcg_field *U, double rho, double eps,
                                  int32_t n, const mcg_fix_opts *opts, mcg_gauge *G, int8_t *const *Z,
                                  mcg_precond_result *res, void *stream);

/* ---- kernel variants and autotuning ------------------------------------------------ */
/* The half-sweep kernel has MCG_NUM_VARIANTS variants: variant v uses blocks
 * of {64, 128, 256}[v % 3] threads and targets 1 + v / 3 waves per SIMD.
 * mcg_autotune times every variant on a scratch copy of U (G = 1; U is not
 * modified) in the context's storage form, in three interleaved passes of 8
 * half-sweeps each, keeps the variant with the smallest median for U's
 * precision and that form, and returns it (best_variant,
 * ms_per_halfsweep[MCG_NUM_VARIANTS] nullable, host: the medians).  The variant fixes the
 * block decomposition of every fixing kernel, hence the order of the FP64
 * partial sums: results at one variant are deterministic. */
#define MCG_NUM_VARIANTS 6
mcg_status mcg_autotune(mcg_ctx *ctx, const mcg_field *U, int32_t *best_variant,
                        double *ms_per_halfsweep, void *stream);
/* mcg_autotune over a batch: every timed launch is one half-sweep over all B
 * fields (U[0..B-1], one precision, host array of descriptors), as
 * mcg_fix_batch runs them; the choice is kept for that precision and storage
 * form.  Uses the scratch that mcg_fix_batch on the same fields uses. */
mcg_status mcg_autotune_batch(mcg_ctx *ctx, int32_t B, const mcg_field *U, int32_t *best_variant,
                              double *ms_per_halfsweep, void *stream);
/* The launch variant and the schedule of the fixing sweeps, tuned on a batch.
 * mcg_tune_batch times whole sweeps (both half-sweeps over all B fields, as
 * mcg_fix_batch runs them: working copies of U with G = 1 in the context's
 * storage form, with its transform ring or FP64 handoff slot) in three
 * stages: every variant under the schedule fixes of this batch would use
 * now; every schedule -- tile order (MCG_OPT_ORDER 0/1/2) x paired sweeps
 * (MCG_OPT_PAIRED: 0/1 for FP32 with the ring, 0/2 for FP64 in the two-row
 * form, else 0) x slabs (MCG_OPT_SLABS 1/2/4) -- under the best variant;
 * every variant under the best schedule, together with the schedule in use
 * before tuning.  Each stage runs three interleaved passes of 4 timed sweeps
 * per point (after one untimed) and ranks points by their median; the last
 * stage keeps the schedule in use unless a point is more than 1 % faster
 * than it in the same passes.  The choice is kept in the context for this batch shape
 * (precision, storage form, transform ring, update variant and the fields'
 * extents in order) and used by mcg_fix and mcg_fix_batch on batches of that
 * shape instead of the context's variant and schedule options, until
 * mcg_set_variant, mcg_set_option(MCG_OPT_ORDER / _PAIRED / _SLABS) or
 * mcg_clear_tuning.  All schedules give the same bits: they change only the
 * order in which independent sites are visited and where a site's g waits.
 * Not available with MCG_OPT_HITS > 1 or MCG_OPT_EXACT (one fixed variant).
 * best (nullable, host): the choice, its median ms per sweep, and that of
 * the schedule the batch had before (ms_default). */
typedef struct {
  int32_t variant;     /* half-sweep variant, as in mcg_set_variant */
  int32_t order;       /* MCG_OPT_ORDER value */
  int32_t paired;      /* MCG_OPT_PAIRED value */
  int32_t slabs;       /* MCG_OPT_SLABS value */
  double ms_per_sweep; /* median over the three passes, one sweep over the batch */
  double ms_default;   /* the same, in the same passes, for the schedule in use before tuning */
} mcg_tune_choice;
mcg_status mcg_tune_batch(mcg_ctx *ctx, int32_t B, const mcg_field *U, mcg_tune_choice *best,
                          void *stream);
mcg_status mcg_clear_tuning(mcg_ctx *ctx);
mcg_status mcg_set_variant(mcg_ctx *ctx, int32_t prec, int32_t variant);
mcg_status mcg_get_variant(mcg_ctx *ctx, int32_t prec, int32_t *variant);

/* ---- options ----------------------------------------------------------------------- */
/* MCG_OPT_TWO_ROW (default 1): the fixing iteration (mcg_fix, mcg_fix_batch,
 * mcg_sweeps) keeps its working field W and transform G in context scratch
 * as their first two rows (row 2 = conj(row 0 x row 1) for SU(3)), moving
 * 2/3 of the bytes per site-update; 0 keeps all three rows.  Caller-visible
 * fields and transforms always use the full layouts above. */
#define MCG_OPT_TWO_ROW 1
/* MCG_OPT_SLABS (1..16, default 1): the sweeps of mcg_fix, mcg_fix_batch and
 * mcg_sweeps run each half-sweep of a field in this many slabs of
 * consecutive time slices (a field too small for slabs of two slices or
 * more stays whole), ordered even slabs 0, 1, then (even k, odd k-1) for
 * k = 2..n-1, then odd n-1, odd 0.  Every odd slab runs after the even slabs
 * it touches and no even slab after an odd slab it touches, so results are
 * bit-identical to whole half-sweeps; the gain is that a slab's links are
 * re-read while they may still sit in the device's last-level cache. */
#define MCG_OPT_SLABS 2
/* Variants of the update rule (both default 1, the method as in mcg_fix):
 * MCG_OPT_HITS (1..16): re-linearisation hits per site visit of mcg_fix,
 * mcg_fix_batch, mcg_sweeps and mcg_halfsweep.  After the first update g,
 * each further hit linearises sum_k |tr(g' M_k)|^2 at the current g,
 * X_g = sum_k conj(tr(g M_k)) M_k, and applies the three over-relaxed
 * subgroup steps to g X_g, continuing g (hits > 1 run with 256-thread
 * blocks whatever the tuned variant).
 * MCG_OPT_STOP_EVERY (1..10^6): the stop test dR < tol of mcg_fix and
 * mcg_fix_batch is applied only after sweeps whose global number
 * (start_sweep + k) is a multiple of this, e.g. 50 for whole blocks. */
#define MCG_OPT_HITS 3
#define MCG_OPT_STOP_EVERY 4
/* MCG_OPT_EXACT (0/1, default 0): each subgroup step maximises
 * sum_k |tr(s g M_k)|^2 over its SU(2) subgroup exactly instead of the
 * linearised functional (then over-relaxes the same way; with omega > 1
 * monotonicity is no longer guaranteed).  The subgroup functional is
 * const + 2 h.a + a^T Q a on the unit 3-sphere; its maximiser comes from the
 * eigendecomposition of the 4x4 Q and a secular equation, in FP64.  Combined
 * with MCG_OPT_HITS, the three exact steps repeat `hits` times.  Runs with
 * 256-thread blocks. */
#define MCG_OPT_EXACT 7
/* MCG_OPT_ORDER (0/1/2, default 2): 1 makes every odd half-sweep visit the
 * lattice tiles in reverse order, so it starts on the links the even
 * half-sweep wrote last (and the next even half-sweep on those the odd one
 * wrote last), which the last-level cache may still hold; the reversal keeps
 * each tile on the XCD that handles it in the forward order.  2: the same
 * alternation, and within each field the blocks that one XCD runs take a
 * contiguous range of its tiles instead of every eighth tile, so a site's
 * neighbours along z mostly lie on the same XCD (the odd half of a paired
 * sweep reads the even g of all eight neighbours).  0: every half-sweep in
 * forward order.  Results are bit-identical for all three: the sites of one
 * parity are independent and the reduction partials belong to tiles, not to
 * the launch order. */
#define MCG_OPT_ORDER 8
/* MCG_OPT_DEFER_G (0/1, default 1): with FP32 links, mcg_fix, mcg_fix_batch
 * and mcg_sweeps let each half-sweep write its per-site g (two rows, FP32)
 * into a ring of at most 25 sweeps instead of reading and writing the FP64
 * transform, and fold the ring into G (one g at a time, in FP64, the same
 * products in the same order) before each re-unitarisation, when the ring
 * is full and at the end: 48 bytes per site-update instead of 192 (two-row
 * form).  The ring of a fix holds ceil(r / ceil(r / 25)) sweeps, r its
 * reunit_every (25 for the default 50: folds after sweeps 25 and 50 of each
 * block), that of mcg_sweeps 25.  Results are bit-identical to 0.  Costs
 * 48 * C * L0*L1*L2*L3 bytes of context scratch per field for a ring of C
 * sweeps (2C slots of 48 bytes per site of one parity; 1200 bytes per site at
 * C = 25); FP64 fixes always update G in place.  The ring is reserved last
 * and is optional: when it does not fit in device memory or under
 * MCG_OPT_SCRATCH_LIMIT_MIB, the call updates G in place instead (the same
 * results) and does not fail. */
#define MCG_OPT_DEFER_G 9
/* MCG_OPT_PAIRED (0/1/2, default 1): where the transform ring is in use (FP32
 * links in the two-row form, MCG_OPT_DEFER_G), the first half-sweep of each
 * sweep only records its g in the ring and leaves the links alone; the second
 * applies that pending g of each neighbour to the links it loads, then its
 * own update.  Each link joins one site of each parity, so it is then read
 * twice and written once per sweep instead of read and written twice (with
 * the ring: 648 instead of 816 bytes per site-update, Sec. II.A's sweep
 * unchanged).  2: FP64 fixes and raw sweeps (two-row form) are paired too,
 * the even g handed over in a one-slot buffer of 48 * L0*L1*L2*L3 bytes per
 * field (optional like the ring) while G is updated in place: 1440 instead
 * of 1728 bytes per site-update, but slower on MI355X, where the FP64
 * half-sweep is bound by its arithmetic at one wave per SIMD.  Results are
 * bit-identical for all values: every form applies g to the links with row
 * 2 rebuilt from rows 0 and 1 and in one fixed FMA order. */
#define MCG_OPT_PAIRED 10
/* MCG_OPT_CHECK (0/1, default 0): every call that reads links or a gauge
 * transform (smear, apply_gauge, fix, fix_batch, center_project,
 * vortex_field, wilson_loops, smear_mcg_backward) first checks them and
 * returns MCG_EINPUT, with the deviation in mcg_last_error, unless
 * max_ij |(U U^dagger - 1)_ij| <= 1e-6 (FP32 links) or 1e-10 (FP64 links and
 * every G) and no entry is NaN.  Costs one extra read of the inputs and a
 * stream synchronisation per call. */
#define MCG_OPT_CHECK 5
/* MCG_OPT_SCRATCH_LIMIT_MIB (>= 0, default 0 = none): the most device memory
 * the context may hold as scratch; a call that would need more returns
 * MCG_ENOMEM and leaves the context usable. */
#define MCG_OPT_SCRATCH_LIMIT_MIB 6
mcg_status mcg_set_option(mcg_ctx *ctx, int32_t option, int32_t value);
mcg_status mcg_get_option(mcg_ctx *ctx, int32_t option, int32_t *value);

/* ---- centre projection and P-vortices (Sec. II.A) -------------------------------- */
/* Z = centre integer of every link of U^G (G nullable: U as given), decided
 * in FP64; *min_margin (nullable, host) = min over links of
 * pi/3 - |arg(t e^{-2 pi i m/3})|. */
mcg_status mcg_center_project(mcg_ctx *ctx, const mcg_field *U, const mcg_gauge *G,
                              int8_t *Z, double *min_margin, void *stream);
/* mcg_center_project for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * Z and *min_margin, bit for bit, but no call allocates anything.  The
 * per-block minima live in a static 512 KiB scratch array of the library,
 * one per GPU (held until the process ends), so lattices of at most 2^25
 * sites are accepted (larger: MCG_EINVAL; use mcg_center_project).
 * min_margin NULL: nothing is copied back and the stream is not
 * synchronised, so the call can be captured into a graph.  MCG_OPT_CHECK is
 * not applied (the check would need scratch).  All calls on one GPU share
 * that array and keep the last call's contents: calls that overlap on one
 * GPU (other streams, other contexts, other threads) race. */
mcg_status mcg_center_project_noalloc(mcg_ctx *ctx, const mcg_field *U, const mcg_gauge *G,
                                      int8_t *Z, double *min_margin, void *stream);
/* P-vortex plaquettes of Z: n = (m_mu(x) + m_nu(x+mu) - m_mu(x+nu) - m_nu(x)) mod 3
 * for mu < nu; counts of n != 0 in total, per plane (0,1),(0,2),(0,3),(1,2),
 * (1,3),(2,3), and per charge n = 1, 2 (host outputs; per_plane/per_charge
 * nullable). */
mcg_status mcg_count_vortices(mcg_ctx *ctx, const int8_t *Z, mcg_dims d, int64_t *total,
                              int64_t *per_plane, int64_t *per_charge, void *stream);

/* ---- vortex-only and vortex-removed fields, Wilson loops (Sec. III.B) ------------- */
/* The projected centre field splits a fixed field as U^G = Z (Z^dagger U^G).
 * mode MCG_VORTEX_ONLY:    out_mu(x) = z(m_mu(x)) 1
 * mode MCG_VORTEX_REMOVED: out_mu(x) = conj(z(m_mu(x))) G(x) U_mu(x) G(x+mu)^dagger
 * with z(m) = exp(2 pi i m / 3), Z as written by mcg_center_project (device,
 * [4][V]), G nullable (identity).  out has U's extents and precision, may
 * alias U, and is written in U's layout (products formed in FP64). */
#define MCG_VORTEX_ONLY 0
#define MCG_VORTEX_REMOVED 1
mcg_status mcg_vortex_field(mcg_ctx *ctx, const mcg_field *U, const mcg_gauge *G, const int8_t *Z,
                            int32_t mode, mcg_field *out, void *stream);
/* Wilson loops W[i][k-1][T-1] (host, nvec * rmax * tmax doubles): the mean
 * over all sites of Re tr(loop)/3 for time extent T = 1..tmax and the
 * spatial side made of k = 1..rmax copies of a staircase path for the
 * integer vector vec[3 i .. 3 i + 2] (host), averaged over the distinct
 * images of that path under the 48 axis permutations and reflections.
 * The staircase takes |v_0| + |v_1| + |v_2| unit steps; each step goes
 * along the axis with steps left whose (steps taken + 1/2) / |v_axis| is
 * smallest, the lower axis on a tie.  Requires 1 <= tmax <= L[3],
 * 0 < |v|_1 <= 24 with |v_j| <= 8, and rmax * max_j |v_j| <= min(L[0], L[1],
 * L[2]); sums in FP64, deterministic.  Synchronises the stream. */
mcg_status mcg_wilson_loops(mcg_ctx *ctx, const mcg_field *U, int32_t nvec, const int32_t *vec,
                            int32_t rmax, int32_t tmax, double *W, void *stream);

/* ---- gradient of the smeared-field functional ---------------------------------- */
/* L = R(S_n(U; rho, eps)^{G*}) at fixed G* (at a converged maximum this is
 * dL/dtheta of the fixed functional by the envelope theorem).  Returns the
 * ambient gradient gradU = dL/dRe U + i dL/dIm U (same layout and precision
 * as U) and host scalars L, dL/drho, dL/deps, summed on the device in a
 * fixed order (the same bits on every call).  Smeared fields are
 * checkpointed every ckpt_every steps and recomputed between checkpoints,
 * except the last segment's, which the forward pass keeps.
 * Device workspace held by the context: with c = ckpt_every (n if <= 0 or
 * > n) and m = (eps == 1 ? 1 : 2), ceil(n/c) * (1 + m) + (c - 1) * (1 + m) + 5
 * fields of U's size (the checkpoints, one segment's fields, and staple sums);
 * if that cannot be allocated (or exceeds MCG_OPT_SCRATCH_LIMIT_MIB), ceil(n/c)
 * + (c - 1) + 5 fields, the staples then formed again in the adjoint (the same
 * results, more time). */
mcg_status mcg_smear_mcg_backward(mcg_ctx *ctx, const mcg_field *U, double rho, double eps,
                                  int32_t n, const mcg_gauge *Gstar, int32_t ckpt_every,
                                  mcg_field *gradU, double *loss, double *dRho, double *dEps,
                                  void *stream);

#ifdef __cplusplus
}
#endif
#endif
