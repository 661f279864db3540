/*
 * mcg_oracle.h -- plain, slow, FP64 CPU oracle for stout-preconditioned
 * Maximal Center Gauge (MCG) fixing in SU(3)
 * (O Cais, Kamleh, Langfeld, Lasscock, Leinweber, Moran, Sternbeck,
 *  von Smekal, "Preconditioning Maximal Center Gauge with Stout Link
 *  Smearing in SU(3)", arXiv:0807.0264).
 *
 * THIS IS TEST INFRASTRUCTURE.  It exists only to check the HIP library.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * Layout (the "interchange" layout):
 *   site index  i = x + Lx*(y + Ly*(z + Lz*t)), periodic in all directions
 *   links       U[(i*4 + mu)*9 + 3*row + col]   complex double
 *   gauge       G[i*9 + 3*row + col]            complex double
 *   center      Z[i*4 + mu]                     int8, m in {-1,0,1}
 * All extents must be even (>= 2) so that every link joins an even and an
 * odd site (checkerboard).
 *
 * Readings where the paper is silent:
 *   - gauge transform  U^G_mu(x) = G(x) U_mu(x) G(x+mu)^dagger
 *   - MCG local update: minorise-maximise step over the SU(2) subgroups
 *     (0,1),(1,2),(0,2) with binomial over-relaxation omega
 *   - one "iteration" = one full even+odd sweep; stop when
 *     R_s - R_{s-1} < tol; G re-unitarised every reunit_every sweeps
 *   - centre phase: argmax over m of Re(t e^{-2 pi i m/3}), ties to
 *     m = 0, then +1, then -1
 *
 * Pins (closed forms, invariants, brute force) live in tests/test_oracle_*.py.
 */
#ifndef MCG_ORACLE_H
#define MCG_ORACLE_H

#include <stdint.h>
#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef double _Complex ocx;

typedef struct {
  double R;        /* functional after the final re-unitarisation          */
  double dR;       /* last R_s - R_{s-1}                                    */
  double theta;    /* stationarity residual (1/V) sum_x |TA X(x)|_F^2       */
  int32_t sweeps;  /* sweeps done in this call                              */
  int32_t status;  /* 0 = converged, 1 = max_sweeps reached                 */
} or_fix_result;

/* ---- lattice ------------------------------------------------------------ */
int64_t or_volume(const int32_t L[4]);

/* ---- SU(3) helpers exported for tests ---------------------------------- */
void or_reunit(ocx M[9]);
/* exp of a traceless anti-Hermitian 3x3 A by diagonalising Q = -iA */
void or_exp_su3_eigen(const ocx A[9], ocx E[9]);
/* exp of a general n x n matrix (n <= 6) by scaling-and-squaring Taylor */
void or_exp_taylor(const ocx *A, int n, ocx *E);

/* ---- gauge transform and functional (Sec. II.A) ------------------------- */
void or_apply_gauge(const int32_t L[4], const ocx *U, const ocx *G, ocx *out);
double or_functional(const int32_t L[4], const ocx *U);
double or_plaquette(const int32_t L[4], const ocx *U);
double or_wilson_loop(const int32_t L[4], const ocx *U, int r, int t);
void or_polyakov(const int32_t L[4], const ocx *U, ocx *P);

/* ---- smearing (Sec. II.B) ----------------------------------------------- */
/* staple sum C_mu(x) with plaquette weight wp and rectangle weight wr
 * (over-improved stout: wp = (5-2eps)/3, wr = -(1-eps)/12), times rho */
void or_staple_sum(const int32_t L[4], const ocx *U, int64_t site, int mu,
                   double rho, double eps, ocx C[9]);
/* plain stout staples written out on their own (plaquettes only) */
void or_stout_staple_plain(const int32_t L[4], const ocx *U, int64_t site,
                           int mu, double rho, ocx C[9]);
void or_smear_link(const int32_t L[4], const ocx *U, int64_t site, int mu,
                   double rho, double eps, ocx out[9]);
void or_smear_step(const int32_t L[4], const ocx *U, ocx *out, double rho,
                   double eps);
void or_smear(const int32_t L[4], const ocx *U, ocx *out, double rho,
              double eps, int n);

/* ---- MCG fixing (Sec. II.A) --------------------------------------------- */
/* local update from the eight link matrices touching a site:
 * M[k] = W_k(x) for k < 4, M[4+mu] = W_mu(x-mu)^dagger               */
void or_site_g(const ocx M[8 * 9], double omega, ocx g[9]);
void or_site_g_hits(const ocx M[8 * 9], double omega, int hits, ocx g[9]);
void or_site_g_exact(const ocx M[8 * 9], double omega, int hits, ocx g[9]);
void or_sphere_max(const double Q[16], const double h[4], double a[4]);
void or_site_g_at(const int32_t L[4], const ocx *W, int64_t site,
                  double omega, ocx g[9]);
void or_halfsweep(const int32_t L[4], ocx *W, ocx *G, int parity,
                  double omega);
double or_theta(const int32_t L[4], const ocx *W);
int or_mcg_fix(const int32_t L[4], const ocx *U, ocx *G, double tol,
               int32_t max_sweeps, double omega, int32_t reunit_every,
               int32_t start_sweep, double *traj, or_fix_result *res);
void or_halfsweep_hits(const int32_t L[4], ocx *W, ocx *G, int parity,
                       double omega, int hits);
void or_halfsweep_v(const int32_t L[4], ocx *W, ocx *G, int parity,
                    double omega, int hits, int exact);
int or_mcg_fix_v(const int32_t L[4], const ocx *U, ocx *G, double tol,
                 int32_t max_sweeps, double omega, int32_t reunit_every,
                 int32_t start_sweep, int32_t hits, int32_t stop_every,
                 int32_t exact, double *traj, or_fix_result *res);

/* ---- centre projection and P-vortices (Sec. II.A) ------------------------ */
void or_center_project(const int32_t L[4], const ocx *U, const ocx *G,
                       int8_t *Z, double *margin);
void or_count_vortices(const int32_t L[4], const int8_t *Z, int64_t *total,
                       int64_t per_plane[6], int64_t per_charge[2],
                       int8_t *n_out);

/* ---- vortex-only / vortex-removed fields, Wilson loops (Sec. III.B) ------ */
/* mode 0: out_mu(x) = z(m_mu(x)) 1 (the projected centre field);
 * mode 1: out_mu(x) = conj(z(m_mu(x))) U^G_mu(x) (P-vortices removed);
 * z(m) = exp(2 pi i m / 3); G may be NULL (identity). */
void or_vortex_field(const int32_t L[4], const ocx *U, const ocx *G,
                     const int8_t *Z, int mode, ocx *out);
/* mean over all sites x of Re tr(loop)/3, the loop running along the spatial
 * steps (+-(axis+1), axis < 3) from x, then t steps up in time, back along the
 * spatial steps reversed, and t steps down in time */
double or_wilson_path(const int32_t L[4], const ocx *U, const int *spatial,
                      int n, int t);

/* ---- smeared-field MCG loss and its FP64 adjoint ------------------------ */
double or_smear_loss(const int32_t L[4], const ocx *U, double rho, double eps,
                     int n, const ocx *Gstar);
void or_smear_loss_grad(const int32_t L[4], const ocx *U, double rho,
                        double eps, int n, const ocx *Gstar, int ckpt_every,
                        ocx *gradU, double *dRho, double *dEps, double *loss, double *absEps);
/* one smearing step: tangent (forward mode) and cotangent (reverse mode) */
void or_step_jvp(const int32_t L[4], const ocx *U, const ocx *dU, double rho,
                 double eps, ocx *dOut);
void or_step_vjp(const int32_t L[4], const ocx *U, const ocx *gOut,
                 double rho, double eps, ocx *gU, double *dRho, double *dEps, double *absEps);

#ifdef __cplusplus
}
#endif
#endif
