/*
 * berryhip -- batched Wilson-loop engine for MI355X (gfx950).
 *
 * C ABI of the hot path: Bloch Hamiltonians from a hopping list, batched
 * Hermitian eigensolver, Wilson loops, nested Wilson loops and
 * spin-resolved Wilson loops. The method is that of BerryEasy
 * (arXiv:2312.13051); each entry point names the passage it implements.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Complex numbers are interleaved (re, im) pairs: "c128" is double2,
 *   "c64" is float2. Matrices are column-major with a leading dimension.
 * - Pointers suffixed _h are host memory; all other array pointers are
 *   device memory owned by the caller. The library never frees caller memory.
 * - Every call is asynchronous on the given stream unless its comment says
 *   it synchronizes. Outputs are valid once the stream has completed. Calls
 *   that synchronize read convergence counts back to the host between
 *   launches, only to stop their iterations early.
 * - HIP graph capture: while the stream is being captured, be_build_hk,
 *   be_eigh_batched, be_wilson_loop, be_plaquette_flux(_noalloc),
 *   be_spin_resolved_wilson and be_spin_sectors read nothing back: their
 *   Newton-Schulz iterations run the whole fixed schedule (8 steps for the
 *   eigenvectors, 51 for the polar factors) with converged matrices skipped
 *   on the device, so a replay reproduces the uncaptured results exactly.
 *   The workspace must not grow under capture (BE_ENOMEM): run the same call
 *   once outside capture first. be_spin_resolved_wilson and be_spin_sectors
 *   then take m_dn_h as input (the sector sizes of an earlier uncaptured
 *   call; at most 256 systems) and flag PSO_GAP where a system's actual size
 *   differs. be_nested_wilson and be_hk_plan_create cannot be captured.
 * - Return value: BE_OK (0) or a negative error code; be_last_error() gives
 *   text. Argument errors are detected on the host before any launch.
 * - Physics conditions (closed gaps, singular overlaps, ...) are never
 *   errors: they set bits in a per-item status word (BE_ST_*). A result is
 *   valid when its status is 0.
 * - A context (be_ctx) owns a device workspace that grows on demand; growing
 *   synchronizes the stream once. Use one context per host thread.
 *
 * k-point grids ("U-grids")
 * ------------------------
 * Wilson-loop calls take the selected eigenvectors of every point of a
 * k-plane, U[s][i][j] for system s, transverse index i < n_perp and loop
 * index j < n_par, at kappa = k0 + (j/n_par) e_par + (i/n_perp) e_perp
 * (fractional coordinates of the (super)cell reciprocal basis). Matrix
 * (s, i, j) starts at element ((s*n_perp + i)*n_par + j) * u_stride of U,
 * is N x m with leading dimension ldu. The loop closes on itself: the point
 * j = n_par is j = 0 (lattice gauge, H(kappa + G) = H(kappa)).
 */
#ifndef BERRYHIP_H
#define BERRYHIP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define BE_OK 0
#define BE_EINVAL (-1)   /* bad argument: null pointer, size out of range   */
#define BE_ENOMEM (-2)   /* device workspace allocation failed              */
#define BE_EHIP (-3)     /* a HIP runtime call failed (text in last_error)  */
#define BE_ENOTIMPL (-4) /* combination of options not implemented          */

/* ---- element types ---- */
#define BE_C128 0 /* complex double */
#define BE_C64 1  /* complex float  */

/* ---- precision of the eigensolver ---- */
#define BE_FP64 0       /* everything in FP64                                   */
#define BE_MIXED_FP32 1 /* FP32 Householder reduction and back-transformation on
                           MFMA with FP32 accumulation; FP64 tridiagonal solve,
                           FP64 re-orthonormalization of the eigenvectors       */
#define BE_MIXED_FP32_REFINED 2 /* BE_MIXED_FP32 for all N bands of an FP32
                           copy of H, then an FP64 correction of the selected
                           bands' subspace from the other bands (first order
                           in the FP32 error, so that error enters squared),
                           FP64 Rayleigh-quotient eigenvalues and FP64
                           orthonormalization; H (BE_C128) is not modified   */
#define BE_MIXED_BF16X 3 /* BE_MIXED_FP32 with the trailing updates and the
                           back-transformation on the bf16 matrix cores: each
                           FP32 operand split into two bf16 parts, three
                           products per real product (x_hi y_hi + x_hi y_lo +
                           x_lo y_hi), FP32 accumulation; ~2^-16 relative error
                           per product instead of FP32's 2^-24. Accuracy is
                           stated, not assumed: be_eigh_batched (BE_C64 input)
                           and the spin paths' eigensolver of the projected
                           spin operator accept it                          */

/* ---- overlap mode ---- */
#define BE_OVL_POLAR 0 /* each overlap replaced by its unitary polar factor */
#define BE_OVL_RAW 1   /* raw overlaps, as printed in eq. 2                 */

/* ---- status bits (per matrix or per system) ---- */
#define BE_ST_GAP_CLOSED 1u         /* selected bands touch their neighbours       */
#define BE_ST_OVERLAP_SINGULAR 2u   /* an overlap has smallest singular value < 1e-8 (polar mode: the
                                        Newton-Schulz iteration needs more steps than sigma = 1e-8 does) */
#define BE_ST_WINDING_UNRESOLVED 4u /* transverse step of Phi > 0.8 pi or non-integer */
#define BE_ST_PSO_GAP 8u            /* projected spin spectrum touches 0 or its sign
                                       count varies over the grid                  */
#define BE_ST_WANNIER_GAP 16u       /* a Wilson phase sits on a sector window edge,
                                       or the sector size varies                   */
#define BE_ST_NONCONVERGED 32u      /* an iteration hit its cap                     */
#define BE_ST_NAN_INF 64u           /* non-finite input or intermediate             */

typedef struct be_ctx be_ctx;
typedef struct be_hk_plan be_hk_plan;

/* Hopping list of one (super)cell, host memory.
 * Entry e is the amplitude t[e] (interleaved re, im) from orbital j[e] in the
 * cell at integer lattice vector R[e*dim .. e*dim+dim-1] to orbital i[e] in
 * the home cell. The list must be Hermitian: after adding duplicate
 * (i, j, R) keys, every (i, j, R, t) must have the partner (j, i, -R, conj t)
 * (relative tolerance 1e-12). 1 <= dim <= 3, 0 <= i, j < N. */
typedef struct {
  int32_t N;
  int32_t dim;
  int64_t nnz;
  const int32_t *i;
  const int32_t *j;
  const int32_t *R;
  const double *t;
} be_hoplist;

/* Create a context on HIP device `device` (the device becomes current on
 * the calling thread). */
int be_create(be_ctx **ctx, int device);
/* Destroy a context and free its workspace. Waits for the device. */
int be_destroy(be_ctx *ctx);
/* Text of the last error on this context (never NULL). */
const char *be_last_error(const be_ctx *ctx);
/* Bytes of device workspace currently held by the context. */
size_t be_workspace_bytes(const be_ctx *ctx);

/* Row (a1) -- model to device hopping list.
 * Packs n_sys hopping lists: merges duplicate (i, j, R) keys, checks that
 * each list is Hermitian, keeps the upper triangle (i <= j) sorted by
 * (j, i, R) and uploads it. Synchronous. The plan is independent of later
 * calls and may be reused for any number of k-points.
 * Errors: BE_EINVAL (bad sizes, index out of range, non-Hermitian list). */
int be_hk_plan_create(be_ctx *ctx, const be_hoplist *sys_h, int32_t n_sys, be_hk_plan **plan);
int be_hk_plan_destroy(be_hk_plan *plan);
/* Orbital count of system s of a plan (or -1). */
int32_t be_hk_plan_N(const be_hk_plan *plan, int32_t s);

/* Row (a2) -- Bloch Hamiltonians (Sec. II-A: Bloch sum with periodic
 * boundary conditions at the (super)cell period; supercells use the
 * reciprocal basis of the supercell, the 2pi -> 2pi/L rule).
 * Builds n_sys_call * n_kap matrices: matrix q = s_local*n_kap + k belongs to
 * system sys_first + s_local of the plan and to the fractional k-point
 * kappa[3k .. 3k+2] (device, float64; components beyond the system's dim are
 * ignored):
 *   H_q[a, b] = sum_e t_e exp(2 pi i kappa_k . R_e) over entries (a, b, R_e).
 * Matrix q is written at H + q*mat_stride elements, column-major with
 * leading dimension ld >= N; rows N..ld-1 are left untouched. Only the upper
 * triangle is summed; the lower triangle is its exact conjugate and the
 * diagonal is exactly real, so H is bitwise Hermitian, and every element is
 * summed by one thread in a fixed order, so H is deterministic. All systems
 * of one call must have the same N. dtype: BE_C128 or BE_C64 (phases and sums
 * in FP64, one rounding at the store). */
int be_build_hk(be_ctx *ctx, const be_hk_plan *plan, int32_t sys_first, int32_t n_sys_call, const double *kappa,
                int32_t n_kap, void *H, int64_t mat_stride, int32_t ld, int32_t dtype, hipStream_t stream);

/* Rows (a3)-(a5) -- batched Hermitian eigensolver (Sec. I: exact
 * diagonalization at many k-points; the selected bands, eq. 2).
 * n_mat matrices of order N (H + q*mat_stride, leading dimension ld, BE_C128
 * for BE_FP64 and BE_MIXED_FP32_REFINED, BE_C64 for BE_MIXED_FP32). Only the
 * lower triangle and the diagonal are read (the diagonal's imaginary parts
 * are taken as zero); the upper triangle is ignored. H is overwritten (its
 * columns hold the Householder vectors afterwards; the upper triangle is left
 * undefined), except with BE_MIXED_FP32_REFINED, which works on copies.
 * BE_MIXED_FP32_REFINED: the mixed path for all N bands of an FP32 copy of
 * H; then, with H in FP64, for each selected band j and each other band i,
 * s_ij = v_i^H H u_j and p_ij = v_i^H u_j (FP64 MFMA GEMMs) give the error of
 * u_j along v_i, (s_ij - lambda_j p_ij) / (lambda_i - lambda_j), which is
 * removed (U += V F); U is then orthonormalized by Newton-Schulz in FP64 and
 * the eigenvalues are the Rayleigh quotients u_j^H H u_j / u_j^H u_j of the
 * uncorrected vectors. The FP32 error of the subspace enters squared: the
 * projector U U^H agrees with the FP64 path's to about 1e-12 where the
 * window is separated from the other bands by a gap well above 1e-6 ||H||;
 * single columns inside the window are eigenvectors to the FP32 path's
 * accuracy only; the eigenvalues are Rayleigh quotients of those columns,
 * second order in their error (typically within 1e-12 ||H||, but a pair of
 * nearly equal eigenvalues inside the window can keep the FP32 path's error,
 * ~1e-7 ||H||; eigenvalues lo-1 and hi: the FP32 path's). Workspace per matrix: about
 * 40 N^2 + 32 N m + 32 (N - m) m bytes besides the mixed path's for m = N.
 * Steps: blocked Householder reduction to real tridiagonal form (panel
 * kernel whose matrix-vector products read the lower triangle once per
 * column + MFMA rank-2k trailing updates of the lower triangle), FP64 bisection for eigenvalues
 * [lo-1, hi], FP64 inverse iteration for bands [lo, hi) (Cholesky QR inside
 * clusters of eigenvalues closer than 1e-12 ||T||), FP64 Newton-Schulz
 * orthonormalization of the tridiagonal eigenvectors, back-transformation
 * with compact-WY blocks on MFMA (FP32 on the mixed path).
 * Outputs:
 *   evals[q*(m+2) + 0]     eigenvalue lo-1 (NaN if lo == 0)
 *   evals[q*(m+2) + 1 + c] eigenvalue lo+c, c < m = hi-lo
 *   evals[q*(m+2) + m + 1] eigenvalue hi   (NaN if hi == N)
 *   U + q*u_stride: N x m eigenvectors (c128), leading dimension ldu >= N;
 *   status[q]: BE_ST_GAP_CLOSED if min gap at lo or hi < 1e-9 max(1, |lambda|max),
 *              BE_ST_NAN_INF, BE_ST_NONCONVERGED.
 * Inside a cluster of (nearly) degenerate eigenvalues the columns are some
 * orthonormal basis of the cluster's invariant subspace; the projector U U^H
 * is the gauge-invariant output. Workspace: the context's, grown on demand;
 * batches are processed in equal sub-batches of at most 4 GiB of it, or, for
 * large N where 4 GiB holds fewer matrices than the device runs at once, of
 * up to that many within 48 GiB (at most half the free device memory).
 * Synchronizes the stream once per sub-batch and orthonormalization step
 * (the largest Gram error of Z is read back).
 * Size limit: the panel vectors (2N complex values) and the tridiagonal
 * solver's arrays ((4N + m + 4) doubles; (3N + m) doubles and N + 1 + 2m
 * ints) are held in LDS and must fit in 160 KiB, which allows N up to about
 * 4000 at m = N/2; a larger order returns BE_EINVAL. */
int be_eigh_batched(be_ctx *ctx, void *H, int32_t dtype, int32_t N, int32_t ld, int64_t mat_stride,
                    int32_t n_mat, int32_t band_lo, int32_t band_hi, int32_t precision, double *evals,
                    void *U, int32_t ldu, int64_t u_stride, uint32_t *status, hipStream_t stream);

/* Matrices of order N that the eigensolver's panel kernel keeps resident on
 * the device at once for `precision` (one workgroup per matrix; depends on
 * the panel thread count chosen for N). be_eigh_batched processes a batch in
 * equal sub-batches of whole such rounds where its workspace cap allows, so a
 * batch of a multiple of *round matrices fills every round. Host-only query
 * (an occupancy calculation), no device work. */
int be_eigh_round(be_ctx *ctx, int32_t N, int32_t precision, int64_t *round);

/* Rows (a6)-(a8) -- Wilson loop over a U-grid (eq. 2 with the path ordering
 * of eq. 1, hybrid centres of eq. 3, Chern winding of eq. 6).
 *   F_j = U(kappa_{j+1})^H U(kappa_j), j < n_par (closing to j = 0);
 *   mode BE_OVL_POLAR replaces F_j by its unitary polar factor (FP64);
 *   W_i = F_{n_par-1} ... F_0;   theta_i = arg eig(W_i) in (-pi, pi],
 *   ascending;  Phi_i = sum_n theta_{i,n} mod 2pi;
 *   winding = (1/2pi) sum_i wrap(Phi_{(i+1) mod n_perp} - Phi_i).
 * U is c128. Outputs (device): theta [n_sys][n_perp][m], phi [n_sys][n_perp],
 * winding [n_sys], status [n_sys] (OVERLAP_SINGULAR, WINDING_UNRESOLVED,
 * NONCONVERGED). In polar mode, synchronizes the stream once per
 * Newton-Schulz iteration (the largest Gram error is read back). */
int be_wilson_loop(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride,
                   int32_t n_sys, int32_t n_par, int32_t n_perp, int32_t mode, double *theta, double *phi,
                   int32_t *winding, uint32_t *status, hipStream_t stream);

/* Row (a9) -- nested Wilson loop (Sec. III, eq. 8).
 * The Wilson loop of each transverse line is diagonalized at base point 0;
 * its eigenvectors with x = theta/2pi in the open window (win_lo, win_hi)
 * form the Wannier sector (size s). They are carried to every base point j
 * by the path-ordered overlaps, w_{i,j} = U_{i,j} nu_S^{(i,j)}, and a second
 * Wilson loop runs along the transverse direction at every j:
 *   nested_theta [n_sys][n_par][m] (first s entries valid, ascending),
 *   p [n_sys][n_par] = sum nested_theta / 2pi in (-1/2, 1/2],
 *   p_mean [n_sys] = mean of p unwrapped along j, reduced to [0, 1),
 *   s_out_h [n_sys] (host) sector sizes, status [n_sys] (WANNIER_GAP, ...).
 * Synchronizes the stream: the sector size is read back, and in polar mode
 * each Newton-Schulz iteration reads back its Gram error. */
int be_nested_wilson(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride,
                     int32_t n_sys, int32_t n_par, int32_t n_perp, int32_t mode, double win_lo, double win_hi,
                     double *nested_theta, double *p, double *p_mean, int32_t *s_out_h, uint32_t *status,
                     hipStream_t stream);

/* Row (a10) -- spin-resolved Wilson loop (Sec. IV; sign convention of Sec. V).
 * Projected spin operator in the occupied space, A = U^H S U with
 * S = diag(spin_diag[s*N .. s*N+N-1]) (device, float64), eigh(A) = (mu, Q);
 * V_minus = U Q[:, mu < 0] (spin down), V_plus = U Q[:, mu > 0] (spin up);
 * Wilson loop and winding of each sector:
 *   pso_evals [n_sys][n_perp][n_par][m] (ascending mu),
 *   theta_dn [n_sys][n_perp][m], theta_up [n_sys][n_perp][m] (first
 *   m_dn_h[s] resp. m - m_dn_h[s] entries valid), C_dn, C_up [n_sys] (int32),
 *   C_s [n_sys] = (C_up - C_dn)/2, m_dn_h [n_sys] (host), status [n_sys]
 *   (PSO_GAP if min |mu| < 1e-6 or the count of mu < 0 varies).
 * precision selects the eigensolver of A: BE_FP64, or BE_MIXED_FP32 (A
 * rounded to c64, FP32 reduction and back-transformation, FP64 tridiagonal
 * solve and orthonormalization), BE_MIXED_BF16X (the same with split-bf16
 * products in its GEMMs); BE_MIXED_FP32_REFINED (for U from the refined
 * eigensolver) takes the FP64 solver; A, U and everything after are FP64.
 * Synchronizes the stream: the sector sizes are read back, and the
 * eigensolver and the polar steps read back their convergence. */
int be_spin_resolved_wilson(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride,
                            int32_t n_sys, int32_t n_par, int32_t n_perp, int32_t mode, int32_t precision,
                            const double *spin_diag,
                            double *pso_evals, double *theta_dn, double *theta_up, int32_t *C_dn, int32_t *C_up,
                            double *C_s, int32_t *m_dn_h, uint32_t *status, hipStream_t stream);

/* Berry flux per plaquette (the coupling-matrix method of the disordered
 * quadrupolar-insulator example, Sec. IV: the zone is cut into plaquettes and
 * the flux through each is integrated along its closed boundary; applied
 * there to the occupied space and to its spin sectors). On a U-grid (the
 * layout above, U c128), with link phases
 *   phi_par(i, j)  = arg det(U(i, j+1)^H U(i, j)),
 *   phi_perp(i, j) = arg det(U(i+1, j)^H U(i, j))   (both periodic),
 * the flux through the plaquette with corners (i, j), (i, j+1), (i+1, j+1),
 * (i+1, j) is
 *   F(i, j) = wrap(phi_par(i+1, j) - phi_par(i, j) + phi_perp(i, j) - phi_perp(i, j+1))
 * in (-pi, pi], oriented so that its sum over the zone is 2 pi times the
 * winding of eq. 6 (be_wilson_loop's on the same grid). Outputs (device):
 *   flux [n_sys][n_perp][n_par], total [n_sys] = sum F / 2 pi (an integer
 *   to rounding: every link enters two plaquettes with opposite signs),
 *   chern [n_sys] = the nearest integer, status [n_sys]:
 *   OVERLAP_SINGULAR if some link has smallest singular value < 1e-8
 *   (its phase is then undetermined; the Wilson loop's criterion for its
 *   overlaps). |det| never exceeds sigma_min, so |det| >= 1e-8 proves a link
 *   regular; other links get an estimate of sigma_min from their LU factors
 *   (inverse iteration, an upper bound that converges to it),
 *   WINDING_UNRESOLVED if some |F| > 0.8 pi or |total - chern| > 1e-6
 *   (the grid is too coarse for the flux), NAN_INF (non-finite flux; chern 0).
 * m = 0 gives zero flux; m > 2544 is rejected (BE_EINVAL). The links of one direction for as many systems as
 * fit in about 1 GiB are held in the context's workspace (at least one
 * system, n_par*n_perp*m*m*16 bytes). */
int be_plaquette_flux(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride,
                      int32_t n_sys, int32_t n_par, int32_t n_perp, double *flux, int32_t *chern, double *total,
                      uint32_t *status, hipStream_t stream);

/* The plaquette flux of be_plaquette_flux without any device allocation,
 * for callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc. Same arguments, layouts,
 * results and errors as be_plaquette_flux. Its scratch (the link matrices of
 * one direction for as many systems per pass as fit, and 32 bytes per
 * k-point) is a fixed array of BE_NOALLOC_SCRATCH_BYTES inside the library,
 * one per device, held until the process ends; its address is looked up
 * when a context is created. A call whose single system needs more
 * (n_par*n_perp*m*m*16 bytes plus 32 per k-point, rounded) returns BE_EINVAL
 * before any launch. Every call on a device shares that device's array and
 * leaves its contents behind (nothing in it is read before being written):
 * calls that overlap in time on one device (other streams or host threads)
 * race on it and give wrong results. */
#define BE_NOALLOC_SCRATCH_BYTES (128u << 20)
int be_plaquette_flux_noalloc(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride,
                              int32_t n_sys, int32_t n_par, int32_t n_perp, double *flux, int32_t *chern,
                              double *total, uint32_t *status, hipStream_t stream);

/* Spin-sector bases of the occupied space (Sec. IV): the projected spin
 * operator and its eigendecomposition exactly as in be_spin_resolved_wilson,
 * on n_k_sys k-points per system (U matrix (s, k) at (s*n_k_sys + k)*u_stride),
 * and V = U Q with the columns in ascending mu: the first m_dn_h[s] columns
 * span the spin-down sector (mu < 0), the rest the spin-up sector.
 *   pso_evals [n_sys][n_k_sys][m], V + (s*n_k_sys + k)*v_stride: N x m
 *   (c128, leading dimension ldv >= N; V must not overlap U), m_dn_h [n_sys]
 *   (host), status [n_sys] (PSO_GAP, NAN_INF, NONCONVERGED).
 * Sector flux maps: be_plaquette_flux on V (m_dn_h[s] columns) and on
 * V + m_dn_h[s]*ldv (m - m_dn_h[s] columns), with ldu = ldv, u_stride = v_stride.
 * Synchronizes the stream: the sector sizes are read back, and the
 * eigensolver reads back its convergence. */
int be_spin_sectors(be_ctx *ctx, const void *U, int32_t N, int32_t m, int32_t ldu, int64_t u_stride, int32_t n_sys,
                    int32_t n_k_sys, int32_t precision, const double *spin_diag, double *pso_evals, void *V,
                    int32_t ldv, int64_t v_stride, int32_t *m_dn_h, uint32_t *status, hipStream_t stream);

/* Launch timing (tracing aid). While enabled, every library launch is
 * bracketed by a pair of hipEvents recorded on its own stream, keyed by the
 * kernel or GEMM call-site name ("hk_scatter", "hetrd_panel", "her2k",
 * "tridiag_eig", "unmtr", "overlap", "polar", "chain", "unitary_eig", ...).
 * be_profile_enable resets all counters. Queries synchronize on the
 * recorded events and return the summed duration and the launch count.
 * be_profile_names writes the comma-separated list of names seen so far. */
int be_profile_enable(be_ctx *ctx, int on);
int be_profile_query(be_ctx *ctx, const char *name, double *total_ms, int64_t *launches);
int be_profile_names(be_ctx *ctx, char *buf, size_t len);

/* Tuning knobs: algorithm variants with identical results up to rounding,
 * chosen per context (by measurement). Unknown knob names and out-of-range
 * values return BE_EINVAL. Knobs:
 *   "hetrd_panel_threads" threads per matrix of the panel kernel: 256, 512
 *                       or 1024 (default 512: two matrices per compute
 *                       unit overlap one's serial reflector steps with the
 *                       other's matrix-vector product).
 *   "hetrd_panel_loads"  loads in flight per lane in the matrix-vector
 *                       product of the 512-thread FP32 panel kernel (the
 *                       mixed paths): 4 (six waves resident per SIMD) or 8
 *                       (four waves); 0 (default) takes 8 from order 960 on.
 *                       The other panel kernels have one form each (FP64
 *                       and 256 threads: 4; 1024-thread FP32: 8), which
 *                       this knob leaves unchanged.
 *   "tri_bisect_max_iter" a debug cap: bisection steps per eigenvalue after
 *                       the multisection, 1 .. 128 (default 128, which never
 *                       binds). A cap that stops an eigenvalue short of its
 *                       tolerance sets BE_ST_NONCONVERGED on its matrix (a
 *                       way to exercise that flag from the host); no
 *                       per-order settings (be_tune_set_orders: BE_EINVAL). */
int be_tune_set(be_ctx *ctx, const char *knob, int32_t value);
int be_tune_get(be_ctx *ctx, const char *knob, int32_t *value);

/* Per-order settings of a knob, as an autotuner writes them: value applies to
 * matrices of order N in [n_lo, n_hi] on the paths of `precision` (BE_FP64:
 * the FP64 reduction; BE_MIXED_FP32 or BE_MIXED_FP32_REFINED: the FP32
 * reduction; -1: both); settings made later take precedence over earlier
 * ones, and be_tune_set's value applies where none matches. be_tune_clear
 * drops a knob's per-order settings and restores its default.
 * (The package's tune.py measures these settings on the device and stores
 * them as JSON; Context.load_tuning applies a stored table.) */
int be_tune_set_orders(be_ctx *ctx, const char *knob, int32_t n_lo, int32_t n_hi, int32_t precision, int32_t value);
int be_tune_clear(be_ctx *ctx, const char *knob);

/* Utility kernel exposed for tests: batched complex GEMM on MFMA,
 *   C_q = alpha op(A_q) op(B_q) + beta C_q,   op = 'N' (none) or 'C'
 * (conjugate transpose), c128, strided batches (element strides). */
int be_zgemm_strided(be_ctx *ctx, char opA, char opB, int32_t M, int32_t Ncol, int32_t K, const double *alpha2_h,
                     const void *A, int32_t lda, int64_t strideA, const void *B, int32_t ldb, int64_t strideB,
                     const double *beta2_h, void *C, int32_t ldc, int64_t strideC, int32_t batch, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* BERRYHIP_H */
