/*
 * shenhip -- batched direct solvers for the wall-normal Shen-Galerkin
 * Helmholtz and biharmonic systems of a Fourier/Chebyshev channel solver
 * (Mortensen, "A spectral-Galerkin turbulent channel flow solver for
 * large-scale simulations", Sec. 3 and Sec. 4), on AMD Instinct MI355X
 * (gfx950).
 *
 * Problem (one independent system per Fourier wavenumber pair (kx, kz)):
 *
 *   Helmholtz  (Shen Dirichlet basis  phi_k = T_k - T_{k+2}, k < n = N-2):
 *       (S + alpha_w B) u_w = f_w,
 *       S_kj = -(phi_j'', phi_k)_sigma,  B_kj = (phi_j, phi_k)_sigma
 *   biharmonic (Shen biharmonic basis phi_k = T_k - 2(k+2)/(k+3) T_{k+2}
 *                                       + (k+1)/(k+3) T_{k+4}, k < n = N-4):
 *       (Q + a_w A + b_w B) u_w = f_w,
 *       Q_kj = (phi_j'''', phi_k)_sigma, A_kj = (phi_j'', phi_k)_sigma,
 *       B_kj = (phi_j, phi_k)_sigma
 *
 * These are the paper's Crank-Nicolson Helmholtz and biharmonic matrices
 * (Sec. 3) divided by nu*dt/2 and -nu*dt/2: alpha = K2 + 2/(nu dt),
 * a = -(2 K2 + 2/(nu dt)), b = K2 (K2 + 2/(nu dt)).  (.,.)_sigma is the
 * N-point Chebyshev-Gauss (default) or Gauss-Lobatto weighted inner product
 * (Sec. 2); the two differ only in the last diagonal entry of B.
 *
 * Data layout (all solve entry points):
 *   f, u   complex128 [nsys][N], C-contiguous, wavenumber-major, 16-byte
 *          aligned DEVICE pointers owned by the caller.  Entries k >= n of f
 *          are not read; entries k >= n of u are written as 0.  u == f
 *          (in place) is allowed; partial overlap is not.
 *   alpha, a, b   float64 [nsys] DEVICE pointers.
 *
 * Execution: every call validates its arguments on the host, then enqueues
 * kernels on opts->stream and returns without synchronising.  The library
 * allocates no memory per call and keeps no state between calls except a
 * per-device table of device properties filled on first use.
 *
 * Errors: argument errors return a negative SHEN_E* code before anything is
 * enqueued (nsys must lie in [0, SHEN_MAX_NSYS]).  Numerical failures never
 * return an error code; when opts->info is non-NULL the kernels write one
 * int32 per system: 0 = ok, k+1 = an unusable pivot first met at row k (u is
 * then unspecified), SHEN_INFO_REFINE_FALLBACK = the FP32 refinement did not
 * converge and the system was re-solved in FP64.  The LU has no pivoting
 * (Sec. 4), so a pivot is unusable when it is zero, not finite, or no larger
 * than 2^-40 times |H_kk| plus the magnitudes of the subdiagonal entries of
 * row k: a singular or numerically singular leading block (an alpha at minus
 * a generalised eigenvalue of the leading rows of (S, B), say) or non-finite
 * inputs.
 */
#ifndef SHENHIP_H
#define SHENHIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHENHIP_ABI_VERSION 4

typedef struct {
  double re, im;
} shen_c128;

/* largest nsys any entry point accepts */
#define SHEN_MAX_NSYS ((int64_t)2147483646)

/* return codes */
#define SHEN_OK 0
#define SHEN_EINVAL (-1)   /* bad argument: NULL, size, alignment, enum */
#define SHEN_ELAUNCH (-2)  /* the HIP runtime refused a launch */
#define SHEN_ENOTSUP (-3)  /* N beyond what the chosen kernel supports */
#define SHEN_EDEVICE (-4)  /* no usable HIP device */
#define SHEN_ESCRATCH (-5) /* more scratch than the static buffer holds    */

/* per-system info codes besides 0 and k+1 */
#define SHEN_INFO_REFINE_FALLBACK (-2)

/* opts.precision */
#define SHEN_FP64 0        /* factor and solve in FP64 */
#define SHEN_FP32_REFINE 1 /* FP32 factor/solve, FP64 residual refinement */

/* opts.quad */
#define SHEN_QUAD_GC 0 /* Chebyshev-Gauss points (default) */
#define SHEN_QUAD_GL 1 /* Chebyshev-Gauss-Lobatto points */

/* families (batched descriptors) */
#define SHEN_HELMHOLTZ 0
#define SHEN_BIHARMONIC 1

/* bases of the wall-normal transforms (Sec. 2) */
#define SHEN_SPACE_CHEBYSHEV 0  /* T_k, k < N                                */
#define SHEN_SPACE_DIRICHLET 1  /* T_k - T_{k+2}, k < N-2                    */
#define SHEN_SPACE_BIHARMONIC 2 /* T_k - 2(k+2)/(k+3) T_{k+2} + (k+1)/(k+3) T_{k+4}, k < N-4 */

typedef struct {
  void* stream;       /* hipStream_t to enqueue on; NULL = null stream       */
  int32_t precision;  /* SHEN_FP64 (default) or SHEN_FP32_REFINE             */
  int32_t transpose;  /* 0: H u = f; 1: H^T u = f (the adjoint system)       */
  int32_t quad;       /* SHEN_QUAD_GC (default) or SHEN_QUAD_GL              */
  int32_t refine_max; /* FP32_REFINE: corrections at most (<= 64); < 0 means
                         8; 0 returns the uncorrected FP32 solution (no
                         residual, no FP64 re-solve unless the FP32 result is
                         not finite)                                          */
  double refine_tol;  /* FP32_REFINE: converged at max|du| <= tol max|u|;
                         <= 0 means 1e-14.  Refinement also stops once a
                         correction fails to halve (the rounding floor,
                         where corrections are noise of about the size of
                         the error left): the system is then accepted if
                         that correction is at most max(tol, 5e-13) max|u|,
                         else re-solved in FP64.                              */
  int32_t* info;      /* optional DEVICE int32[nsys] status per system       */
  int32_t variant;    /* kernel choice: 0 = automatic (SHEN_VARIANT_*)       */
  int32_t chunk;      /* wave kernels of the solves, adjoints and factor
                         calls: chunk length (coefficients per lane and
                         parity chain); 0 = automatic.  Nonzero values must
                         be offered for the family and N (8 or 16 for most
                         N, 4 for Helmholtz N <= 64), else SHEN_EINVAL.  A
                         tuning knob: results agree to rounding.  Ignored by
                         the other entry points.                             */
  int32_t* iters;     /* optional DEVICE int32[nsys]: FP32_REFINE solves
                         write the number of corrections applied per system
                         (0 .. refine_max); not written otherwise            */
  void* work;         /* optional DEVICE scratch for in-place FP64 solves
                         (u == f) of N the wave solves serve (N <= 8192,
                         the large-N solves included): with
                         work_bytes >= nsys * shen_factor_bytes(family, N,
                         opts) they run as a factor call into `work`
                         followed by the factored solve in place (the
                         wave kernels) instead of on the lane-per-chain
                         kernels.  Owned by the caller; must not overlap
                         f / u; its contents on entry do not matter.
                         NULL: in-place calls take the lane-per-chain
                         kernels.  Ignored by out-of-place calls.       */
  int64_t work_bytes; /* size of `work` in bytes                           */
} shen_opts;

/* kernel variants (opts.variant); 0 picks per N and mode */
#define SHEN_VARIANT_AUTO 0
#define SHEN_VARIANT_CHAIN 1 /* one lane per odd/even chain, LDS-resident     */
#define SHEN_VARIANT_WAVE 2  /* one wavefront per system, register-resident  */

/* Fill *opts with the defaults (null stream, FP64, no transpose, GC). */
void shen_opts_default(shen_opts* opts);

/* Version of this interface (SHENHIP_ABI_VERSION). */
int shen_abi_version(void);

/* Static string describing a SHEN_* return code. */
const char* shen_status_string(int code);

/* Largest N the solves accept on the current device for the given family
 * and precision: the larger of the lane-per-chain kernels' limit (set by the
 * device's LDS size) and, for SHEN_FP64, the large-N wave path's (N <= 8192,
 * chains spread over up to four wavefronts of one work group: both parity
 * chains of a system per work group up to N = 4096, one per work group past
 * it; out-of-place solves only).  In-place calls, SHEN_FP32_REFINE, the adjoints, the
 * factor-once form and the products are limited by the lane-per-chain
 * kernels past N = 1024. */
int32_t shen_max_n(int32_t family, int32_t precision);

/* The wave-kernel configuration the solves of (family, N) use with chunk
 * length `chunk` (0 = automatic): *C rows per lane and parity chain, *G lanes
 * per chain (2G lanes per system).  Returns SHEN_OK, or SHEN_EINVAL when the
 * chunk is not offered for (family, N), or SHEN_ENOTSUP when (family, N) has
 * no wave configuration (the chain kernels serve it). */
int shen_wave_config(int32_t family, int32_t N, int32_t chunk, int32_t* C, int32_t* G);

/*
 * Helmholtz solve (Sec. 4, the odd/even upper-Hessenberg LU with the
 * constant tail of U):  (S + alpha_w B) u_w = f_w  for w < nsys,
 * or the transposed system when opts->transpose.  N >= 3.
 * Transposed solves (FP64 only, else SHEN_ENOTSUP) are the adjoint solve
 * without gradients: out of place at N with a wave configuration they run
 * on the adjoint wave kernels, otherwise on the lane-per-chain kernels
 * (variant SHEN_VARIANT_WAVE in place: SHEN_ENOTSUP).  The same holds for
 * biharmonic_solve.
 */
int helmholtz_solve(int32_t N, int64_t nsys, const double* alpha, const shen_c128* f, shen_c128* u,
                    const shen_opts* opts);

/*
 * Biharmonic solve (Sec. 4, Alg. LUbiharmonic, ReduceAB and
 * LUSolveBiharmonic, in a compact form that keeps two rows of U):
 * (Q + a_w A + b_w B) u_w = f_w, or the transposed system.  N >= 5.
 */
int biharmonic_solve(int32_t N, int64_t nsys, const double* a, const double* b, const shen_c128* f,
                     shen_c128* u, const shen_opts* opts);

/*
 * Adjoint of the Helmholtz solve u = H^{-1} f for a real loss L, given
 * gbar = dL/dRe(u) + i dL/dIm(u) (complex128 [nsys][N]) and the forward
 * solution u: writes lambda = H^{-T} gbar (= the gradient with respect to f,
 * tail zero) and, when grad_alpha != NULL, grad_alpha[w] =
 * -Re(lambda_w^H B u_w) (float64 [nsys]).  lambda may alias gbar.
 */
int helmholtz_adjoint(int32_t N, int64_t nsys, const double* alpha, const shen_c128* u,
                      const shen_c128* gbar, shen_c128* lambda, double* grad_alpha,
                      const shen_opts* opts);

/*
 * Adjoint of the biharmonic solve: lambda = H^{-T} gbar, and when non-NULL
 * grad_a[w] = -Re(lambda_w^H A u_w), grad_b[w] = -Re(lambda_w^H B u_w).
 */
int biharmonic_adjoint(int32_t N, int64_t nsys, const double* a, const double* b, const shen_c128* u,
                       const shen_c128* gbar, shen_c128* lambda, double* grad_a, double* grad_b,
                       const shen_opts* opts);

/*
 * Factor-once / solve-many (the time-stepping use: Alg. NS factors every
 * wavenumber pair's matrix once and reuses the factors at every step, Sec. 3
 * and Sec. 4).  Here the factor is compact: the LU restart state at each
 * chunk start of both parity chains, computed by the sequential recurrence
 * once; every later solve recomputes the factors inside each chunk from
 * these states and reads only f, u and the states.
 *
 * fac: caller-owned DEVICE buffer, 16-byte aligned, of nsys *
 *   shen_factor_bytes(family, N, opts) bytes, layout [nsys][bytes/16]
 *   double2, opaque.  It is valid for the coefficients, N, opts->quad and
 *   opts->chunk of the factor call; the solve must pass the same.
 * The factor call writes fac and nothing else (opts->info is not touched);
 * the solve writes u and, when opts->info is non-NULL, the per-system status
 * as helmholtz_solve does.  u == f (in place) is allowed; fac must not
 * overlap u.  FP64 only, no transpose, wave kernels only: SHEN_ENOTSUP for
 * opts->precision != SHEN_FP64, opts->transpose, opts->variant ==
 * SHEN_VARIANT_CHAIN, or an N neither the one-wavefront nor the large-N
 * wave solves serve (N <= 8192; past 1024 opts->chunk must be 0).  Results
 * are bitwise those of helmholtz_solve / biharmonic_solve with the same opts.
 */
int64_t shen_factor_bytes(int32_t family, int32_t N, const shen_opts* opts); /* per system, or < 0 */
int helmholtz_factor(int32_t N, int64_t nsys, const double* alpha, void* fac, const shen_opts* opts);
int biharmonic_factor(int32_t N, int64_t nsys, const double* a, const double* b, void* fac, const shen_opts* opts);
int helmholtz_solve_factored(int32_t N, int64_t nsys, const double* alpha, const void* fac, const shen_c128* f, shen_c128* u,
                             const shen_opts* opts);
int biharmonic_solve_factored(int32_t N, int64_t nsys, const double* a, const double* b, const void* fac, const shen_c128* f,
                              shen_c128* u, const shen_opts* opts);

/*
 * Adjoints from the states of helmholtz_factor / biharmonic_factor (same
 * coefficients, N, quad and chunk): as helmholtz_adjoint / biharmonic_adjoint,
 * bitwise, without their boundary walk; a differentiable time step can thus
 * factor once for its forward solve and its backward pass.  lambda may alias
 * gbar here; fac must not overlap lambda.  Wave kernels only: SHEN_ENOTSUP
 * for opts->variant == SHEN_VARIANT_CHAIN or an N without a one-wavefront
 * configuration (N > 1024: the factor calls serve the solves only).
 */
int helmholtz_adjoint_factored(int32_t N, int64_t nsys, const double* alpha, const void* fac, const shen_c128* u,
                               const shen_c128* gbar, shen_c128* lambda, double* grad_alpha, const shen_opts* opts);
int biharmonic_adjoint_factored(int32_t N, int64_t nsys, const double* a, const double* b, const void* fac, const shen_c128* u,
                                const shen_c128* gbar, shen_c128* lambda, double* grad_a, double* grad_b,
                                const shen_opts* opts);

/*
 * Matrix-vector products Hu (or H^T u) in O(N) per system, FP64: the banded
 * part plus same-parity suffix sums for the rank-structured tail (Sec. 3
 * right-hand sides; also the residual of the refinement).  Hu must not
 * alias u.
 */
int helmholtz_matvec(int32_t N, int64_t nsys, const double* alpha, const shen_c128* u, shen_c128* Hu,
                     const shen_opts* opts);
int biharmonic_matvec(int32_t N, int64_t nsys, const double* a, const double* b, const shen_c128* u,
                      shen_c128* Hu, const shen_opts* opts);

/*
 * Mass-matrix solves u = B^{-1} f, FP64, for every system: the last step of
 * a forward Shen transform (Sec. 2, the complete transformation
 * u_hat = B^{-1} S(u), where S(u) holds the scalar products (u, phi_l)_sigma).
 * dirichlet_mass_solve uses Bbar = (phi_j, phi_k) of the Dirichlet basis
 * (three nonzero diagonals, appendix matrix table), biharmonic_mass_solve
 * Bchk of the biharmonic basis (five); per parity chain they are tri- and
 * pentadiagonal.  The matrix depends on N and opts->quad only, so there is
 * no coefficient argument.
 *
 * f, u: DEVICE arrays [nsys][N] of complex128, caller-owned, 16-byte
 *   aligned; entries k >= n of f are ignored, those of u written as 0.
 *   u may equal f (in place) but must not overlap it otherwise.
 * opts: quad and stream are used; transpose is accepted and changes nothing
 *   (B is symmetric); info is not written (B is positive definite).
 * Returns SHEN_OK once enqueued; SHEN_EINVAL for bad arguments; SHEN_ENOTSUP
 *   for precision SHEN_FP32_REFINE, variant SHEN_VARIANT_CHAIN or N > 1024.
 * Accuracy: B is ill-conditioned (condition number about 2.7e4 for Bbar and
 *   9e7 for Bchk at N = 512, growing like N^2 and N^4), and the result carries
 *   the error of a plain FP64 factorisation of B, a small multiple of
 *   cond(B) times the unit roundoff relative to max |u|.
 */
int dirichlet_mass_solve(int32_t N, int64_t nsys, const shen_c128* f, shen_c128* u, const shen_opts* opts);
int biharmonic_mass_solve(int32_t N, int64_t nsys, const shen_c128* f, shen_c128* u, const shen_opts* opts);

/*
 * Derivative projection fhat = Bbar^{-1} Cbar uhat for every system (Sec. 3,
 * the last wall-normal system of a time step): uhat holds coefficients in the
 * biharmonic basis, fhat receives the Dirichlet-basis Galerkin coefficients of
 * du/dx.  Cbar_kj = (phichk_j', phibar_k)_sigma (appendix matrix table)
 * couples Dirichlet row k to the biharmonic coefficients k-3, k-1, k+1.
 *
 * uhat, fhat: DEVICE arrays [nsys][N] of complex128, caller-owned, 16-byte
 *   aligned; entries k >= N-4 of uhat are ignored, entries k >= N-2 of fhat
 *   written as 0.  fhat may equal uhat (in place) but must not overlap it
 *   otherwise.  N >= 5.
 * opts, return codes and accuracy: as for dirichlet_mass_solve.
 */
int dirichlet_derivative_solve(int32_t N, int64_t nsys, const shen_c128* uhat, shen_c128* fhat, const shen_opts* opts);

/*
 * Wall-normal Shen transforms (Sec. 2, the forward transform uhat = B^{-1} S(u)
 * and the inverse u = S^{-1} uhat; the appendix algorithms for the forward
 * scalar products / transforms and the inverse transforms), one per
 * wavenumber pair, at the N Chebyshev-Gauss points x_j = cos(pi (2j+1)/(2N))
 * (opts.quad = SHEN_QUAD_GC, weights pi/N) or Chebyshev-Gauss-Lobatto points
 * x_j = cos(pi j/(N-1)) (SHEN_QUAD_GL, weights pi/(c_j (N-1)), c_0 = c_{N-1}
 * = 2), in the space SHEN_SPACE_*:
 *
 *   shen_scalar_product:    s_k = sum_j u(x_j) phi_k(x_j) sigma_j, k < n
 *   shen_forward_transform: uhat = B^{-1} s, B_kl = (phi_l, phi_k)_sigma
 *                           (Chebyshev: diagonal; Dirichlet, biharmonic: the
 *                           mass solves above, N <= 1024)
 *   shen_backward_transform: u(x_j) = sum_{k<n} uhat_k phi_k(x_j)
 *
 * with n = N, N-2, N-4.  Gauss points and N a power of two in 8 .. 2048 take
 * an FFT of length N per system; other N and Gauss-Lobatto points take
 * O(N^2) cosine sums.
 *
 * u: DEVICE complex128 [nsys][N] point values (index j); uhat, s: DEVICE
 *   complex128 [nsys][N] coefficients, entries k >= n written as 0 (read
 *   as ignored).  Input and output must not overlap (they may not be the same
 *   array either).  N <= 2048 (forward transform of the Dirichlet and
 *   biharmonic spaces: N <= 1024); N >= 1, 3, 5 for the three spaces.
 * Returns SHEN_EINVAL for bad sizes, pointers or space, SHEN_ENOTSUP for N
 * beyond the limits.
 */
int shen_scalar_product(int32_t N, int64_t nsys, int32_t space, const shen_c128* u, shen_c128* s, const shen_opts* opts);
int shen_forward_transform(int32_t N, int64_t nsys, int32_t space, const shen_c128* u, shen_c128* uhat,
                           const shen_opts* opts);
int shen_backward_transform(int32_t N, int64_t nsys, int32_t space, const shen_c128* uhat, shen_c128* u,
                            const shen_opts* opts);

/*
 * Right-hand sides of one Crank-Nicolson step of the channel solver (Sec. 3,
 * eq. gfin for the Dirichlet-basis g equation, eq. ufin for the
 * biharmonic-basis u equation), in the scaling of helmholtz_solve and
 * biharmonic_solve, so that solving with alpha = K2 + 2/(nu dt), resp.
 * a = -(2 K2 + 2/(nu dt)), b = K2 (K2 + 2/(nu dt)), advances one step:
 *
 *   helmholtz_rhs:  rhs = 2/(nu dt) [ (2 Bbar - Hbar) ghat + dt S(h_g) ]
 *                       = (2/nu) S(h_g) - (S + (K2 - 2/(nu dt)) B) ghat
 *   biharmonic_rhs: rhs = -2/(nu dt) [ (2 Achk - 2 K2 Bchk - Hchk) uhat + dt S(h_u) ]
 *                       = (-2/nu) S(h_u) - (Q + a' A + b' B) uhat,
 *                         a' = 2/(nu dt) - 2 K2,  b' = K2 (K2 - 2/(nu dt))
 *
 * with Hbar, Hchk the paper's Crank-Nicolson matrices (eqs.
 * Helmholtz_matrix, Biharmonic_matrix) at z^2 = K2.  One O(N) product per
 * system; nothing is allocated.
 *
 * K2: DEVICE float64 [nsys], the squared wavenumber m^2 + n^2 per system.
 * nu, dt: viscosity and time step (> 0; 2/(nu dt) finite).
 * ghat / uhat: DEVICE complex128 [nsys][N], the current coefficients
 *   (entries k >= n ignored).
 * sh: DEVICE complex128 [nsys][N], the scalar products S(h) of the
 *   explicit terms (entries k >= n ignored), or NULL to omit that term.
 * rhs: DEVICE complex128 [nsys][N], written (entries k >= n as 0).  It must
 *   not overlap ghat / uhat; it may equal sh (accumulate in place) but not
 *   overlap it otherwise.
 * opts: stream, quad (GC / GL mass matrix), variant; transpose must be 0.
 * Returns SHEN_EINVAL for bad sizes, pointers, nu or dt.
 */
int helmholtz_rhs(int32_t N, int64_t nsys, const double* K2, double nu, double dt, const shen_c128* ghat,
                  const shen_c128* sh, shen_c128* rhs, const shen_opts* opts);
int biharmonic_rhs(int32_t N, int64_t nsys, const double* K2, double nu, double dt, const shen_c128* uhat,
                   const shen_c128* sh, shen_c128* rhs, const shen_opts* opts);

/*
 * One batch of independent problems (many grids of uneven N, both
 * families, every (kx, kz) of each) in one call: the grids are grouped by
 * class (family, N, wave configuration), and each class is solved by the
 * kernels of the single-grid path over all of its grids at once (the
 * boundary walk, then the persistent LDS-streamed wave solve, which pulls
 * work items of sys_per_tile systems from a queue).  Grids with
 * 1024 < N <= 8192 take the large-N solves of helmholtz_solve /
 * biharmonic_solve, one walk and one solve per grid (chunk must be 0 there;
 * sys_per_tile is ignored).  The classes are dealt to four side streams
 * forked from opts->stream and joined back to it before the call returns
 * (the library creates them, with their events, once per device, at default
 * priority, in shen_batched_plan or else at the first call), so the whole
 * call is ordered on opts->stream; it may be captured in a hipGraph and
 * replayed (the descriptors are read at capture).
 *
 * desc: HOST array of ndesc descriptors, planned by shen_batched_plan and
 *   read by the library at every call.  c0 = alpha (Helmholtz) or a
 *   (biharmonic), c1 = b (biharmonic, else unused), all DEVICE pointers;
 *   info may be NULL.  f and u must not overlap (restart states are parked
 *   in u).
 * work: DEVICE scratch of shen_batched_work_bytes(ndesc) bytes, owned by the
 *   caller; its contents on entry do not matter (the library clears the
 *   counters it uses with its first kernel).  Concurrent calls must not
 *   share `work`.
 * Returns SHEN_EINVAL for a descriptor the plan would refuse or that was not
 * planned, SHEN_ENOTSUP for an N beyond 8192.
 */
typedef struct {
  int32_t family;  /* SHEN_HELMHOLTZ or SHEN_BIHARMONIC */
  int32_t N;
  int64_t nsys;
  const double* c0;
  const double* c1;
  const shen_c128* f;
  shen_c128* u;
  int32_t* info;
  int64_t tile_begin;   /* filled by shen_batched_plan: first work item      */
  int32_t sys_per_tile; /* systems per work item of the queue (rounded up to
                           whole wavefront groups); 0 = 32 (plan fills it)  */
  int32_t chunk;        /* wave-kernel chunk length for this grid (as
                           opts.chunk of the solves); 0 = automatic         */
} shen_problem;

/* Host-side planning: checks each HOST descriptor, fills tile_begin and a
 * default sys_per_tile, and returns the total number of work items (or a
 * negative code). */
int64_t shen_batched_plan(shen_problem* desc_host, int32_t ndesc, const shen_opts* opts);

/* Bytes of the `work` scratch for batched_solve (8 per descriptor, at least
 * 256). */
int64_t shen_batched_work_bytes(int32_t ndesc);

int batched_solve(const shen_problem* desc, int32_t ndesc, void* work, const shen_opts* opts);

/*
 * batched_solve without the `work` argument, for callers that cannot
 * allocate device memory (code under hipGraph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the work counters live in a static
 * device array of shen_batched_static_bytes() bytes (4 KiB) that the library
 * holds on each device it runs on until the process ends.  The call itself
 * allocates nothing, and creates no streams: its classes run one after
 * another on opts->stream.  Same descriptors, planning, arguments, results
 * and errors as batched_solve, plus SHEN_ESCRATCH when
 * shen_batched_work_bytes(ndesc) exceeds the static buffer.  Every call on
 * one device shares that device's buffer: calls that overlap on a device
 * (other streams, other threads, or two replays of graphs that captured
 * this call) race and must be serialised by the caller.  The buffer keeps
 * the last call's contents; each call clears what it uses with its first
 * kernel.
 */
int64_t shen_batched_static_bytes(void);
int batched_solve_static(const shen_problem* desc, int32_t ndesc, const shen_opts* opts);

#ifdef __cplusplus
}
#endif

#endif /* SHENHIP_H */
