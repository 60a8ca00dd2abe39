/*
 * tvdeblur -- lagged-diffusivity total-variation deblurring with reflective
 * and anti-reflective boundary conditions and fast-transform
 * preconditioners, on AMD Instinct MI355X (gfx950).
 *
 * Method: Z.-J. Bai, M. Donatelli, S. Serra-Capizzano, "Fast Preconditioners
 * for Total Variation Deblurring with Anti-Reflective Boundary Conditions"
 * (arXiv 1011.5964).
 *
 * Problem solved (Section 1, eqs. (nbf), (mp), (fp)): given an observed image
 * v (ny x nx), a normalised, quadrantally symmetric PSF h ((2my+1) x (2mx+1),
 * sum h = 1; Section 2 restricts fast diagonalisation to this case), the
 * boundary condition used for the blur H (reflective or anti-reflective,
 * Section 2) and alpha > 0, beta > 0, return
 *     u ~ argmin 1/2 ||H u - v||^2 + alpha sum sqrt(|grad u|^2 + beta^2)
 * computed by the lagged-diffusivity fixed point
 *     (H^T H + alpha L(u^k)) u^{k+1} = H^T v,   u^0 = v          (eq. (fp))
 * with each linear system solved by preconditioned conjugate gradients
 * warm-started at u^k and stopped at ||r|| / ||r_0|| < inner_tol (Section 5).
 * L(u^k) is the zero-Neumann TV diffusion operator with cell diffusivity
 * 1/sqrt(|grad u^k|^2 + beta^2) (forward differences, unit grid spacing).
 * Preconditioners (Section 3): none, the diagonal D = I + alpha diag(L)
 * (eq. (D)), X, D_X = D^{1/2} X D^{1/2}, and X_D for the scaled system
 * (eq. (scalesys)), where X is R (DCT-II, reflective) or M (DST-I on the
 * interior, S^ = diag(1, S_{n-2}, 1), anti-reflective); Section 3.2 gives
 * their 2D (tensor) forms.
 *
 * Conventions for every entry point
 *  - Images are dense row-major ny x nx arrays (element (i, j) at i*nx + j),
 *    resident in device memory of the handle's device and owned by the
 *    caller; the library never frees or retains them.  Element type is
 *    double for TVD_F64 handles and float for TVD_F32_MIXED handles.
 *  - Host pointers are named *_host; everything else named *_dev is device.
 *  - Work is queued on the handle's HIP stream; calls return after that
 *    stream has completed the call's work, unless stated otherwise.
 *  - Return value 0 (TVD_OK) on success or a negative TVD_E* code.  The
 *    message for the last failure is returned by tvdeblur_last_error().
 *    No C++ exception or abort crosses this interface.
 *  - A handle must not be used from two host threads at once.
 */
#ifndef TVDEBLUR_H
#define TVDEBLUR_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tvdeblur_handle* tvdeblur_t;

/* status codes */
#define TVD_OK           0
#define TVD_EINVAL      -1   /* bad argument, NaN/Inf parameter, aliasing buffers */
#define TVD_ENOTSYM     -2   /* PSF not quadrantally symmetric (to 1e-12 max|h|) */
#define TVD_ENORM       -3   /* |sum h - 1| > 1e-12 (no silent renormalisation) */
#define TVD_ESIZE       -4   /* PSF too large for the image / image too small */
#define TVD_ESTATE      -5   /* solve before set_psf / set_bc, or op before setup */
#define TVD_EDEVICE     -6   /* HIP runtime error (message in last_error) */
#define TVD_EBREAKDOWN  -7   /* PCG curvature p^T A p <= 0 (singular system) */
#define TVD_ENOMEM      -8   /* device allocation failed */

/* precision of a handle */
#define TVD_F64        0     /* all vectors and arithmetic in IEEE double */
#define TVD_F32_MIXED  1     /* float vectors, convolution, stencil and
                                transforms inside PCG; every inner product,
                                the CG scalars, the stopping test, the
                                fixed-point change, the preconditioner
                                eigenvalue setup, b = H^T v and the residual
                                b - A u^k that starts each fixed-point step
                                (iterative refinement) in double */

/* boundary condition of the blur H (Section 2) */
#define TVD_BC_REFLECTIVE      1
#define TVD_BC_ANTIREFLECTIVE  2
/* the two classical BCs the paper compares with (Sections 1-2): zero ghosts
 * (Toeplitz blur; preconditioned in the DCT-II algebra with the optimal
 * projection diag(Q2 H Q2^T) of the blur) and periodic ghosts (circulant
 * blur; the real Fourier basis diagonalises it, symbol at 2 pi k / n) */
#define TVD_BC_DIRICHLET       3
#define TVD_BC_PERIODIC        4

/* preconditioner (columns I, D, X, D_X, X_D of Tables 1-3) */
#define TVD_PREC_NONE  0
#define TVD_PREC_DIAG  1
#define TVD_PREC_X     2
#define TVD_PREC_D_X   3
#define TVD_PREC_X_D   4

#define TVD_MAX_OUTER  256

typedef struct {
    double alpha;              /* regularisation weight, > 0 (0 allowed only with TVD_PREC_NONE/X) */
    double beta;               /* smoothing of |grad u|, > 0 */
    int    max_outer;          /* fixed-point steps K, 1..TVD_MAX_OUTER */
    double fp_tol;             /* stop when ||u^{k+1}-u^k||/||u^{k+1}|| < fp_tol; 0 = run exactly K */
    double inner_tol;          /* PCG stop ||r|| < inner_tol ||r_0|| (strict); >= 0 */
    int    max_inner;          /* PCG iteration cap per step, >= 1 */
    int    precond;            /* TVD_PREC_* (default choice: TVD_PREC_X_D) */
    const void* u0_dev;        /* initial iterate, or NULL for u^0 = v (Section 5) */
    const int*  replay_host;   /* NULL, or max_outer PCG iteration counts to run exactly
                                  (stopping test skipped); used to compare with a
                                  reference that took the same number of steps */
    void*  iterates_dev;       /* NULL, or room for (max_outer+1) images: u^0..u^K are
                                  stored there (checkpoints for the adjoint) */
    int    record_objective;   /* nonzero: tvdeblur_solve / _noalloc fill
                                  tvd_stats.tv_objective (one extra blur and
                                  reduction per step, FP64) */
    int    use_graph;          /* nonzero: tvdeblur_solve replays the PCG iterations of
                                  transform-preconditioned solves from HIP graphs of two
                                  iterations each (captured on first use, cached by the
                                  handle); 0: the launches go one by one, which measured
                                  faster on MI355X (512^2: 30.6 against 32.9 ms per
                                  restore).  Same bits either way.  Ignored by
                                  tvdeblur_solve_noalloc (instantiating a graph
                                  allocates). */
} tvd_params;

typedef struct {
    int    outer_steps;                    /* fixed-point steps taken */
    int    inner_iters[TVD_MAX_OUTER];     /* PCG iterations of each step */
    double relres[TVD_MAX_OUTER];          /* final ||r||/||r_0|| of each step */
    double fp_change[TVD_MAX_OUTER];       /* ||u^{k+1}-u^k|| / ||u^{k+1}|| */
    int    all_converged;                  /* every step met inner_tol */
    int    breakdown;                      /* a step stopped on p^T A p <= 0 */
    long long total_inner_iters;
    double time_total_s;                   /* wall time of the call */
    double time_setup_s;                   /* per-step setup (diffusivity, eigenvalues) */
    double time_inner_s;                   /* PCG loops */
    double tv_objective[TVD_MAX_OUTER + 1]; /* with record_objective: T(u^0)..T(u^K) of
                                              eq. (mp), 1/2 ||H u - v||^2 + alpha sum
                                              sqrt(|grad u|^2 + beta^2) in FP64 (the
                                              lagged-diffusivity steps decrease it);
                                              else 0 */
} tvd_stats;

/* Create a handle for ny x nx images on the current HIP device, queuing
 * work on hip_stream (a hipStream_t; NULL = the null stream).  ny, nx >= 3.
 * Errors: TVD_EINVAL, TVD_ESIZE, TVD_EDEVICE. */
int tvdeblur_create(tvdeblur_t* out, int ny, int nx, int precision, void* hip_stream);

/* Copy the PSF (host, row-major py x px, both odd; centre at (py/2, px/2)).
 * Checks: odd sizes; quadrantal symmetry h(a,b) = h(-a,b) = h(a,-b) to
 * 1e-12 max|h| (Section 2, 2D case); |sum h - 1| <= 1e-12 (the normalised
 * PSF of eq. (blur1d)); finite entries.  The PSF half-widths must satisfy
 * m <= n-1 for anti-reflective and m <= n for reflective BCs (checked at
 * set_bc and solve).  Errors: TVD_EINVAL, TVD_ENOTSYM, TVD_ENORM. */
int tvdeblur_set_psf(tvdeblur_t h, const double* psf_host, int py, int px);

/* Boundary condition of H: TVD_BC_REFLECTIVE or TVD_BC_ANTIREFLECTIVE
 * (Section 2), or one of the two classical BCs the paper compares with:
 * TVD_BC_DIRICHLET (zero ghosts; the DCT-II preconditioners) and
 * TVD_BC_PERIODIC (wrap-around ghosts; the real Fourier basis, whose
 * transforms always run as matrix-core products; needs 4m + 1 <= n per axis).
 * L(u) is always zero-Neumann.  The reblurring system takes anti-reflective
 * BCs only; the batching form all but periodic.  Errors: TVD_EINVAL,
 * TVD_ESIZE. */
int tvdeblur_set_bc(tvdeblur_t h, int bc);

/* Run the fixed-point / PCG method (eq. (fp)) on v_dev, writing u_dev.
 * v_dev and u_dev must not alias.  stats (host, may be NULL) is filled in.
 * Non-convergence of an inner solve within max_inner is not an error (the
 * paper caps iterations too): it shows in stats.all_converged.
 * Errors: TVD_EINVAL, TVD_ESTATE, TVD_ESIZE, TVD_EDEVICE, TVD_ENOMEM,
 * TVD_EBREAKDOWN (u_dev then holds the last iterate). */
int tvdeblur_solve(tvdeblur_t h, const void* v_dev, void* u_dev,
                   const tvd_params* p, tvd_stats* stats);

/* ---- allocation-free solve ----
 * For callers that cannot allocate device memory when they call: serving
 * loops and harnesses that forbid hipMalloc after start-up.  Arguments,
 * arithmetic, results, stats and errors are those of tvdeblur_solve, with
 * these differences:
 *  - the per-solve work buffers (the PCG vectors, per-block partial sums and
 *    the control block) live in one static device array of
 *    TVD_NOALLOC_SCRATCH_BYTES that the library holds on every device it
 *    runs on until the process ends; the call allocates nothing (no
 *    hipMalloc, hipFree or allocating library routine);
 *  - the handle must already be built for its PSF and BC (tvdeblur_solve
 *    or tvdeblur_get_transform once after set_psf / set_bc; building
 *    allocates the handle's tables), else TVD_ESTATE;
 *  - images whose work buffers exceed TVD_NOALLOC_SCRATCH_BYTES fail with
 *    TVD_ESIZE (about 16 float + 2 double images plus partials: up to
 *    ~910 x 910 for TVD_F32_MIXED, ~680 x 680 for TVD_F64);
 *  - kernel profiling (tvdeblur_set_profiling) must be off, else TVD_EINVAL.
 * Every call on one device shares that device's array, and its contents are
 * whatever the last call left (each solve initialises what it reads): calls
 * that overlap in time on one device race and give wrong results, whether
 * from two host threads or two streams.  Calls on different devices do not
 * interact.  tvdeblur_time_kernel after this call times the handle's own
 * buffers. */
#define TVD_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int tvdeblur_solve_noalloc(tvdeblur_t h, const void* v_dev, void* u_dev,
                           const tvd_params* p, tvd_stats* stats);

/* Caller-owned work area for tvdeblur_solve (Section 5's PCG vectors, in
 * memory the caller's allocator owns, e.g. a torch tensor).
 * tvdeblur_workspace_bytes builds the handle for its PSF and BC if needed
 * (else TVD_ESTATE) and writes the bytes the area must hold: the per-solve
 * work buffers (about 16 images in the working precision plus 2 FP64
 * images, per-block partial sums and the control block).  The handle's
 * tables and per-step eigenvalue arrays stay in its own memory.
 * tvdeblur_set_workspace(h, ws_dev, bytes) makes every later tvdeblur_solve
 * on h carve those buffers from ws_dev (device memory, 256-byte aligned,
 * at least the size above, else TVD_EINVAL / TVD_ESIZE); ws_dev = NULL
 * returns to the handle's own buffers.  The library never frees ws_dev:
 * it must stay valid, and untouched by other work, while solves on h run.
 * A later set_psf / set_bc that enlarges the need makes tvdeblur_solve fail
 * with TVD_ESIZE until a large enough area is set.  Results are identical
 * to those of the handle's own buffers. */
int tvdeblur_workspace_bytes(tvdeblur_t h, size_t* bytes_out);
int tvdeblur_set_workspace(tvdeblur_t h, void* ws_dev, size_t bytes);

/* Differentiation form: reverse-mode derivative of the K fixed-point steps of
 * eq. (fp), u^{k+1} = (H^T H + alpha L(u^k))^{-1} H^T v with u^0 = v.
 * iterates_dev holds u^0..u^K as written by tvdeblur_solve (iterates_dev of
 * its params; K = its stats.outer_steps), ubar_dev = dl/du^K.  Writes
 * vbar_dev = dl/dv (device, the image type of the handle) and *abar_host =
 * dl/dalpha, *bbar_host = dl/dbeta.  Step k recomputes kappa(u^k) and the
 * preconditioner from the checkpoint and solves the adjoint system
 * A_k lambda = ubar^{k+1} with the same PCG and preconditioner (A_k is
 * symmetric), from lambda = 0, with p->inner_tol / max_inner / precond;
 * alpha and beta must equal the forward call's.  The result is the
 * derivative of the exact fixed-point map, so gradient checks use a tight
 * inner_tol in both calls.  stats (nullable) reports the adjoint PCG
 * iterations per step (index K-1-k for step k).  The derivative assumes
 * u^0 = v (it adds dl/du^0 to dl/dv): if the handle's last tvdeblur_solve
 * started from tvd_params.u0_dev, the call fails with TVD_EINVAL.
 * Errors: as tvdeblur_solve. */
int tvdeblur_solve_adjoint(tvdeblur_t h, const void* iterates_dev, int K, const void* ubar_dev,
                           void* vbar_dev, double* abar_host, double* bbar_host,
                           const tvd_params* p, tvd_stats* stats);

/* Release the handle and its device workspace. NULL is accepted. */
int tvdeblur_destroy(tvdeblur_t h);

/* Message of the last failure on h (or of the last failed create when h is
 * NULL).  Valid until the next call on h. */
const char* tvdeblur_last_error(tvdeblur_t h);

/* ---- the reblurring system (Section 3, eq. (fpp)) ----
 *
 * Fixed-point steps (H'H + alpha L(u^k)) u^{k+1} = H'v with u^0 = v, where
 * H' is the anti-reflective blur of the PSF rotated by 180 degrees (= H, the
 * PSF being quadrantally symmetric) and L(u^k) the zero-Neumann TV operator.
 * The system is not symmetric; each step runs preconditioned BiCGstab (van
 * der Vorst 1992) warm-started at u^k, with the reblurring preconditioners of
 * Section 3 / Section 3.2 in the algebra of T_n (x) T_n (Section 2), or the
 * plain ones of the paper's tables:
 *   precond TVD_PREC_NONE -> I (no preconditioner)
 *           TVD_PREC_DIAG -> D = I + alpha diag(L(u^k)) (eq. (D))
 *           TVD_PREC_X   -> P   = H'H + alpha AR_2(L(u^k))
 *           TVD_PREC_D_X -> D_P = D^{1/2} P D^{1/2}
 *           TVD_PREC_X_D -> P_D for the scaled system eq. (scalereb), applied
 *                           to eq. (fpp) as D^{1/2} P_D D^{1/2}
 * AR_2(.) takes the level-2 tau projection of the operator's inner block for
 * the interior eigenvalues and the corner rule of AR(.) for the two y = 0
 * frequencies of each axis.
 * Arguments, layout and ownership as tvdeblur_solve (v_dev, u_dev: ny x nx
 * row-major device images of the handle's precision; p, stats: host).  One
 * iteration (stats.inner_iters) = two preconditioner solves and two operator
 * products; the test ||r_i|| < inner_tol ||r_0|| runs once per iteration, on
 * the updated residual.  p->replay_host runs exactly the given counts.
 * Requirements: anti-reflective BC (set_bc); any PSF set_psf accepts.  A
 * separable PSF (h = g_y g_x^T) of half-widths <= 16 runs the operator
 * H H z + alpha L z in one tile pass; other PSFs (rank r > 1, or wider)
 * run it as two rank-r band passes, H z and then H (H z) with the stencil.
 * The P / D_P / P_D solves run in the handle's transform form: products
 * with T^{-1} and T (TVD_TRANSFORM_GEMM) or line transforms (FFT: S^ with
 * the two end values' linear interpolant removed before it and restored
 * after it).
 * Errors: TVD_EINVAL (also for an unsupported BC / PSF / preconditioner),
 * TVD_ESTATE, TVD_ESIZE, TVD_EDEVICE, TVD_ENOMEM, TVD_EBREAKDOWN (rho,
 * <rhat, v> or omega became 0; u_dev then holds the last iterate). */
int tvdeblur_solve_reblur(tvdeblur_t h, const void* v_dev, void* u_dev,
                          const tvd_params* p, tvd_stats* stats);

/* Boundary condition of L(u^k) in the reblurring system (Section 3 defines
 * the preconditioners with zero-Neumann L; its experiments also impose
 * anti-reflective BCs on L): TVD_L_NEUMANN (default) or
 * TVD_BC_ANTIREFLECTIVE.  The anti-reflective L takes the diffusivity on
 * every face of the image, the ghost faces included, from the
 * anti-reflectively extended u^k, and applies the flux divergence with the
 * argument extended the same way (one ghost line per side): it differs from
 * the Neumann L only in the edge rows and columns and is not symmetric.  The
 * preconditioners keep the Neumann eigenvalues and D (the inner block of L is
 * the same).  Applies to later tvdeblur_solve_reblur and op_reblur_* calls.
 * Errors: TVD_EINVAL. */
#define TVD_L_NEUMANN 0
int tvdeblur_set_reblur_l_bc(tvdeblur_t h, int l_bc);

/* Setup of the reblurring preconditioner (any of the five above) from uk_dev;
 * tvdeblur_op_export then returns its kappa, s, mu, lambda_H and D. */
int tvdeblur_op_reblur_setup(tvdeblur_t h, const void* uk_dev, double alpha, double beta, int precond);

/* y = (H'H + alpha L(u^k)) x with the state of the last op_reblur_setup
 * (x, y device images; must not alias).  Errors: TVD_ESTATE before it. */
int tvdeblur_op_reblur_normal(tvdeblur_t h, const void* x_dev, void* y_dev);

/* z = M^{-1} r for the reblurring preconditioner of the last op_reblur_setup
 * (r, z must not alias).  Errors: TVD_ESTATE before it. */
int tvdeblur_op_reblur_precond(tvdeblur_t h, const void* r_dev, void* z_dev);

/* ---- single operators, for verification of each step on its own ---- */

/* y = H x, the blur under the handle's BC (Section 2). */
int tvdeblur_op_blur(tvdeblur_t h, const void* x_dev, void* y_dev);

/* y = H^T x. */
int tvdeblur_op_blur_adjoint(tvdeblur_t h, const void* x_dev, void* y_dev);

/* Per-fixed-point-step setup from the iterate uk_dev: diffusivity
 * kappa(u^k), D = I + alpha diag(L(u^k)) (eq. (D)) and the preconditioner
 * eigenvalues of the chosen variant (Section 3.2).  Kept in the handle for
 * the two calls below. */
int tvdeblur_op_setup(tvdeblur_t h, const void* uk_dev, double alpha, double beta, int precond);

/* y = (H^T H + alpha L(u^k)) x with the state of the last op_setup (eq. (fp)). */
int tvdeblur_op_normal(tvdeblur_t h, const void* x_dev, void* y_dev);

/* z = P^{-1} r for the preconditioner of the last op_setup. */
int tvdeblur_op_precond(tvdeblur_t h, const void* r_dev, void* z_dev);

/* Copy an internal array of the last op_setup into dst_dev as ny x nx
 * doubles: 0 = kappa, 1 = scaling s (D^{-1/2}, or 1), 2 = eigenvalues mu,
 * 3 = lambda_H (PSF symbol on the BC grid), 4 = D. */
int tvdeblur_op_export(tvdeblur_t h, int which, void* dst_dev);

/* ---- transform implementation of the preconditioner ----
 *
 * The 2D transforms of the X, D_X and X_D preconditioners (Section 3.2) run
 * either as line transforms on the handle's own FFT in LDS (DST-I through a
 * real DFT of length 2(n-1), DCT-II through one of length 2n; Bluestein
 * for lengths that are not powers of two) or as dense products with the n x n
 * basis matrix on the matrix cores (4 products of n^3 multiply-adds per
 * application; in TVD_F32_MIXED the 64 x 64 tiles compute each FP32 product
 * as six bf16 products of three-way operand splits, to FP32 accuracy).  The
 * two differ only in rounding.  TVD_TRANSFORM_AUTO (the default) times one
 * application of each when the handle is built (at the first solve or op
 * after set_psf / set_bc) and keeps the line transforms unless the products
 * are at least 5% faster. */
#define TVD_TRANSFORM_AUTO  0
#define TVD_TRANSFORM_FFT   1
#define TVD_TRANSFORM_GEMM  2

/* Select the transform implementation (takes effect now if the handle is
 * built, else when it is).  GEMM on a handle without the product form falls
 * back to FFT; tvdeblur_get_transform tells which one runs.
 * Errors: TVD_EINVAL. */
int tvdeblur_set_transform(tvdeblur_t h, int mode);

/* The implementation in use (TVD_TRANSFORM_FFT or TVD_TRANSFORM_GEMM) into
 * *active (host); builds the handle first if needed.
 * Errors: TVD_EINVAL, TVD_ESTATE, TVD_EDEVICE. */
int tvdeblur_get_transform(tvdeblur_t h, int* active);

/* Block tile of the matrix-core products (32: four waves (eight in FP64)
 * split the K of one 32 x 32 tile; 64: a 64 x 64 tile, one 32 x 32 quadrant
 * per wave, two groups of four waves splitting K for a single image) into
 * *tile (host).  Picked with the transform form by timing at build (both
 * tiles, interleaved, three times each; cached per process by shape, PSF
 * widths, BC and precision).  Builds the handle first if needed.
 * Errors: TVD_EINVAL, TVD_ESTATE, TVD_EDEVICE. */
int tvdeblur_get_gemm_tile(tvdeblur_t h, int* tile);

/* Request a block tile for the products: 0 (default) times both at build,
 * 32 or 64 uses that one (takes effect now if the handle is built, else when
 * it is).  The two differ only in rounding (the order of the K sums).
 * Errors: TVD_EINVAL (other values). */
int tvdeblur_set_gemm_tile(tvdeblur_t h, int tile);

/* ---- kernel timing (HIP events on the handle's stream) ---- */

#define TVD_KTIME_KINDS 12
typedef struct {
    int    n_kinds;                         /* entries filled */
    char   name[TVD_KTIME_KINDS][24];       /* kernel class */
    long long launches[TVD_KTIME_KINDS];    /* launches timed (the sampled ones) */
    double total_ms[TVD_KTIME_KINDS];       /* summed event-to-event time */
} tvd_kernel_times;

/* every >= 1: from now on every every-th launch of each kernel class of
 * tvdeblur_solve is timed and its duration accumulated per class (band
 * operator, forward row transform, column transform, inverse row transform,
 * residual, setup, other, PCG update, transform product on the matrix
 * cores, row half of the normal operator); the counters are reset.  A single-kernel class is
 * timed by a start/stop event pair carried on that kernel's own dispatch
 * (its execution time); the residual and setup classes, which span several
 * kernels, by marker events around them.  A timed launch delays the next
 * one by several microseconds, hence the sampling.  every == 0 stops. */
int tvdeblur_set_profiling(tvdeblur_t h, int every);

/* Copy the accumulated per-class counts and times into *out (host). */
int tvdeblur_get_kernel_times(tvdeblur_t h, tvd_kernel_times* out);

/* Average execution time of one PCG-loop kernel class, measured by a pair of
 * marker events around `reps` back-to-back repetitions on the handle's stream
 * (no events on the dispatches themselves), with the handle's current
 * buffers and parameters; *avg_us (host) receives the time per kernel launch.
 * kind is a class index of tvd_kernel_times: 0 band operator (the y-pass of
 * the active transform form; for a PSF that is not split into row and column
 * passes, the band launch(es) of one operator application, averaged per
 * launch), 2 column transform, 7 PCG update (product form), 8 transform
 * products (the four products of one preconditioner application, averaged
 * per product), 9 row half of the normal operator.  Needs a completed tvdeblur_solve on the
 * handle (its parameters and preconditioner); overwrites the handle's work
 * buffers, so call it between solves.  TVD_EINVAL for another kind, a kind
 * the active form does not run, reps < 1, or no solve yet. */
int tvdeblur_time_kernel(tvdeblur_t h, int kind, int reps, double* avg_us);

/* ---- batching form: many independent images, one launch per PCG stage ----
 *
 * Each image is its own instance of the problem of eq. (fp) -- its own size,
 * PSF, alpha and beta -- under one boundary condition and precision for the
 * whole batch.  Every stage of the method (diffusivity and eigenvalue setup,
 * residual, the transform passes of the preconditioner of Section 3.2, the
 * operator application) is one kernel launch covering all images; each image
 * keeps its own CG scalars and its own stopping test (Section 5), and an
 * image whose PCG has stopped skips its share of later launches.  The
 * arithmetic of each image is that of tvdeblur_solve with the same
 * parameters, so each image's result matches a single-image solve up to
 * floating-point rounding order.
 *
 * Restrictions: separable PSFs (h = g_y g_x^T, e.g. Gaussians) of half-width
 * <= 16, and a transform preconditioner (TVD_PREC_X, TVD_PREC_D_X or
 * TVD_PREC_X_D).  Other cases use tvdeblur_solve. */

typedef struct tvdeblur_batch* tvdeblur_batch_t;

typedef struct {
    int ny, nx;                 /* image size, >= 3 each, <= 2048 */
    const double* psf_host;     /* row-major py x px PSF, checked as in tvdeblur_set_psf */
    int py, px;
} tvd_image_desc;

typedef struct {
    const double* alpha_host;   /* count per-image alpha (> 0) */
    const double* beta_host;    /* count per-image beta (> 0), or NULL: beta for all */
    double beta;
    int    max_outer;           /* fixed-point steps, 1..TVD_MAX_OUTER */
    double fp_tol;              /* per image: stop its steps when the relative change
                                   falls below fp_tol; 0 = every image runs max_outer */
    double inner_tol;           /* PCG stop ||r|| < inner_tol ||r_0||, per image */
    int    max_inner;           /* PCG iteration cap per step, >= 1 */
    int    precond;             /* TVD_PREC_X, TVD_PREC_D_X or TVD_PREC_X_D */
    int    use_graph;           /* != 0: replay the PCG iteration launches from HIP
                                   graphs captured on the batch's stream */
    const int* replay_host;     /* NULL, or count x max_outer PCG iteration counts
                                   (image-major: [i * max_outer + k]) to run exactly,
                                   stopping test skipped, as tvd_params.replay_host */
    int    transform;           /* TVD_TRANSFORM_AUTO (the implementation picked at
                                   create), TVD_TRANSFORM_FFT or TVD_TRANSFORM_GEMM */
    int    gemm_tile;           /* block tile of the products: 0 (the one picked at
                                   create), 32 or 64 */
} tvd_batch_params;

#define TVD_TUNE_MAX 4
typedef struct {
    int    count;                       /* images in the batch */
    int    line_threads;                /* threads per block of the transform passes */
    int    tables_in_lds;               /* FFT tables staged in LDS */
    int    from_cache;                  /* choice reused from an earlier batch of the same shapes */
    int    n_candidates;                /* candidates timed (0 when from_cache) */
    int    cand_threads[TVD_TUNE_MAX];
    double cand_us[TVD_TUNE_MAX];       /* time of one set of transform passes */
    double gemm_us;                     /* the same with the products on the matrix cores
                                           (32 x 32 block tiles) */
    int    transform;                   /* implementation of the last solve (TVD_TRANSFORM_*) */
    long long graph_launches;           /* graph replays since create */
    double time_setup_s;                /* last solve: diffusivity/eigenvalue setup */
    double time_inner_s;                /* last solve: PCG loops */
    double gemm64_us;                   /* the products with 64 x 64 block tiles */
    int    gemm_tile;                   /* block tile the products use (32 or 64) */
} tvd_batch_info;

/* Create a batch of `count` (1..4096) image problems on the current HIP
 * device.  The PSFs are copied.  Work runs on a stream owned by the batch;
 * it waits for the work queued so far on hip_stream (a hipStream_t, NULL =
 * null stream) at each solve, and each solve returns with its results
 * complete.  At create the thread count of the transform passes is picked by
 * timing the candidates on this batch's shapes (cached per process by the
 * shapes, PSF widths, BC and precision).
 * Errors: TVD_EINVAL, TVD_ENOTSYM, TVD_ENORM, TVD_ESIZE, TVD_EDEVICE,
 * TVD_ENOMEM (message from tvdeblur_batch_last_error(NULL)). */
int tvdeblur_batch_create(tvdeblur_batch_t* out, int count, const tvd_image_desc* descs, int precision,
                          int bc, void* hip_stream);

/* Solve every image: v_dev_host[i] / u_dev_host[i] (host arrays of `count`
 * device pointers; image i is a dense row-major ny_i x nx_i array of the
 * batch's element type; no u may alias any v).  u^0 = v.  stats_host (may be
 * NULL) receives `count` tvd_stats, one per image; their time fields are
 * the batch's.  A breakdown stops that image only; the call then returns
 * TVD_EBREAKDOWN after the others have finished.
 * Errors: TVD_EINVAL, TVD_EDEVICE, TVD_EBREAKDOWN. */
int tvdeblur_batch_solve(tvdeblur_batch_t b, const void* const* v_dev_host, void* const* u_dev_host,
                         const tvd_batch_params* p, tvd_stats* stats_host);

/* Tuning choice and timings of the batch (host *out). */
int tvdeblur_batch_get_info(tvdeblur_batch_t b, tvd_batch_info* out);

/* Release the batch. NULL is accepted. */
int tvdeblur_batch_destroy(tvdeblur_batch_t b);

/* Message of the last failure on b, or of the last failed batch create when b is NULL. */
const char* tvdeblur_batch_last_error(tvdeblur_batch_t b);

/* ---- 1D signals (Section 5.1): many independent signals, one launch ----
 *
 * Each signal is its own instance of eq. (fp) in one dimension,
 * (H^T H + alpha L(u^k)) u^{k+1} = H^T v with u^0 = v, where H is the 1D blur
 * of a symmetric normalised PSF (e.g. the out-of-focus PSF of eq. (of))
 * under the signal's boundary condition and L(u^k) the zero-Neumann TV
 * operator with cell diffusivity 1/sqrt((u_{i+1} - u_i)^2 + beta^2).  Each
 * step runs PCG warm-started at u^k with the signal's preconditioner (I, D of
 * eq. (D), X = R or M of Section 3, D_X, X_D) and the stopping test of
 * Section 5 (or, for the reblurring system of eq. (fpp), PBiCGstab with P,
 * D_P, P_D as tvdeblur_solve_reblur); the fixed-point loop stops after
 * max_outer steps or at the first relative change below fp_tol.  One workgroup runs one signal from start to
 * finish, so a solve of the whole batch is a single kernel launch.  All
 * arithmetic is IEEE double (the paper's precision; there is no FP32 form).
 * Signals are packed back to back in one device buffer: signal i starts at
 * the sum of the n of the signals before it. */

typedef struct tvdeblur_signals* tvdeblur_signals_t;

typedef struct {
    int n;                    /* samples, 3..4096 */
    const double* psf_host;   /* plen taps (odd), centre at plen/2, symmetric,
                                 sum 1 (checked as in tvdeblur_set_psf); copied */
    int plen;                 /* half-width plen/2 <= n-1 (AR) or <= n (reflective) */
    int bc;                   /* TVD_BC_* (periodic: 4 plen/2 + 1 <= n) */
    int reblur;               /* nonzero: also build the tables of the reblurring
                                 system (anti-reflective only; two more n x n arrays) */
} tvd_signal_desc;

typedef struct {
    const double* alpha_host;  /* count alphas (>= 0, finite) */
    const double* beta_host;   /* count betas (> 0), or NULL: beta for all */
    double beta;
    const int* precond_host;   /* count TVD_PREC_* codes, or NULL: precond for all */
    int    precond;
    int    max_outer;          /* 1..TVD_MAX_OUTER */
    double fp_tol;             /* 0 = run exactly max_outer steps */
    double inner_tol;          /* ||r|| < inner_tol ||r_0|| (strict) */
    int    max_inner;          /* >= 1 */
    const int* replay_host;    /* NULL, or count x max_outer iteration counts
                                  (signal-major) to run exactly, stopping test skipped */
    const int* system_host;    /* count of 0 / 1, or NULL: system for all */
    int    system;             /* 0: eq. (fp) by PCG with I, D, X, D_X, X_D;
                                  1: the reblurring system eq. (fpp),
                                  (H'H + alpha L(u^k)) u^{k+1} = H'v, by PBiCGstab with
                                  I, D, P, D_P, P_D (precond codes NONE, DIAG, X, D_X,
                                  X_D) as tvdeblur_solve_reblur; one iteration = two
                                  operator products */
} tvd_signal_params;

/* Build the tables of `count` (1..65536) signals on the current device: the
 * bands of H^T H and H^T with the BC folded in, the transform basis, the
 * symbol eigenvalues on the BC grid.  Work is queued on hip_stream (a
 * hipStream_t, NULL = null stream).  Errors: TVD_EINVAL, TVD_ENOTSYM,
 * TVD_ENORM, TVD_ESIZE, TVD_ENOMEM, TVD_EDEVICE (message from
 * tvdeblur_signals_last_error(NULL)). */
int tvdeblur_signals_create(tvdeblur_signals_t* out, int count, const tvd_signal_desc* descs, void* hip_stream);

/* Solve every signal: v_dev, u_dev are device buffers of sum(n) doubles
 * (packed as above, caller-owned, must not alias).  stats_host (may be NULL)
 * receives count tvd_stats; their time fields are the launch's.  Returns
 * after the results are complete.  A breakdown stops that signal only and
 * the call returns TVD_EBREAKDOWN after the others have finished.
 * Errors: TVD_EINVAL, TVD_EDEVICE, TVD_EBREAKDOWN. */
int tvdeblur_signals_solve(tvdeblur_signals_t s, const double* v_dev, double* u_dev,
                           const tvd_signal_params* p, tvd_stats* stats_host);

/* Release the signals' tables and work area.  NULL is accepted. */
int tvdeblur_signals_destroy(tvdeblur_signals_t s);

/* Message of the last failure on s, or of the last failed create when s is NULL. */
const char* tvdeblur_signals_last_error(tvdeblur_signals_t s);

#ifdef __cplusplus
}
#endif

#endif /* TVDEBLUR_H */
