/*
 * ras_pml.h -- C ABI of the MI355X RAS-PML GMRES hot path.
 *
 * What it computes (Xie, Gong, Graham, Spence, Zhang, "Massively parallel
 * Schwarz methods for the high frequency Helmholtz equation"):
 *
 *   * the P1 finite-element discretisation of  Delta u + k^2 u = -f  on the
 *     unit square surrounded by a Cartesian PML (Section 1, eq. (pml),
 *     (weak)), written in its complex-symmetric form;
 *   * the restricted additive Schwarz preconditioner with PML transmission
 *     conditions  B^{-1} = sum_j R~_j^T A_j^{-1} R_j  (Section 2, discrete
 *     RAS, eq. (local-ras-discrete) and (update1)), with impedance
 *     (Section 3 (ii), eq. (impedance)) or Dirichlet local conditions;
 *   * GMRES accelerated by that preconditioner (Section 4.1).
 *
 * Conventions shared by every entry point:
 *
 *   * Vectors are DEVICE pointers to interleaved complex128 values
 *     (re, im, re, im, ...), one value per unknown.  Unknowns are the
 *     interior mesh nodes (i, j), 1 <= i, j <= Nc-1, numbered
 *     (j-1)(Nc-1) + (i-1) (x fastest), Nc = grid + 2 * global_pml.
 *     A handle built by ras_pml_setup_batch concatenates the unknowns of
 *     its problems in problem order.
 *   * The caller owns every vector; the handle owns everything else
 *     (operators, factors, workspaces).  Nothing is freed behind the
 *     caller's back except by ras_pml_destroy.
 *   * `stream` is a hipStream_t (NULL = the default stream).  Every entry
 *     point enqueues its work on that stream and, unless stated otherwise,
 *     returns without waiting for it.
 *   * Every function returns RAS_OK (0) or a status below; no C++
 *     exception crosses the ABI.  Parameter checks run on the host before
 *     any device work.  ras_pml_last_error gives the message of the last
 *     failure on a handle.
 *   * A handle is not thread-safe; use one handle per stream.
 */
#ifndef RAS_PML_H
#define RAS_PML_H

#ifdef __cplusplus
extern "C" {
#endif

enum ras_status {
    RAS_OK = 0,
    RAS_EINVAL = 1,      /* invalid argument (message says which)              */
    RAS_ENOMEM = 2,      /* device allocation failed                           */
    RAS_EHIP = 3,        /* a HIP runtime call failed                          */
    RAS_EZEROPIVOT = 4,  /* a local factorisation met a (near) zero pivot      */
    RAS_ENONFINITE = 5,  /* a right-hand side or an iterate is not finite      */
    RAS_ENOTCONV = 6,    /* GMRES stopped at maxit; x holds the last iterate   */
    RAS_EBREAKDOWN = 7,  /* Arnoldi broke down without reaching the tolerance  */
    RAS_ENOTSUP = 8      /* a size beyond what the kernels are built for       */
};

enum { RAS_BC_IMP = 0, RAS_BC_DRCH = 1 };          /* local boundary condition */
enum { RAS_POU_LINEAR = 0, RAS_POU_BOOLEAN = 1 };  /* partition of unity       */
enum { RAS_MIXED = 0, RAS_FP64 = 1 };              /* local factor precision   */
enum { RAS_FLAG_TIMING = 1,                        /* record HIP events        */
       RAS_FLAG_UNFUSED_ARNOLDI = 2,               /* one launch per MGS step  */
       RAS_FLAG_GRAPH_STEPS = 4 };                 /* GMRES steps replayed
                                                      from a HIP graph (see
                                                      gmres_solve)             */

typedef struct ras_pml_handle *ras_pml_t;

typedef struct {
    double sigma;      /* PML profile g(x) = sigma x^3 (Section 4 uses 10 k);
                          <= 0 selects 10 k                                  */
    int global_pml;    /* global PML thickness in cells; < 0 selects pml_width */
    int bc;            /* RAS_BC_IMP (Section 3 (ii)) or RAS_BC_DRCH          */
    int pou;           /* RAS_POU_LINEAR (Section 4) or RAS_POU_BOOLEAN       */
    int precision;     /* RAS_MIXED: complex64 local factors and solves, all
                          global vectors, SpMV and Krylov work complex128;
                          RAS_FP64: complex128 everywhere                     */
    int flags;         /* bitwise OR of RAS_FLAG_*                            */
    const char *tune_cache; /* path of a tuning cache written by
                          ras_pml_autotune, or NULL: setup then uses the
                          cached kernel variants for the configurations the
                          file knows (a missing file is an empty cache)       */
    double width_c_delta; /* Section 3 (iii) width rule (eq. igg_width) used  */
    double width_c_kappa; /* for an overlap / pml_width of RAS_WIDTH_RULE:     */
    double width_k0;      /* C_delta, C_kappa and k0; defaults 1/6, 1/2, 150
                             (the constants of Tables 3 and 4)               */
} ras_pml_opts;

/* Pass as overlap and/or pml_width to take the width from the Section 3
 * (iii) rule with the constants in ras_pml_opts (see ras_pml_width_rule). */
#define RAS_WIDTH_RULE (-1)

/* Number of int32 fields in one subdomain descriptor (ras_pml_plan). */
#define RAS_DESC_INTS 24

/* Fill *o with the defaults (sigma = 10 k, global PML = pml_width,
 * impedance, linear PoU, mixed precision, no flags, no tuning cache, width
 * rule constants C_delta = 1/6, C_kappa = 1/2, k0 = 150). */
void ras_pml_default_opts(ras_pml_opts *o);

/* Host-only planning: validates the parameters exactly as ras_pml_setup
 * does and writes the subdomain table without touching any GPU.
 *   k          wavenumber (> 0)
 *   h          mesh width; grid[0] * h == 1 and grid[1] == grid[0] required
 *   grid       cells of the interior box (0,1)^2 per side
 *   subdomains number of subdomains per side (Section 2 Cartesian covering)
 *   overlap    delta in cells (>= 0), pml_width kappa in cells (>= 0);
 *              either may be RAS_WIDTH_RULE
 *   nsub       out: number of subdomains
 *   desc       nullable; if given, nsub * RAS_DESC_INTS int32 (host memory):
 *              [0] n_local  [1] n_fast  [2] W = n_fast + 2 rounded up to
 *              even, or to a multiple of 64 when that exceeds 128 (factor
 *              column length; at most 448)  [3] x_fast  [4] first unknown
 *              node i  [5] n_x
 *              [6] first unknown node j  [7] n_y  [8] chunk p  [9] chunk q
 *              [10..13] Omega_int x lo, x hi, y lo, y hi (node indices)
 *              [14..17] Omega_j box x lo, x hi, y lo, y hi (node indices)
 *              [18] flags: bit0/1 PML added below/above in x, bit2/3 in y,
 *              bit4..7 impedance on the x-lo, x-hi, y-lo, y-hi side
 *              [19] problem index  [20] overlap delta  [21] PML width kappa
 *              [22] global PML width (cells; as resolved from the
 *              arguments, RAS_WIDTH_RULE and global_pml)  [23] reserved (0)
 *   desc_cap   capacity of desc in subdomains (ignored when desc is NULL)
 * Returns RAS_EINVAL (message via ras_pml_strerror) or RAS_ENOTSUP.        */
int ras_pml_plan(double k, double h, const int grid[2], const int subdomains[2],
                 int overlap, int pml_width, const ras_pml_opts *opts,
                 int *nsub, int *desc, int desc_cap);

/* Section 3 (iii), eq. (igg_width): overlap and PML widths of C l(k)
 * wavelengths, l(k) = k/(k - k0) log2(k/k0) (limit 1/ln 2 at k = k0); the
 * paper takes k0 = 150, C = 1/6 for the overlap delta and C = 1/2 (Tables
 * 3/4) for the PML width kappa.  Host only, touches no GPU.
 *   k, h   wavenumber and mesh width (> 0)
 *   C      width constant (>= 0), k0 reference wavenumber (> 0)
 *   cells  out: floor(C l(k) (2 pi / k) / h), the width in mesh cells
 * Returns RAS_EINVAL (message via ras_pml_plan_error) on a bad argument.    */
int ras_pml_width_rule(double k, double h, double C, double k0, int *cells);

/* Message of the last failed ras_pml_plan / setup call on this thread. */
const char *ras_pml_plan_error(void);

/* Build the operator A (Section 1), every local operator A_j with its PML
 * (Section 2, local scaling function) and impedance or Dirichlet
 * condition, and factorise every A_j once (A_j = L_j D_j L_j^T, no
 * pivoting).  Arguments as for ras_pml_plan; the handle is written to *out.
 * Synchronises `stream` before returning (the pivot check needs it).
 * Errors: RAS_EINVAL, RAS_ENOTSUP, RAS_ENOMEM, RAS_EHIP, RAS_EZEROPIVOT
 * (no handle is returned on error).                                         */
int ras_pml_setup(double k, double h, const int grid[2], const int subdomains[2],
                  int overlap, int pml_width, const ras_pml_opts *opts,
                  void *stream, ras_pml_t *out);

/* One handle for `nprob` independent problems (multi-problem batching).
 * Arrays of length nprob; every problem shares `opts`.  The unknowns of
 * problem p start at offset ras_pml_problem_offset(H, p).                 */
int ras_pml_setup_batch(int nprob, const double *k, const double *h, const int *grid,
                        const int *subdomains, const int *overlap, const int *pml_width,
                        const ras_pml_opts *opts, void *stream, ras_pml_t *out);

void ras_pml_destroy(ras_pml_t H);

/* Sizes. */
int ras_pml_num_dofs(ras_pml_t H, long long *n);        /* all problems */
int ras_pml_num_problems(ras_pml_t H, int *nprob);
int ras_pml_problem_offset(ras_pml_t H, int p, long long *off, long long *n);
int ras_pml_num_subdomains(ras_pml_t H, int *nsub);
int ras_pml_num_local(ras_pml_t H, long long *nloc);    /* sum of n_local */
int ras_pml_subdomain_desc(ras_pml_t H, int *desc, int desc_cap);  /* host */

/* b = M f : the P1 mass matrix (unweighted) applied to nodal source values
 * f at the unknowns (the source is taken as zero on the boundary of Omega).
 * Right-hand side of the weak form (Section 1, eq. (weak)).               */
int ras_pml_rhs(ras_pml_t H, const void *f, void *b, void *stream);

/* y = A x, the complex-symmetric 7-point P1 operator (Section 1). */
int ras_pml_spmv(ras_pml_t H, const void *x, void *y, void *stream);

/* z = B^{-1} v = sum_j R~_j^T A_j^{-1} R_j v (Section 2).  v and z must not
 * alias.  Deterministic: the same input gives bitwise the same output.
 * Enqueues two kernels on `stream` and nothing else (no allocation, memset
 * or synchronisation), so it can be recorded into a HIP graph by stream
 * capture (with RAS_FLAG_TIMING off: it records events).  Calls on one
 * handle share its local work vectors: they must not overlap in time.     */
int ras_pml_apply(ras_pml_t H, const void *v, void *z, void *stream);

/* Local solutions x_j = A_j^{-1} R_j v of every subdomain, back to back in
 * subdomain order (n_local each), complex128, before the PoU-weighted sum.
 * xloc may be NULL: then only the batched band solve runs (the first of
 * the two kernels of ras_pml_apply, one launch) and its result stays in the
 * handle's work vector -- for timing that kernel alone.                   */
int ras_pml_local_solve(ras_pml_t H, const void *v, void *xloc, void *stream);

/* Flexible GMRES(restart), right preconditioned by B^{-1} (Section 4.1),
 * modified Gram-Schmidt, complex Givens rotations, all Krylov arithmetic in
 * complex128.  x holds x0 on entry and the iterate on return.  Stops when
 * the true residual ||b - A x|| <= rtol ||b|| (checked at every restart and
 * at the end) or after maxit Arnoldi steps.  iters/relres (nullable) get
 * the step count and the final true relative residual; hist (nullable,
 * maxit+1 doubles, host) gets the residual estimate after every step.
 * For a batch handle every problem is solved independently with its own
 * stopping test; iters/relres then describe the slowest problem and
 * ras_pml_batch_result gives each one.  Synchronises `stream`.
 * Steps are enqueued eight at a time between looks at the convergence
 * flags; with RAS_FLAG_GRAPH_STEPS (and the fused Arnoldi step, without
 * RAS_FLAG_TIMING) the eight steps are one launch of a HIP graph, recorded
 * on the handle's own stream at the first solve (and again when restart or
 * the Krylov workspace changes) and replayed: the same kernels with the same
 * arguments as the eager steps, so the results are the same bit for bit.
 * Errors: RAS_EINVAL, RAS_ENONFINITE, RAS_ENOTCONV, RAS_EBREAKDOWN,
 * RAS_ENOMEM, RAS_EHIP.                                                    */
int gmres_solve(ras_pml_t H, const void *b, void *x, double rtol, int restart, int maxit,
                int *iters, double *relres, double *hist, void *stream);

/* gmres_solve for a batch handle with one tolerance per problem: rtol,
 * iters and relres are host arrays of ras_pml_num_problems values (iters
 * and relres nullable: the steps and final true relative residual of each
 * problem); hist as for gmres_solve (the worst problem after each step).
 * Errors as gmres_solve; RAS_ENOTCONV when some problem missed its
 * tolerance.                                                              */
int gmres_solve_batch(ras_pml_t H, const void *b, void *x, const double *rtol, int restart,
                      int maxit, int *iters, double *relres, double *hist, void *stream);

/* Algorithm 1 (Section 2) as a solver: the fixed-point iteration
 * x <- x + B^{-1} (b - A x), every step one batched local solve and the
 * PoU-weighted sum added into x, the residual in complex128.  x holds x0 on
 * entry and the iterate on return.  Stops when ||b - A x|| <= rtol ||b||
 * (checked after every step) or after maxit steps.  iters/relres
 * (nullable) get the step count and the final relative residual; hist
 * (nullable, maxit+1 doubles, host) gets the relative residual of x0 and
 * of every iterate.  Batch handles: as gmres_solve (each problem stops on
 * its own; hist and relres give the worst problem; per problem through
 * ras_pml_batch_result).  The stopping test runs on the device; the host
 * enqueues steps ahead and reads the flags every eight steps (steps
 * enqueued after a problem stopped skip it).  Synchronises `stream`.
 * Errors: RAS_EINVAL, RAS_ENONFINITE (also when a diverging iteration
 * overflows: *iters then holds the steps taken, *relres = HUGE_VAL),
 * RAS_ENOTCONV, RAS_ENOMEM, RAS_EHIP.                                       */
int ras_pml_richardson(ras_pml_t H, const void *b, void *x, double rtol, int maxit, int *iters,
                       double *relres, double *hist, void *stream);

/* ras_pml_richardson for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc): same arguments,
 * results and errors, computed by the same kernels in the same order (the
 * results equal ras_pml_richardson's bit for bit), but every buffer of the
 * solve -- the residual vector, the reduction partials and counters, the
 * per-problem state and the residual history -- lives in one static device
 * array of 64 MiB that the library holds on each device it runs on until
 * the process ends; no hipMalloc, hipFree or other allocating call is made
 * (host arrays are on the stack; the handle's own factors and local work
 * vectors, allocated by setup, are used as they are).  Limits: at most 64
 * problems per handle, and 16 * unknowns + 8 * problems * (maxit + 1) plus
 * about 8 KB per problem must fit in the 64 MiB (k = 640 with 1.7 M unknowns
 * and maxit 500 takes 27 MB); beyond them it returns RAS_EINVAL with a
 * message.  Every call on a device shares that device's array, which keeps
 * the last call's contents: calls that overlap in time on one device, on
 * any handles or streams, race and must not be made.  Timing events
 * (RAS_FLAG_TIMING) are not recorded.  Synchronises `stream`.            */
int ras_pml_richardson_noalloc(ras_pml_t H, const void *b, void *x, double rtol, int maxit,
                               int *iters, double *relres, double *hist, void *stream);

/* Per-problem outcome of the last gmres_solve or ras_pml_richardson on a
 * batch handle. */
int ras_pml_batch_result(ras_pml_t H, int p, int *iters, double *relres, int *converged);

/* ------------------------------------------------------------------------
 * Learned warm start (a learned initial guess for the solvers; an addition
 * to the paper's method).  A convolutional encoder-decoder maps the source,
 * sampled on the grid x grid nodes of the interior box (node (G + gx,
 * G + gy) for gx, gy in [0, grid), x_i = (i - G) h), to k^2 times a guess
 * of the solution on the same nodes; the guess is zero elsewhere.  Five
 * levels (grid divisible by 16), level widths c0..c4 (each 1..64, c3 == c4):
 *   e0 = relu(conv(x)), e_l = relu(conv(pool(e_{l-1}))) for l = 1..4,
 *   d3 = relu(conv(up(e4) + e3)), d2 = relu(conv(up(d3) + e2)),
 *   d1 = relu(conv(up(d2) + e1)), d0 = relu(conv(up(d1) + e0)),
 *   y = conv(d0) (2 channels);
 * conv: 3 x 3, zero padding, no bias; pool: 2 x 2 mean; up: nearest.
 * bfloat16 weights and activations, fp32 accumulation (matrix cores), fp32
 * master weights and Adam (beta 0.9 / 0.999, eps 1e-8).  Weights, in this
 * order: e0 e1 e2 e3 e4 d3 d2 d1 d0 head, each W[ky][kx][cin][cout] fp32.
 * Grids (x, y, target) are device fp32 arrays (batch, grid, grid, 2), real
 * and imaginary parts interleaved.  A network object is used by one stream
 * at a time.                                                               */
typedef struct ras_pml_wsnet *ras_pml_wsnet_t;

/* Allocates every buffer for batches up to batch_max (weights zero until
 * ras_pml_wsnet_set_weights).  Errors: RAS_EINVAL, RAS_ENOMEM.            */
int ras_pml_wsnet_create(int grid, const int channels[5], int batch_max, ras_pml_wsnet_t *out);
void ras_pml_wsnet_destroy(ras_pml_wsnet_t N);
int ras_pml_wsnet_num_weights(ras_pml_wsnet_t N, long long *n);
/* Host fp32 weights in, out (n = ras_pml_wsnet_num_weights); setting them
 * resets Adam's moments and step count.  Synchronises the device.        */
int ras_pml_wsnet_set_weights(ras_pml_wsnet_t N, const float *host, long long n);
int ras_pml_wsnet_get_weights(ras_pml_wsnet_t N, float *host, long long n);
/* y = network(x) for `batch` grids (device pointers).                    */
int ras_pml_wsnet_forward(ras_pml_wsnet_t N, const float *x, int batch, float *y, void *stream);
/* Forward, mean squared error against target, backward.  loss (host,
 * nullable: then no synchronisation) gets the mean squared error;
 * grad_host (host, nullable, ras_pml_wsnet_num_weights floats) the weight
 * gradient in the order of the weights.  The gradient stays in the object
 * for ras_pml_wsnet_adam.                                                 */
int ras_pml_wsnet_gradient(ras_pml_wsnet_t N, const float *x, const float *target, int batch,
                           double *loss, float *grad_host, void *stream);
/* One Adam step with the last gradient (learning rate lr > 0).            */
int ras_pml_wsnet_adam(ras_pml_wsnet_t N, float lr, void *stream);
/* ras_pml_wsnet_gradient followed by ras_pml_wsnet_adam.                 */
int ras_pml_wsnet_train_step(ras_pml_wsnet_t N, const float *x, const float *target, int batch,
                             float lr, double *loss, void *stream);
const char *ras_pml_wsnet_last_error(ras_pml_wsnet_t N);

/* Samples a complex128 vector over the unknowns of a single-problem handle
 * on the grid of the interior box (grid = 1/h nodes per side, as above),
 * times `scale`, into grid_out (device fp32, grid x grid x 2).            */
int ras_pml_grid_sample(ras_pml_t H, const void *vec, double scale, float *grid_out, void *stream);

/* Initial guess for gmres_solve / ras_pml_richardson: x0 = fscale *
 * network(f / fscale on the grid) / k^2 on the grid nodes, 0 elsewhere (the
 * map from f to u is linear: fscale, > 0, is the scale the network was
 * trained at); kept only if ||b - A x0|| <= ||b||, else x0 = 0.  *used
 * (nullable) = 1 when kept.  Single-problem handles whose grid equals the
 * network's.  f, b, x0: device complex128 over the unknowns.  Synchronises
 * `stream`.                                                               */
int ras_pml_warm_start(ras_pml_t H, ras_pml_wsnet_t N, const void *f, const void *b, void *x0,
                       double fscale, int *used, void *stream);

/* Inspection (tests).  All outputs are HOST memory, complex128.
 *   export_stencil: 4 * n_dofs values: the C, E, N and NE couplings of every
 *     unknown (E = to (i+1,j), N = to (i,j+1), NE = to (i+1,j+1); zero where
 *     the neighbour is not an unknown).
 *   export_local: 4 * n_local values for subdomain j in the local ordering:
 *     diagonal, fast-axis (+1), slow-axis (+n_fast), diagonal (+n_fast+1).
 *   export_factor: (n_pad * W) L entries of subdomain j, column c at
 *     c * W, row r at position r mod W (position c mod W holds 0); then the
 *     same entries by rows (row r at r * W, column c at position c mod W,
 *     position r mod W holds 0); then n_pad values of D^{-1};
 *     n_pad = n_local rounded up to 64, 2 * n_pad * W + n_pad values.      */
int ras_pml_export_stencil(ras_pml_t H, void *host_out);
int ras_pml_export_local(ras_pml_t H, int j, void *host_out);
int ras_pml_export_factor(ras_pml_t H, int j, void *host_out, long long cap_values);

/* Timing statistics recorded with RAS_FLAG_TIMING (milliseconds, summed
 * over launches since setup or the last reset).  Synchronises.            */
typedef struct {
    long long n_solve;     double solve_ms;    /* batched band solves         */
    long long n_sum;       double sum_ms;      /* PoU-weighted sums           */
    long long n_spmv;      double spmv_ms;
    long long n_mgs;       double mgs_ms;      /* projections + norms         */
    long long n_givens;    double givens_ms;
    double setup_assemble_ms, setup_factor_ms;
    double solve_bytes;    /* algorithmic bytes of one band-solve launch      */
    double factor_bytes;   /* bytes of all stored factors                     */
    double alloc_ms;       /* host wall time spent in the handle's device
                              allocations (setup and Krylov workspace; always
                              recorded, kept by reset_stats)                  */
} ras_pml_stats;
/* Launch counts cover the GMRES steps that ran: steps enqueued after every
 * problem had stopped (gmres_solve enqueues up to eight ahead of its
 * convergence test) return at once and are not counted; their few
 * microseconds remain in the times. */
int ras_pml_get_stats(ras_pml_t H, ras_pml_stats *out);
int ras_pml_reset_stats(ras_pml_t H);

/* Device-memory cache (process-wide; performance only).  Every device
 * buffer of a handle comes from it: ras_pml_destroy (and a Krylov or
 * history buffer that grows) waits for the handle's device, as hipFree
 * would, and keeps the released blocks mapped for later handles on the same
 * device whose buffers fit them (rounded size within 1/8).  A device
 * allocation that runs out of memory first hands that device's idle blocks
 * back to the driver.  Thread-safe.
 *   ras_pml_empty_cache: hands every idle block back to the driver;
 *     released_bytes (nullable) receives their total.
 *   ras_pml_set_cache_limit: most bytes kept idle (0: keep none; negative:
 *     the default, a third of the device's memory); trims idle blocks now.
 *   ras_pml_cache_info: idle and handed-out bytes (each nullable).
 *   ras_pml_fill_idle_cache: sets every byte of the current device's idle
 *     blocks to `byte` and waits (tests: a handle must not depend on what
 *     reused memory holds); RAS_EHIP if a fill fails.
 * The others return RAS_OK.                                               */
int ras_pml_empty_cache(long long *released_bytes);
int ras_pml_set_cache_limit(long long bytes);
int ras_pml_cache_info(long long *cached_bytes, long long *live_bytes);
int ras_pml_fill_idle_cache(int byte);

/* Autotuner (performance only).  Times, on this handle's own factors and
 * subdomain tables, the kernel variants whose best choice depends on the
 * band width and the number of subdomains, and keeps the fastest for the
 * handle's later calls:
 *   - per factorisation window class (tiles of 16 per side, both
 *     precisions): the blocked kernel with the matrix-core trailing update,
 *     unconstrained (variant 0) or held to the register budget of four
 *     (complex64) / two (complex128) workgroups per CU (variant 1), or the
 *     one-column kernel on the vector ALUs (variant 2); one class at a time
 *     with the others at their current choice, each timed as the whole
 *     factorisation (the classes run side by side).  The variants round
 *     differently (the blocked ones alike): the factor is formed again with
 *     the chosen variants, as a setup with these choices forms it;
 *   - the band solve's prefetch depth (RAS_KNOB_SOLVE_DEEP) and, with more
 *     subdomains than SIMDs, its dispatch (RAS_KNOB_SOLVE_QUEUE); these
 *     compute the same values bit for bit;
 *   - the fused Arnoldi step's variant (RAS_KNOB_ARNOLDI), timed on the
 *     handle's Krylov workspace (allocated for 22 vectors if smaller); the
 *     variants differ only in the rounding of their reductions.
 * cache_path (nullable): the choices are merged into this flat JSON file,
 * keyed "arch/precision/kernel/class/count" (counts rounded up to a power
 * of two), for ras_pml_opts.tune_cache.  Allocates one temporary vector;
 * synchronises `stream`.  Errors: RAS_EINVAL (no handle, or the cache file
 * cannot be written), RAS_ENOMEM, RAS_EHIP, RAS_EZEROPIVOT (a chosen
 * variant met a zero pivot).                                              */
int ras_pml_autotune(ras_pml_t H, const char *cache_path, void *stream);

/* Current variant choices: *solve_deep (1: deep prefetch); *n_groups
 * factorisation window classes, the first cap_groups of them as (tiles per
 * side, subdomains, variant 0/1/2 as in ras_pml_autotune) triples in
 * groups.  Errors: RAS_EINVAL.                                             */
int ras_pml_tuning(ras_pml_t H, int *solve_deep, int *groups, int cap_groups, int *n_groups);

/* Timings of the last ras_pml_autotune on this handle (milliseconds, best
 * of its runs): for each factorisation window class in the order of
 * ras_pml_tuning, the whole factorisation with that class at variant 0, 1
 * and 2; then the band solve at (dispatch, prefetch) = (hardware, half),
 * (hardware, deep), (queue, half), (queue, deep); then one fused Arnoldi
 * step (step index 20) in variants 0, 1, 2; 1e30 where not measured.
 * *n = 3 * classes + 7 (0 before any autotune); the first cap values go to
 * ms.  Errors: RAS_EINVAL.                                                */
int ras_pml_tune_report(ras_pml_t H, double *ms, int cap, int *n);

/* Kernel variant choices of a handle (performance only: every variant
 * computes the same values, bit for bit):
 *   RAS_KNOB_SOLVE_DEEP   band-solve prefetch depth: 1 = 16 vectors (32 for
 *                         a complex64 handle whose bands all have W <= 64),
 *                         0 = half of that (default 1);
 *   RAS_KNOB_SOLVE_QUEUE  band-solve dispatch: 0 = one wave per subdomain,
 *                         largest first, placed by the hardware dispatcher;
 *                         1 = one persistent wave per SIMD taking subdomains,
 *                         largest first, from an atomic work counter (used
 *                         only when there are more subdomains than SIMDs)
 *                         (default 0).
 *   RAS_KNOB_ARNOLDI      fused Arnoldi step variant (gmres_solve): 0 = 8
 *                         unknowns per thread, 1 = 16, both keeping v_i in
 *                         registers across the grid barrier, 2 = 12 with v_i
 *                         read again (fewer registers, more blocks per CU);
 *                         -1 = the first whose grid stays co-resident
 *                         (default); a variant whose grid would not stay
 *                         co-resident is passed over.  Reading it gives the
 *                         variant in use (-2: the one-launch-per-projection
 *                         path), or the preference before the first solve.
 * ras_pml_set_knob takes effect for the handle's later launches;
 * ras_pml_autotune sets all three from measurements.  Errors: RAS_EINVAL
 * (no handle, unknown knob or value).                                      */
enum { RAS_KNOB_SOLVE_DEEP = 0, RAS_KNOB_SOLVE_QUEUE = 1, RAS_KNOB_ARNOLDI = 2 };
int ras_pml_set_knob(ras_pml_t H, int knob, int value);
int ras_pml_get_knob(ras_pml_t H, int knob, int *value);

const char *ras_pml_strerror(int status);
const char *ras_pml_last_error(ras_pml_t H);

/* Process teardown: waits for and destroys the library's auxiliary streams
 * (one per device, used by the factorisation) and hands every idle cached
 * device block back to the driver (ras_pml_empty_cache), so that nothing of
 * the library outlives the HIP runtime or a profiler's tool library at
 * exit.  Handles still alive keep working (an auxiliary stream is created
 * again on demand) and release their blocks into the cache when destroyed.
 * The Python binding calls it from an exit hook.  Returns RAS_OK.           */
int ras_pml_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* RAS_PML_H */
