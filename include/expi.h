/*
 * expi.h - C ABI of the MI355X exponential-integrator hot path.
 *
 * Einkemmer & Ostermann, "Exponential Integrators on Graphic Processing
 * Units" (HPCS 2013).  The library evaluates the action phi_k(tau A) v of the
 * phi functions of a sparse operator A by Newton interpolation at real Leja
 * points (Sec. III-C), which reduces the work to repeated products
 * (alpha A + beta I) x (Sec. II-C, eq. (3)), and builds the exponential Euler
 * step of eq. (2) on it.  A is a matrix-free 2D/3D stencil with the boundary
 * conditions folded into it (Sec. III-A, III-B) or a CSR matrix (Sec. III-D).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Device memory.  Every vector, matrix array, coefficient array and
 *   workspace is device memory owned by the caller (the Python binding
 *   allocates it with PyTorch).  The library allocates no device memory on
 *   any call.  An operator handle BORROWS the device pointers given at
 *   creation; they must stay valid until the handle is destroyed.
 * - Streams.  `stream` is a hipStream_t passed as `void *` (NULL = the null
 *   stream).  All device work of a call is enqueued on it.  phi_action and
 *   expeuler_step bring a 128-byte status record back to pinned host memory
 *   (the last stop-test kernel of a batch of launches writes it there) a
 *   few times per Newton loop to decide how many further products to
 *   enqueue, so they return only after their device work has completed.
 *   apply_op and expi_op_interval(cached) return without synchronising.
 * - Grid vectors are contiguous, x fastest: 2D index i + nx*j, 3D index
 *   i + nx*(j + ny*k).  CSR uses int32 row pointers and column indices,
 *   float64 values, columns sorted within a row.
 * - Errors.  Every int-returning function returns EXPI_OK (0) or a negative
 *   EXPI_E* code; expi_last_error() gives a message for the calling thread.
 *   Argument validation happens before any HIP call, so it needs no GPU.
 * - Concurrency.  Calls on different streams must use different workspaces.
 *   An operator handle may be shared between threads and streams.
 */
#ifndef EXPI_H
#define EXPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define EXPI_OK            0
#define EXPI_EINVAL       -1  /* bad argument (null pointer, size, enum)         */
#define EXPI_EALIAS       -2  /* output aliases an input that is read after it   */
#define EXPI_EWORKSPACE   -3  /* workspace missing or smaller than required      */
#define EXPI_ENOTCONV     -4  /* no convergence within m_max after all retries   */
#define EXPI_ENONFINITE   -5  /* a norm became inf/NaN (input not finite)        */
#define EXPI_EHIP         -6  /* a HIP runtime call failed                       */
#define EXPI_EUNSUPPORTED -7  /* combination not implemented (e.g. k>=2, s>1)    */

/* ---- enums -------------------------------------------------------------- */
/* Storage of the Newton vectors w_j and the running sum p.  Solution vectors
 * (v, y of phi_action; u of expeuler_step) are always float64; divided
 * differences, norms and the stop test are always float64. */
#define EXPI_F64 0
#define EXPI_F32 1

/* Boundary handling folded into the stencil (Sec. II-C: "incorporated into
 * the matrix A"; Sec. III-A's two options). */
#define EXPI_DIRICHLET0    0  /* u = 0 beyond the array; the face towards the
                                 missing neighbour carries the cell's own a  */
#define EXPI_NEUMANN0      1  /* zero flux through the boundary faces        */
#define EXPI_INTERIOR_ONLY 2  /* rows of the outermost layer are zero: only
                                 points whose stencil lies inside are updated */

/* Diffusion coefficient a of div(a grad u); face value = mean of the two
 * adjacent grid values (Sec. III-B uses a position-dependent coefficient). */
#define EXPI_COEF_CONST     0 /* a = c0                                        */
#define EXPI_COEF_SEPARABLE 1 /* a = c0 + c1 * tx[i] * ty[j] (* tz[k])          */
#define EXPI_COEF_FIELD     2 /* a = field[index], float64, same layout as u    */
#define EXPI_COEF_DLAP      3 /* the operator is c0 * D(x, y) times the
                                 constant-coefficient stencil Laplacian, with
                                 D = 1/sqrt(1 + x^2 + y^2) computed in the
                                 kernel (Sec. III-B, Table II); grid
                                 positions: index i at (i + 1) h (DIRICHLET0),
                                 (i + 1/2) h (NEUMANN0), i h (INTERIOR_ONLY)  */

/* Inhomogeneous Dirichlet data of Sec. III-A (the rows of Table I with
 * boundary values f): the product becomes affine, A_0 u + b_f, where the
 * stencil reads f at the boundary node instead of 0 (expi_op_set_boundary_data). */
#define EXPI_BDATA_NONE          0
#define EXPI_BDATA_Z1MZ_XY       1  /* f = z (1 - z) x y                       */
#define EXPI_BDATA_SINPIZ_EXPMXY 2  /* f = sin(pi z) exp(-x y)                 */
#define EXPI_BDATA_IN_KERNEL     0  /* f evaluated inside the stencil sweep    */
#define EXPI_BDATA_SEPARATE      1  /* a second kernel adds the boundary term  */

/* Pointwise nonlinearity g of u' = A u + g(u). */
#define EXPI_G_CUBIC           0  /* g(u) = u - u^3                              */
#define EXPI_G_COMBUSTION      1  /* g(u) = (2 - u)/4 exp(20 (1 - 1/u)), the
                                     combustion model of Sec. III-C, eq. (4)-(5),
                                     IEEE division and the library exp          */
#define EXPI_G_COMBUSTION_FAST 2  /* the same through the hardware FP32
                                     reciprocal and base-2 exponential (Table
                                     III's fast math; relative error ~1e-6)     */

/* ---- types -------------------------------------------------------------- */
typedef struct expi_op expi_op;   /* opaque operator handle */

/* Per-call statistics (any field may be left 0 by an early error). */
typedef struct {
    int32_t substeps;       /* s: number of substeps of the last attempt        */
    int32_t newton_steps;   /* products inside the Newton loops                 */
    int32_t matvecs;        /* all products with A (Newton + start vectors)     */
    int32_t retries;        /* substep doublings after a non-converged substep  */
    int32_t converged;      /* 1 if every substep met the stop test             */
    int32_t degree_max;     /* largest Newton degree m over the substeps        */
    int32_t degree_last;    /* Newton degree of the last substep                */
    int32_t timed_products; /* fused Newton products timed (params.profile)     */
    double  err_est;        /* largest (t_{m-1} + t_m)/||p|| over the substeps  */
    double  interval_a;     /* spectral interval [a, b] used                    */
    double  interval_b;
    double  newton_ms;      /* summed device time of the Newton sweep launches
                               (single products and pair sweeps; HIP events
                               recorded on `stream` around each launch) that
                               did work: launches that began before the stop */
    double  rnorm;          /* ||r|| of the first substep's start vector        */
    double  t_first[5];     /* |d_j| ||w_j||, j = 0..4, of the first substep
                               (features of the step selector)                 */
    int32_t pred_degree;    /* step selector: predicted degree (0 if unused)    */
    int32_t pred_substeps;  /* step selector: predicted substep count           */
    int32_t fallback;       /* step selector: products beyond the prediction     */
    int32_t finalized;      /* products whose norms were reduced (stop tests)   */
    int32_t timed_pairs;    /* pair sweeps among the timed launches (each covers
                               two products; timed_products counts both)       */
    double  pair_ms;        /* summed device time of those pair sweeps          */
    int32_t pair_launches;  /* pair sweeps that did work (began before the stop) */
    int32_t single_launches;/* single-product sweeps that did work              */
    int32_t fused_starts;   /* start vectors formed inside a pair sweep         */
    int32_t reserved3;
} expi_stats;

/* Interpolation parameters; pass NULL for the defaults
 * (l_max = 100, m_max = 100, max_retries = 4, Gershgorin interval,
 * no profiling). */
typedef struct {
    double  l_max;          /* largest delta*(b-a) per substep                   */
    int32_t m_max;          /* largest number of Newton products per substep    */
    int32_t max_retries;    /* substep doublings after a non-converged substep  */
    int32_t have_interval;  /* 1: use [interval_a, interval_b] below            */
    int32_t profile;        /* 1: time each fused Newton launch from product 1
                             * on (stats); 2: only the first of each Newton
                             * loop (two timing events per loop instead of two
                             * per launch); other values: EXPI_EINVAL         */
    double  interval_a;
    double  interval_b;
    /* Learned step selector (optional): device float buffer laid out as
     * x_mean[8], x_std[8], y_mean[2], y_std[2], then the network parameters
     * (expi_mlp_param_count(selector_hidden) values).  When set, each Newton
     * loop takes its first four products with stop tests, the network
     * predicts the degree m from the features (interval, tau, ||r||,
     * t_0..t_4), the products up to m run without norm reductions, and the
     * two-term stop test judges the result at m; if it is not met the plain
     * error-controlled loop continues (fallback). */
    const void *selector;
    int32_t selector_hidden;
    /* 1: never fuse two Newton products into one sweep.  By default, on 3D
     * stencils with a constant or separable coefficient and rows of at most
     * 512 points, and on 2D stencils with a constant coefficient (any
     * boundary handling), consecutive products run
     * as pair sweeps that keep w_{j+1} on chip (same arithmetic, half the
     * vector traffic) and test the stop rule after each of the two (unless
     * the operator's pair setting, expi_op_set_pairs, is 0). */
    int32_t no_pairs;
    /* Exponential Euler steps: the start-vector sweep r = A u + u - u^3 of
     * the first substep can run as the first half of a pair sweep whose
     * second half is Newton product 0 (pair sweeps on, u 16-byte aligned;
     * with FP32 storage r is still formed in FP64, from the FP64 u, and
     * rounded to FP32); a stop at degree m then takes ceil((m+1)/2) sweeps
     * instead of 1 + ceil(m/2).  0: fuse when the previous step with the
     * same step size stopped at an odd degree; 1: never; 2: whenever it
     * applies.  Other values: EXPI_EINVAL. */
    int32_t fuse_start;
    /* Learned step selector, exponential Euler steps: the largest
     * delta*(b-a) per substep the network's substep count may reach
     * (0: 500).  A predicted substep count s' with
     * ceil(tau (b-a) / selector_l_max) <= s' < s (s from l_max) restarts the
     * step with s' substeps, each run with the predicted degree and its
     * two-term stop test; if a substep then misses the test within m_max
     * products, the step is redone by the plain method with s substeps
     * (counted in stats.fallback). */
    double  selector_l_max;
    /* Optional device float[8]: the selector kernel writes the raw features
     * of its last prediction there (for checking them against the host). */
    void   *selector_features;
} expi_params;

/* ---- operators ---------------------------------------------------------- */

/* Matrix-free stencil A = div(a grad .) discretised with the 5-point (dim 2)
 * or 7-point (dim 3) formula of Sec. III-A, boundary handling `bc` folded in,
 * coefficient per Sec. III-B:
 *   (A u)_c = sum over the 2*dim faces f of c:  a_f (u_nb - u_c) / h_d^2,
 * a_f = (a_c + a_nb)/2.  For a = 1 and EXPI_DIRICHLET0 this is exactly the
 * paper's seven-point formula divided by (dx)^2.
 *   n[dim], h[dim]: host arrays, x first.  n[d] >= 1, product < 2^30.
 *   tab_x/tab_y/tab_z: device float64 tables of length n[0], n[1], n[2]
 *   (SEPARABLE only; tab_z ignored in 2D).  field: device float64 array of
 *   the grid's size (FIELD only).  Borrowed.
 * Returns EXPI_EINVAL on a bad dim/size/spacing/enum or a missing table. */
int expi_op_create_stencil(expi_op **op, int dim, const int64_t *n, const double *h,
                           int bc, int coef_kind, double c0, double c1,
                           const double *tab_x, const double *tab_y, const double *tab_z,
                           const double *field);

/* Boundary data of a 3D DIRICHLET0 stencil (node grid, boundary nodes at
 * coordinates 0 and (n_d + 1) h_d): kind EXPI_BDATA_*, mode
 * EXPI_BDATA_IN_KERNEL (f evaluated by the sweep at boundary-adjacent
 * points) or EXPI_BDATA_SEPARATE (a second launch over the boundary layer adds
 * the term; Sec. III-A compares the two).  Afterwards apply_op computes
 * y = alpha (A_0 x + b_f) + beta x, and expeuler_step / exprk2_step solve
 * u' = A_0 u + b_f + g(u).  phi_action is unaffected (it uses the linear
 * part A_0).  EXPI_EINVAL for a CSR operator, 2D, another boundary condition,
 * EXPI_COEF_DLAP, or an unknown kind/mode.  EXPI_BDATA_NONE switches it off. */
int expi_op_set_boundary_data(expi_op *op, int kind, int mode);

/* CSR matrix (Sec. III-D): n rows, nnz entries; rowptr int32[n+1],
 * colind int32[nnz] (sorted per row), val float64[nnz]; device, borrowed. */
int expi_op_create_csr(expi_op **op, int64_t n, int64_t nnz, const int32_t *rowptr,
                       const int32_t *colind, const double *val);

/* Complex Hermitian matrix H in CSR (Sec. II-C allows K = C; Sec. III-D's
 * spin system is stored this way): val holds complex128 values as nnz
 * interleaved (re, im) float64 pairs; rowptr, colind as for
 * expi_op_create_csr.  The operator serves apply_op (x, y complex128 pairs,
 * EXPI_F64 only; alpha, beta real) and expi_skew_phi_action; phi_action and
 * the integrator steps refuse it.  H is assumed Hermitian: its Gershgorin
 * interval uses the real part of the diagonal. */
int expi_op_create_csr_complex(expi_op **op, int64_t n, int64_t nnz, const int32_t *rowptr,
                               const int32_t *colind, const double *val);

int expi_op_destroy(expi_op *op);

/* Number of unknowns of the operator. */
int64_t expi_op_size(const expi_op *op);

/* Tile setting of the operator's sweeps (the autotuner's knob; results do
 * not depend on it beyond rounding order).  Stencils: vec = x points per
 * thread (1 or 2; 2 needs an even x size and 16-byte aligned arrays, else 1
 * is used), waves = 64-thread waves per workgroup (1..8, rows of a 3D tile),
 * march = points each thread marches along the slowest axis (4..120, a
 * multiple of 4).
 * CSR: vec = lanes per row (4, 8 or 16), waves (1..8), march = 1.
 * EXPI_EINVAL for anything else.  The workspace size does not depend on it. */
int expi_op_set_tiles(expi_op *op, int vec, int waves, int march);
int expi_op_get_tiles(const expi_op *op, int *vec, int *waves, int *march);

/* Pair sweeps (two consecutive Newton products per pass, Sec. III-C's
 * Newton recurrence taken two steps at a time; on 3D stencils with a
 * constant or separable coefficient and rows of at most 512 points, and on
 * 2D stencils with a constant coefficient and any boundary handling):
 * use = 1 (the default) takes them wherever they
 * apply, 0 runs single products.  On a 2D operator with pair sweeps,
 * use = 4..64 (a multiple of 4) takes them with tiles of that many grid
 * rows (with 1 the height follows the grid size: 16 rows, fewer where the
 * grid has too few tiles for the device).  EXPI_EINVAL for other values.
 * expi_op_get_pairs returns the stored value (0, 1 or a row count). */
int expi_op_set_pairs(expi_op *op, int use);
int expi_op_get_pairs(const expi_op *op, int *use);

/* Autotuner: times the fused Newton product (the hot loop's sweep, each
 * product doing full work) under every candidate tile setting on this
 * operator and storage dtype, `reps` launches each after one warm-up, with
 * HIP events on `stream`, and keeps the fastest as the operator's setting.
 * Candidates: stencils vec {2,1} x waves {1,2,4,8} x march {8,16,32,64}
 * (3D) or {4,8,16,32} (2D); CSR lanes {4,8,16} x waves {1,2,4,8}.  Where
 * a pair sweep applies, it is timed last (listed as (0, 0, 2), time per
 * launch of two products) and the operator's pair setting becomes 1 if it
 * takes less per product than the best single product, else 0.  A 2D pair
 * sweep is timed at tile heights 4, 8, 16 and, where the grid has the
 * rows, 32 and 64 (listed as (0, rows, 2)); the pair setting becomes the
 * fastest height if that one takes less per product than the best single
 * product, else 0.  The
 * workspace (expi_workspace_bytes(op, dtype)) supplies the vectors and is
 * overwritten.  If cand/us are given, the first max_cand tried settings
 * (vec, waves, march triples) and their mean microseconds per launch are
 * written there; *n_cand receives the number tried.  Synchronises `stream`. */
int expi_op_autotune(expi_op *op, int dtype, int reps, void *ws, size_t ws_bytes, void *stream,
                     int *cand, float *us, int max_cand, int *n_cand);

/* Bytes of device workspace phi_action / expeuler_step / expi_op_interval
 * need for this operator and storage dtype (EXPI_F64 or EXPI_F32). */
size_t expi_workspace_bytes(const expi_op *op, int dtype);

/* Gershgorin interval [a, b] of A (Sec. II-C needs an a-priori bound of the
 * field of values): a = min_i (A_ii - R_i), b = max_i (A_ii + R_i),
 * R_i = sum_{j != i} |A_ij|.  Computed on the device once per handle (one
 * sweep over the operator, then a 128-byte read-back on `stream`) and cached. */
int expi_op_interval(expi_op *op, double *a, double *b, void *ws, size_t ws_bytes,
                     void *stream);

/* ---- the three calls of the hot path ------------------------------------ */

/* y = (alpha A + beta I) x   (eq. (3)).  x, y: device arrays of the
 * operator's size, float64 (dtype EXPI_F64) or float32 (EXPI_F32); y must not
 * alias x (EXPI_EALIAS).  One kernel launch on `stream`, no synchronisation. */
int apply_op(const expi_op *op, double alpha, double beta, const void *x, void *y,
             int dtype, void *stream);

/* y = phi_k(tau A) v by Newton interpolation at Leja points (Sec. III-C,
 * Sec. II-C), 0 <= k <= 20, any substep count.  Substeps of phi_k, k >= 1,
 * follow y(t) = t^k phi_k(tA) v, the solution of y' = A y + t^(k-1)/(k-1)! v,
 * y(0) = 0: each substep after the first takes k extra products for its
 * start vector (matvecs counts them).  v, y: float64 device arrays; y must
 * not alias v.  tol: relative 2-norm tolerance of the two-term stop test per
 * substep.  dtype: storage of the Newton vectors (EXPI_F64 / EXPI_F32).
 * ws: device workspace of at least expi_workspace_bytes(op, dtype) bytes,
 * 256-byte aligned.  st may be NULL.  On EXPI_ENOTCONV y holds the last
 * attempt's result; on EXPI_ENONFINITE its contents are unspecified. */
int phi_action(expi_op *op, int k, double tau, const double *v, double *y, double tol,
               int dtype, const expi_params *params, void *ws, size_t ws_bytes,
               expi_stats *st, void *stream);

/* y = phi_k(-i tau H) v for a Hermitian H (complex CSR operator), k = 0
 * (y = e^{-i tau H} v, the solution of psi' = -i H psi at tau) or 1.  The
 * Newton recurrence is that of phi_action with A replaced by H: real
 * products (alpha H + beta_j I) x of complex vectors (eq. (3) with K = C),
 * real Leja points of [-2, 2] mapped to the Gershgorin interval [a, b] of H,
 * and complex divided differences of x -> phi_k(-i delta (c + gamma x)).
 * Substeps as in phi_action (s = ceil(tau (b - a) / l_max)); for k = 1,
 * y(t) = t phi_1(-i t H) v solves y' = -i H y + v.  v, y: complex128 device
 * arrays as interleaved (re, im) pairs; FP64 storage; ws: at least
 * expi_workspace_bytes(op, EXPI_F64) bytes.  Errors as for phi_action
 * (EXPI_EINVAL for a real operator or k not 0/1). */
int expi_skew_phi_action(expi_op *op, int k, double tau, const double *v, double *y, double tol,
                         const expi_params *params, void *ws, size_t ws_bytes, expi_stats *st,
                         void *stream);

/* One exponential Euler step (eq. (2)) for u' = A u + g(u), written as
 * u <- u + tau phi_1(tau A) (A u + g(u)), which equals eq. (2) in exact
 * arithmetic and needs one phi_1 action.  u: float64 device array, updated in
 * place only when the step converged (left unchanged on any error).
 * nonlin: EXPI_G_CUBIC, EXPI_G_COMBUSTION or EXPI_G_COMBUSTION_FAST.  Other
 * arguments as for phi_action. */
int expeuler_step(expi_op *op, int nonlin, double tau, double *u, double tol, int dtype,
                  const expi_params *params, void *ws, size_t ws_bytes, expi_stats *st,
                  void *stream);

/* One step of the second-order exponential Runge-Kutta method with c_2 = 1
 * (a higher-order exponential integrator of the kind Sec. II-C points to):
 *   U = u + tau phi_1(tau A)(A u + g(u))          (the exponential Euler step)
 *   u <- U + tau phi_2(tau A)(g(U) - g(u)).
 * Two Newton loops (phi_1, then phi_2).  ws: at least
 * expi_exprk2_workspace_bytes(op, dtype) bytes (phi_action's workspace plus
 * one float64 vector).  u is overwritten by the result only when both
 * actions converged; on an error in the second one it holds the stage U.
 * st sums the counts of both loops (degree_last: the phi_2 loop's). */
size_t expi_exprk2_workspace_bytes(const expi_op *op, int dtype);
int exprk2_step(expi_op *op, int nonlin, double tau, double *u, double tol, int dtype,
                const expi_params *params, void *ws, size_t ws_bytes, expi_stats *st,
                void *stream);

/* g = nonlinearity(u) pointwise over n values (the kernel Table III times):
 * u, g device arrays of float64 (dtype EXPI_F64) or float32 (EXPI_F32); g
 * may equal u (in place) but must not overlap it otherwise.  One launch on
 * `stream`, no synchronisation. */
int expi_nonlinearity(int nonlin, int64_t n, const void *u, void *g, int dtype, void *stream);

/* ---- allocation-free variant of phi_action ------------------------------- */

/* For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid hipMalloc).  The library holds one scratch array of
 * EXPI_NOALLOC_SCRATCH_BYTES in device memory (a static device variable of
 * the library's code object, present on every GPU the library runs on until
 * the process ends) and uses it as phi_action's workspace.
 *
 * expi_noalloc_init: set-up, once per (host thread, device), with that device
 * current: looks up the device address of this device's scratch array and
 * prepares the calling thread's pinned status slots and timing events (these
 * are allocations, so they belong here and not in the call).  EXPI_EHIP if a
 * HIP call fails.
 *
 * phi_action_noalloc: phi_action with the scratch array as workspace; same
 * arguments, results and errors, minus ws/ws_bytes.  It calls no hipMalloc,
 * hipFree or other allocating routine.  EXPI_EINVAL if expi_noalloc_init has
 * not run on this thread and device; EXPI_EWORKSPACE if the operator needs
 * more than EXPI_NOALLOC_SCRATCH_BYTES (expi_workspace_bytes(op, dtype):
 * about 32 bytes per unknown in FP64, so up to about 2 million unknowns).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (the status record is reset by each call): calls that overlap in
 * time on one GPU, from any thread or stream, race and must not be made. */
#define EXPI_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int expi_noalloc_init(void);
int phi_action_noalloc(expi_op *op, int k, double tau, const double *v, double *y, double tol,
                       int dtype, const expi_params *params, expi_stats *st, void *stream);

/* ---- many problems in one batch ------------------------------------------ */

/* A batch of independent 2D problems y_i = phi_1(tau_i A_i) v_i, A_i the
 * constant-coefficient 5-point operator coef * Laplacian on an nx_i x ny_i
 * grid with spacings hx_i, hy_i and boundary handling `bc` (DIRICHLET0 or
 * NEUMANN0), each by the same Leja interpolation as phi_action (Sec. III-C),
 * all of them together.  The host computes each interval (closed-form
 * Gershgorin bound [-4 coef (1/hx^2 + 1/hy^2), 0]), substep count and
 * divided differences at creation.  Vectors of all instances are
 * concatenated: instance i occupies [off_i, off_i + nx_i ny_i) of v and y
 * (float64, device), with off_i from expi_batch_offsets and total length
 * expi_batch_total_length.  dtype sets the storage of the Newton vectors
 * (EXPI_F32 for the FP32-storage mode); divided differences, norms, the stop
 * test and y stay float64.
 *
 * The work runs in rounds; in each round every unfinished instance takes one
 * step (start vector, Newton products, or the substep update).  A round is
 * three kernels (the tiles of the instances whose step is a start vector,
 * an update or a product that reads the float64 input; the tiles of the
 * other products; then one stop test per instance); nothing inside waits
 * on memory.  By default a step after the first product forms two Newton
 * products in one pass (expi_batch_set_pairs): w_{j+1} stays in registers,
 * so w_j and p are read and w_{j+2} and p written once for both, and the
 * stop test is applied after each of the two as single products would
 * apply it (a stop after the first leaves the second product's term in p,
 * and the update subtracts it); newton_steps then counts both products.  At
 * most expi_batch_max_rounds rounds are needed.  No retries: an instance
 * that misses the stop test within m_max products reports EXPI_ENOTCONV. */
typedef struct expi_batch expi_batch;
typedef struct {
    int32_t status;         /* 0, EXPI_ENOTCONV or EXPI_ENONFINITE            */
    int32_t substeps;
    int32_t newton_steps;   /* products over all substeps                     */
    int32_t degree_max;
    int32_t degree_last;
    int32_t reserved;
    double  err_est;        /* largest (t_{m-1} + t_m)/||p|| over the substeps */
} expi_batch_stat;

int expi_batch_create(expi_batch **b, int count, const int32_t *nx, const int32_t *ny,
                      const double *hx, const double *hy, const double *tau, int bc,
                      double coef, double tol, int dtype, const expi_params *params);
int expi_batch_destroy(expi_batch *b);
/* Tile setting of the batch's sweeps: waves per workgroup (1..8), rows
 * marched per thread (4..64, multiple of 4).  Requires expi_batch_prepare
 * again; not allowed after expi_batch_capture. */
int expi_batch_set_tiles(expi_batch *b, int waves, int march);
int64_t expi_batch_total_length(const expi_batch *b);
int expi_batch_offsets(const expi_batch *b, int64_t *off /* count entries */);
size_t expi_batch_workspace_bytes(const expi_batch *b);
/* Upper bound on the rounds any instance needs: the largest substep count
 * times (m_max + 2), plus 2. */
int expi_batch_max_rounds(const expi_batch *b);
/* Upload the instance table to the workspace (host-to-device copies), size
 * the grids from the occupancy of this device; synchronises. */
int expi_batch_prepare(expi_batch *b, void *ws, size_t ws_bytes, void *stream);
/* Solve the batch: enqueue the state reset and rounds on `stream` until
 * every instance has finished, reading a 64-byte status block back to
 * pinned host memory after every 8 rounds (one chunk of rounds stays
 * enqueued ahead of the check).  Returns after the device is done (the
 * call synchronises `stream`); results via expi_batch_results.  y must not
 * overlap v (EXPI_EALIAS). */
int expi_batch_launch(expi_batch *b, const double *v, double *y, void *ws, size_t ws_bytes,
                      void *stream);
/* Build a HIP graph (owned by the batch) of the state reset and `rounds`
 * rounds as kernel nodes, for v, y and ws as given; rounds more than
 * expi_batch_max_rounds take expi_batch_max_rounds, enough for every
 * instance.  rounds = 0: the rounds the last expi_batch_launch needed plus
 * 1/64 and 8 more (the same inputs need exactly as many), or
 * expi_batch_max_rounds if there was none.  Rounds after the last instance
 * finished return at once.  With too few rounds, unfinished instances
 * report EXPI_ENOTCONV (expi_batch_results).  Replay with
 * expi_batch_replay (asynchronous, one graph launch on `stream`).  The
 * graph holds no copies or fills.  `stream` of capture is unused. */
int expi_batch_capture(expi_batch *b, const double *v, double *y, void *ws, size_t ws_bytes,
                       int rounds, void *stream);
int expi_batch_replay(expi_batch *b, void *stream);
/* Autotuner: solves the batch (v, y, ws as for expi_batch_launch; y is
 * overwritten) under every candidate tile setting, waves {2,4,8} x march
 * {4,8,16,32}, one warm-up and `reps` timed solves each (host wall clock
 * around the synchronising solve), and keeps the fastest, prepared for
 * `ws`.  A captured graph is dropped.  If cand/ms are given, the first
 * max_cand (waves, march) pairs tried and their milliseconds per solve are
 * written there; *n_cand receives the number tried. */
int expi_batch_autotune(expi_batch *b, const double *v, double *y, void *ws, size_t ws_bytes,
                        int reps, void *stream, int *cand, float *ms, int max_cand, int *n_cand);
int expi_batch_get_tiles(const expi_batch *b, int *waves, int *march);
/* Newton products two per round (on = 1, the default) or one per round
 * (on = 0); the same interpolant up to rounding and the stop decisions
 * rounding can move.  EXPI_EINVAL for other values or after
 * expi_batch_capture (the captured graph holds the setting); applies to the
 * next solve, persistent or in rounds. */
int expi_batch_set_pairs(expi_batch *b, int on);
int expi_batch_get_pairs(const expi_batch *b, int *on);
/* Rounds of the captured graph (0 if none). */
int expi_batch_graph_rounds(const expi_batch *b);
/* Read per-instance results back (synchronises); returns EXPI_OK if every
 * instance converged.  `rounds` (may be NULL) receives the rounds in which
 * some instance was still unfinished. */
int expi_batch_results(expi_batch *b, void *ws, void *stream, expi_batch_stat *out, int *rounds);
/* All rounds in ONE persistent kernel (Sec. III-C's method per instance, as
 * expi_batch_launch): the tiles of a round in grid-stride order, grid
 * barriers between them and the round's stop tests, a cooperative launch
 * so that every workgroup is resident; directly or as a cooperative graph
 * node (replays run the whole solve).  Needs expi_batch_prepare with this workspace.
 * Every wait is bounded: a grid barrier wait past 2 s aborts the launch,
 * and expi_batch_results then returns EXPI_EHIP. */
int expi_batch_launch_persistent(expi_batch *b, const double *v, double *y, void *ws,
                                 size_t ws_bytes, void *stream);
int expi_batch_capture_persistent(expi_batch *b, const double *v, double *y, void *ws,
                                  size_t ws_bytes, void *stream);

/* ---- step-selector network (float32, device buffers) --------------------- */

/* Network 8 -> H -> H -> 2 (ReLU); parameters packed as W1 (H x 8, row-major),
 * b1 (H), W2 (H x H), b2 (H), W3 (2 x H), b3 (2).  Returns 0 for H outside
 * [1, 256]. */
size_t expi_mlp_param_count(int hidden);
/* Floats of scratch memory expi_mlp_backward needs for n samples. */
size_t expi_mlp_scratch_floats(int hidden, int n);
/* out[n x 2] = network(x[n x 8]); act (n x 2H, may be NULL) keeps the
 * pre-activations for the backward pass. */
int expi_mlp_forward(int hidden, const float *params, const float *x, int n, float *out,
                     float *act, void *stream);
/* Gradient of the asymmetric loss L = 1/(2n) sum w (out - target)^2,
 * w = kappa where out < target, else 1, into grad (param_count floats);
 * *loss (device float, may be NULL) receives L.  Sample sums run in index
 * order (deterministic). */
int expi_mlp_backward(int hidden, const float *params, const float *x, const float *act,
                      const float *out, const float *target, int n, float kappa, float *grad,
                      float *loss, float *scratch, void *stream);
/* One Adam step (bias-corrected moments), step counts from 1. */
int expi_mlp_adam(int count, float *params, const float *grad, float *m, float *v, int step,
                  float lr, float beta1, float beta2, float eps, void *stream);

/* ---- host-side interpolation data (no GPU needed) ----------------------- */

/* The first `count` (1..256) real Leja points of [-2, 2]: xi_0 = 2 and xi_k
 * maximises prod_{j<k} |x - xi_j| over [-2, 2], ties to the larger point. */
int expi_leja_points(double *out, int count);

/* Divided differences f[xi_0..xi_j], j < count, of
 * f(x) = phi_k(delta (c + gamma x)) at the Leja points (the coefficients of
 * the Newton form that approximates phi_k(delta A) for (A - cI)/gamma with
 * spectrum in [-2, 2]).  count <= 256. */
int expi_divided_differences(int k, double delta, double c, double gamma, int count,
                             double *out);

/* Complex divided differences f[xi_0..xi_j], j < count, of
 * f(x) = phi_k(-i delta (c + gamma x)) (real parts into re, imaginary parts
 * into im): the coefficients expi_skew_phi_action uses.  count <= 256. */
int expi_divided_differences_skew(int k, double delta, double c, double gamma, int count,
                                  double *re, double *im);

/* Thread-local message of the last error (never NULL). */
const char *expi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EXPI_H */
