/*
 * rcp.h -- C interface of librcp, randomized CP decomposition on AMD MI355X
 * (gfx950).
 *
 * Method: Erichson, Manohar, Brunton, Kutz, "Randomized CP Tensor
 * Decomposition".  Section 3.1 / Algorithm 1 (randomized tensor
 * compression), Section 3.2.1 / Algorithm 2 (CP-ALS on the compressed
 * tensor, back-projection eq. qbs), Section 3.3 (fit and stopping rule).
 *
 * Conventions shared by every entry point
 *   - Tensors are dense, float32, C order (last index fastest).  Matrices are
 *     row-major.  Mode indices are 0-based.
 *   - Every tensor / matrix pointer is a DEVICE pointer unless stated.
 *     Arrays of pointers (``float* const* A``) are HOST arrays of device
 *     pointers, one per mode.
 *   - l_n = min(k + p_n, I_n) is the sketch width of mode n (p_n = p unless
 *     rcp_problem.per_mode_p; l_n = I_n for a mode left out of
 *     compress_mask); the core has dims l_0 x ... x l_{N-1}; R = k is the
 *     CP rank.
 *   - The library never allocates device memory.  The caller provides one
 *     workspace buffer (size from rcp_workspace_size) and every input and
 *     output buffer; the library owns only the host-side plan object.
 *   - Calls only enqueue work on the HIP stream given to rcp_init and return
 *     without synchronising.  The returned status covers argument checking
 *     and launch errors only.  Numeric outcomes (Cholesky fallback taken, a
 *     non-finite fit) are written to the device-side rcp_als_info.
 *   - A plan is not thread-safe; distinct plans are independent.  Calls on
 *     one plan must not overlap (they share the workspace), which holds
 *     automatically when they are issued on the plan's stream.
 *   - The library never aborts, throws across this interface or prints.
 */
#ifndef RCP_H_
#define RCP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rcp_status {
    RCP_OK = 0,
    RCP_ERR_INVALID_ARG = 1,   /* bad size, null or misaligned pointer, aliasing */
    RCP_ERR_WORKSPACE = 2,     /* workspace missing or too small */
    RCP_ERR_HIP = 3,           /* a HIP runtime call or kernel launch failed */
    RCP_ERR_NUMERIC = 4,       /* reserved for synchronous numeric failures */
    RCP_ERR_UNSUPPORTED = 5    /* valid request the library does not implement */
} rcp_status;

/* rcp_problem.precision: operand precision of the range finder's
 * contractions (the sketch and the power-iteration products of Algorithm 1
 * the sketch and the power iterations' products).  FP32 feeds the matrix cores float32 operands; BF16 /
 * FP16 round the float32 tensor tiles and the test-matrix or basis operands
 * to bfloat16 / float16 (nearest even) on their way to the matrix cores.
 * Their rounding only perturbs the basis Q_n.  The mode products of the projection
 * B <- B x_n Q_n^T (Algorithm 1),
 * whose output is the core itself, keep float32 operands in every precision.
 * Accumulation is float32, and the cross-workgroup sums, the QR and every
 * ALS solve stay float64 in all cases; X is read as float32. */
enum { RCP_PREC_FP32 = 0, RCP_PREC_BF16 = 1, RCP_PREC_FP16 = 2 };

/* rcp_problem.scheme (Section 3.1): SEQUENTIAL sketches mode n on the tensor
 * already compressed in modes < n, as Algorithm 1 does (it replaces X by
 * B_n after each mode); INDEPENDENT takes every basis from X itself and
 * forms the core by chained mode products afterwards. */
enum { RCP_SCHEME_SEQUENTIAL = 0, RCP_SCHEME_INDEPENDENT = 1 };

/* rcp_problem.test_matrix: Omega_n of Algorithm 1 (the test-matrix draw), a pure function of
 * (seed, mode, batch, row j, column c), never stored:
 *   GAUSSIAN  N(0, 1) entries (Section 3.1): Philox4x32-10 on the counter
 *             (j mod 2^32, j >> 32, c / 4, (batch << 8) | mode) with key
 *             (seed mod 2^32, seed >> 32), uniforms ((x >> 8) + 1) 2^-24,
 *             Box-Muller on the pairs (u0, u1), (u2, u3);
 *   UNIFORM   the uniforms themselves, entry c taking word c mod 4 (the
 *             rand(J, l) of Algorithm 1's test-matrix draw; the remark after it);
 *   HALTON    quasi-random (the note in Section 3.1): entry (j, c) is the
 *             radical inverse of j + 1 in the c-th prime base (no seed);
 *   COLUMNS   l randomly selected columns of the unfolding (the remark after
 *             Algorithm 1): Floyd's sampling without replacement, draw s
 *             taking t = floor(x (i + 1) / 2^64) on {0..i}, i = J - l + s,
 *             x = (word1 << 32) | word0 of the counter (s mod 2^32, s >> 32,
 *             2^31, (batch << 8) | mode); indices sorted ascending; needs
 *             l_n <= J_n (the product of the other current mode sizes). */
enum { RCP_TEST_GAUSSIAN = 0, RCP_TEST_UNIFORM = 1, RCP_TEST_HALTON = 2, RCP_TEST_COLUMNS = 3 };

/* rcp_problem.solver: the CP solver rcp_decompose runs on the core.  ALS is
 * Section 3.2.1 / Algorithm 2 (rcp_als); BCD is the rank-one block coordinate
 * descent of Section 3.2.2 / Algorithm 3 (rcp_bcd), whose max_iters and tol
 * apply to each component.  CP_ALS is the deterministic method the
 * randomized one is measured against (Section 3.3): Algorithm 2 on X itself,
 * no compression (rcp_cp_als); its plan sizes the workspace for that. */
enum { RCP_SOLVER_ALS = 0, RCP_SOLVER_BCD = 1, RCP_SOLVER_CP_ALS = 2 };

/* Device-side status bits: rcp_als_info.status holds those of one CP-ALS
 * run (the first three); the plan's status word (rcp_read_status) collects
 * every bit any call on the plan has raised since it was last read. */
enum {
    RCP_INFO_PINV_FALLBACK = 1,  /* a Gram matrix was singular: pseudo-inverse used (Definition 2) */
    RCP_INFO_NONFINITE = 2,      /* the fit became NaN/Inf */
    RCP_INFO_EIG_NOT_CONVERGED = 4, /* the eigenvector start's Jacobi sweeps did not converge */
    RCP_INFO_QR_HOUSEHOLDER = 8  /* a sketch was numerically rank deficient: its QR
                                    (Algorithm 1's orthonormalisations) fell back to Householder */
};

#define RCP_MAX_NDIM 8     /* tensor order N in [2, 8] */
#define RCP_MAX_L 64       /* k + p <= 64 */
#define RCP_MAX_RANK 64    /* k <= 64 */

/* The problem, as Algorithm 1 and 2 state it: an N-way tensor, target rank
 * k (= CP rank R), oversampling p (Algorithm 1: l = k + p) and q
 * normalised power iterations (Algorithm 1). */
typedef struct rcp_problem {
    int32_t ndim;                    /* N, 2..RCP_MAX_NDIM */
    int32_t k;                       /* target rank = CP rank R, >= 1 */
    int32_t p;                       /* oversampling, >= 0, k + p <= RCP_MAX_L */
    int32_t q;                       /* power iterations, >= 0 */
    int64_t dims[RCP_MAX_NDIM];      /* I_0 .. I_{N-1}, each >= 1 */
    int32_t max_iters;               /* ALS sweeps, >= 1 */
    int32_t precision;               /* RCP_PREC_* */
    int32_t scheme;                  /* RCP_SCHEME_* */
    int32_t solver;                  /* RCP_SOLVER_*: CP solver on the core */
    double tol;                      /* stop when |rho_j - rho_{j-1}| < tol (j >= 2); 0 = run max_iters */
    uint64_t seed;                   /* seed of the random test matrices */
    /* variants of Algorithm 1 (all zero = the defaults above) */
    int32_t test_matrix;             /* RCP_TEST_*: Algorithm 1's test matrix Omega_n */
    uint32_t compress_mask;          /* bit n set: compress mode n; 0 = every mode.  A mode
                                        left out keeps Q_n = I (needs I_n <= 64) */
    int32_t per_mode_p;              /* nonzero: mode_p[n] replaces p for mode n */
    int32_t mode_p[RCP_MAX_NDIM];    /* per-mode oversampling, >= 0, k + mode_p[n] <= 64 */
} rcp_problem;

/* Written on the device by rcp_als / rcp_decompose. */
typedef struct rcp_als_info {
    int32_t iters;                   /* sweeps run */
    int32_t status;                  /* RCP_INFO_* bits */
    double rho;                      /* fit of Section 3.3 after the last sweep */
    double rel_err;                  /* sqrt(max(0, 1 - rho)) = ||X - Xhat|| / ||X|| */
    double normX2;                   /* ||X||_F^2 used for the fit */
} rcp_als_info;

typedef struct rcp_plan_t* rcp_plan;

/* Bytes of device workspace a plan for *prob needs (host only, no GPU call).
 * Returns RCP_ERR_INVALID_ARG for an invalid problem (see rcp_init). */
rcp_status rcp_workspace_size(const rcp_problem* prob, size_t* bytes);

/* Validates *prob, binds the workspace (device pointer, 256-byte aligned,
 * >= rcp_workspace_size bytes) and the HIP stream (hipStream_t passed as
 * void*; NULL = the null stream) and returns a plan in *plan.
 * RCP_ERR_INVALID_ARG: ndim outside [2, 8], a dim < 1, k < 1, p < 0, q < 0,
 *   k + p > 64, k > l_n for some n, max_iters < 1, tol < 0, unknown
 *   precision/scheme/solver, or a null plan / problem pointer.
 * RCP_ERR_WORKSPACE: null or too small workspace.
 * RCP_ERR_UNSUPPORTED: the core factors and Gram matrices of CP-ALS do not
 *   fit one workgroup's LDS (rank and l too large together), or the device
 *   is not gfx950. */
rcp_status rcp_init(rcp_plan* plan, const rcp_problem* prob, void* workspace,
                    size_t workspace_bytes, void* hip_stream);

/* Frees the host-side plan.  Does not touch the workspace. */
rcp_status rcp_destroy(rcp_plan plan);

/* Reads the plan's device status word (RCP_INFO_* bits raised by every call
 * on the plan since rcp_init or the previous read) into *status (host) and
 * clears it.  Blocks: the read is ordered after all work enqueued on the
 * plan's stream.  RCP_ERR_INVALID_ARG for null arguments, RCP_ERR_HIP if the
 * copy fails. */
rcp_status rcp_read_status(rcp_plan plan, int32_t* status);

/* Randomised range finder of one mode (Algorithm 1, up to the final
 * orthonormalisation).
 * T: current tensor with dims cur_dims[0..N-1] (host array); mode n; the
 * sketch width is l = min(k + p, cur_dims[n]).  Writes the orthonormal
 * basis Q (cur_dims[n] x l, row-major, diag(R) > 0 convention) built from
 * Y = T_(n) Omega_n and q normalised power iterations.  Omega_n is the
 * counter-based Gaussian matrix of (seed, mode n, batch 0).
 * cur_dims may differ from the plan's dims (the sequential scheme passes a
 * partly compressed tensor) but no dim may exceed the plan's dims. */
rcp_status rcp_sketch(rcp_plan plan, const float* T, const int64_t* cur_dims,
                      int32_t mode, float* Q);

/* Mode-n projection T_out = T x_n Q^T (Algorithm 1's projection; the n-mode
 * product of Definition 1).  Q is cur_dims[n] x l row-major, l = its
 * width as rcp_sketch defines it; T_out has dims cur_dims with mode n
 * replaced by l.  T and T_out must not overlap. */
rcp_status rcp_compress(rcp_plan plan, const float* T, const int64_t* cur_dims,
                        int32_t mode, const float* Q, float* T_out);

/* ||X||_F^2 in float64 of count float32 values (written to *out, device). */
rcp_status rcp_norm2(rcp_plan plan, const float* X, int64_t count, double* out);

/* CP-ALS on the core (Algorithm 2: initialisation and sweeps).  core: l_0 x ... x l_{N-1}
 * (the plan's sketch widths).  At[n]: l_n x R outputs (row-major); lambda:
 * R outputs; info: device rcp_als_info.  normX2: device pointer to ||X||^2
 * of the uncompressed tensor for the fit (NULL: use ||core||^2).
 * Initialisation: leading R eigenvectors of B_(n) B_(n)^T for modes
 * 1..N-1 (Algorithm 2's initialisation); with use_given_init != 0 the sweeps start
 * instead from the factors the caller left in At[1..N-1] (a warm start, the
 * way to resume an interrupted run: At[0] is computed first and not read).
 * Sweeps: for n = 0..N-1, Ã_n = B_(n)
 * KR(Ã_{m!=n}) (*_{m!=n} Ã_m^T Ã_m)^+, column-normalised, lambda from the
 * last mode (the factor updates of a sweep).  Stops after max_iters sweeps, or earlier when
 * tol > 0 and the fit changes by less than tol (the convergence test).  A core that fits
 * in one workgroup's LDS runs the whole sweep loop in one launch; a larger
 * one runs its mode products over the whole GPU with a one-workgroup solve
 * per mode (every max_iters sweep is enqueued; after the stopping rule fires
 * the remaining launches return at once).  Results agree to rounding. */
rcp_status rcp_als(rcp_plan plan, const float* core, float* const* At,
                   float* lambda, const double* normX2, rcp_als_info* info,
                   int32_t use_given_init);

/* Block coordinate descent on the core (Algorithm 3: initialisation and rank-one sweeps; arguments
 * as rcp_als).  Components r = 0..R-1 one after another: each sweep updates
 * a_r^(0..N-1) in mode order, each the least-squares rank-one block update on
 * the residual B - sum_{s<r} lam_s a_s^(0) o ... o a_s^(N-1) (evaluated
 * without forming it), unit-normalised with the last mode's norm as
 * lambda_r; max_iters sweeps per component, fewer when tol > 0 and the fit
 * of components 0..r changes by less than tol (after sweep 2).
 * info->iters is the sum of the components' sweeps.  Starts from the leading
 * eigenvectors of B_(n) B_(n)^T (column r for component r) or, with
 * use_given_init != 0, from At[1..N-1].  RCP_ERR_UNSUPPORTED when a core
 * mode exceeds 64 or the float64 factors do not fit one workgroup's LDS. */
rcp_status rcp_bcd(rcp_plan plan, const float* core, float* const* At,
                   float* lambda, const double* normX2, rcp_als_info* info,
                   int32_t use_given_init);

/* Deterministic CP-ALS on the full tensor X (Section 3.3: Algorithm 2 with
 * Q_n = I, the Tensor Toolbox's scheme the paper follows), for a plan whose
 * solver is RCP_SOLVER_CP_ALS (else RCP_ERR_INVALID_ARG).  X: the plan's
 * dims, C-order float32; outputs A[n] (I_n x R), lambda (R) and info as for
 * rcp_decompose (ordered by lambda, signs fixed, fit exact on X).
 * Start (A_init == NULL): for modes 1..N-1 the leading R eigenvectors of
 * X_(n) X_(n)^T (Algorithm 2's initialisation), computed by subspace iteration: the
 * plan's q power steps of Algorithm 1 on an l_n = min(k + p, I_n) wide block
 * (the plan's test matrix and seed), then the eigenvectors of the l_n x l_n
 * Gram Q^T X_(n) X_(n)^T Q (Rayleigh-Ritz); equal to the exact ones up to
 * (sigma_{l_n + 1} / sigma_R)^(2q + 1), so q sets the accuracy.  Each column
 * is unit and signed as the oracle's eigenvectors (largest-magnitude entry
 * positive).  With A_init (host array of N device pointers, I_n x R float32;
 * A_init[0] is not read) the sweeps start from the caller's factors.
 * Sweeps: per mode the product X_(n) KR(A_{m != n}) streams X once over the
 * whole GPU, then one solve with V = *_{m != n} A_m^T A_m (pseudo-inverse
 * fallback as rcp_als), unit columns, lambda from the last mode; stops after
 * max_iters sweeps or, with tol > 0, when the fit changes by less than tol. */
rcp_status rcp_cp_als(rcp_plan plan, const float* X, const float* const* A_init,
                      float* const* A, float* lambda, rcp_als_info* info);

/* Back-projection A_n = Q_n Ã_n (eq. qbs, Algorithm 2's factor recovery) and the
 * final renormalisation: unit columns, norms folded into lambda,
 * components sorted by lambda (descending), the largest-magnitude entry of
 * each column of modes 0..N-2 made positive with the sign moved to mode
 * N-1.  Q[n]: I_n x l_n, At[n]: l_n x R, lambda_in: R; outputs A[n]:
 * I_n x R and lambda_out: R (may equal lambda_in). */
rcp_status rcp_expand(rcp_plan plan, const float* const* Q, const float* const* At,
                      const float* lambda_in, float* const* A, float* lambda_out);

/* The whole path on X (dims = the plan's dims): ||X||^2, the compression of
 * Algorithm 1 (scheme from the plan), CP-ALS on the core and the
 * back-projection.  Outputs A[n] (I_n x R), lambda (R) and info (device).
 * The bases and the core stay in the workspace (rcp_get_bases / rcp_get_core).
 * A plan with solver RCP_SOLVER_CP_ALS runs rcp_cp_als(plan, X, NULL, ...)
 * instead (no bases or core: rcp_get_bases / rcp_get_core then return
 * RCP_ERR_UNSUPPORTED). */
rcp_status rcp_decompose(rcp_plan plan, const float* X, float* const* A,
                         float* lambda, rcp_als_info* info);

/* For callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): rcp_decompose without a plan or workspace.  Same arguments
 * and results as rcp_init + rcp_decompose + rcp_destroy (prob as for
 * rcp_init, X and the outputs as for rcp_decompose, hip_stream as for
 * rcp_init); the workspace is a device array inside the library of
 * RCP_NOALLOC_SCRATCH_BYTES, one per GPU, held until the process ends, found
 * on the first call on each device.  The call allocates nothing and enqueues
 * only kernels (no memset or copy nodes).  RCP_ERR_WORKSPACE when the
 * problem's rcp_workspace_size exceeds RCP_NOALLOC_SCRATCH_BYTES (e.g.
 * 256^3 with k + p = 26 fits; 400^3 with k + p = 30 does not);
 * RCP_ERR_INVALID_ARG / RCP_ERR_UNSUPPORTED as rcp_init / rcp_decompose.
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents: calls that overlap on one GPU (different streams or
 * threads without ordering between them) race and give undefined results.
 * The status bits that rcp_read_status would report are not readable for
 * this entry point; CP-ALS outcomes still land in info->status. */
#define RCP_NOALLOC_SCRATCH_BYTES (32u << 20)
rcp_status rcp_decompose_noalloc(const rcp_problem* prob, const float* X, float* const* A,
                                 float* lambda, rcp_als_info* info, void* hip_stream);

/* Device pointers, inside the workspace, of the bases Q_n (I_n x l_n) and of
 * the core (l_0 x ... x l_{N-1}) that the last rcp_decompose produced.
 * Q: host array of N pointers to fill.  core_dims: host array of N (may be NULL). */
rcp_status rcp_get_bases(rcp_plan plan, float** Q);
rcp_status rcp_get_core(rcp_plan plan, float** core, int64_t* core_dims);

/* Rows [row0, row0 + nrows) of the test matrix Omega of a mode, width
 * l <= 64 (nrows x l row-major, device), of the plan's kind (GAUSSIAN,
 * UNIFORM or HALTON as rcp_problem.test_matrix describes, batch 0; for
 * COLUMNS see rcp_debug_columns). */
rcp_status rcp_debug_omega(rcp_plan plan, int32_t mode, int64_t row0, int64_t nrows,
                           int32_t l, float* omega);

/* The raw Philox4x32-10 output behind the same rows: for row j = row0 + r
 * and column group g < ngroups (columns 4g..4g+3), words[(r * ngroups + g) * 4
 * + i] (device, uint32) is word i of the generator applied to the counter
 * (j mod 2^32, j >> 32, g, mode) under the key (seed mod 2^32, seed >> 32).
 * ngroups in [1, 16]. */
rcp_status rcp_debug_philox(rcp_plan plan, int32_t mode, int64_t row0, int64_t nrows,
                            int32_t ngroups, uint32_t* words);

/* The l column indices (device int64, sorted ascending) that the COLUMNS
 * test matrix selects out of J for a mode (seed of the plan, batch 0).
 * RCP_ERR_INVALID_ARG unless 1 <= l <= min(J, 64). */
rcp_status rcp_debug_columns(rcp_plan plan, int32_t mode, int64_t J, int32_t l, int64_t* idx);

/* Per-kernel timing of a plan's launches (for roofline reporting).
 * rcp_profile(plan, 1) starts recording a HIP event pair around every kernel
 * launch the plan makes (at most 4096 launches are recorded; later ones are
 * counted but not timed), with the algorithmic bytes moved and flops done by
 * each launch, computed on the host from its shapes: for the streaming
 * kernels, every element of the current tensor read once (4 B), the outputs
 * written once, and 2 flops per multiply-add of the contraction.
 * rcp_profile(plan, 0) stops recording and clears the totals.
 * rcp_profile_read waits for the recorded events (host blocking) and returns
 * the totals of one kernel class (RCP_KERNEL_*): launches, milliseconds,
 * bytes and flops.  Any pointer may be NULL. */
enum {
    RCP_KERNEL_SKETCH = 0,       /* Y = T_(n) Omega, Omega generated in-kernel */
    RCP_KERNEL_POWER = 1,        /* Y = T_(n) (T_(n)^T Q), fused single pass */
    RCP_KERNEL_CONTRACT_IN = 2,  /* T x_n Q^T (compression, or stored Z) */
    RCP_KERNEL_CONTRACT_OUT = 3, /* Y = T_(n) Z with a stored Z */
    RCP_KERNEL_REDUCE = 4,       /* partial-sum reduction */
    RCP_KERNEL_QR = 5,           /* QR of a sketch (shifted Cholesky QR, Householder fallback) */
    RCP_KERNEL_ALS = 6,          /* CP-ALS on the core */
    RCP_KERNEL_EXPAND = 7,       /* back-projection and renormalisation */
    RCP_KERNEL_OTHER = 8,
    RCP_KERNEL_BCD = 9,          /* block coordinate descent on the core */
    RCP_KERNEL_MTTKRP = 10,      /* X_(n) KR(A_{m != n}) over the full tensor (rcp_cp_als) */
    RCP_KERNEL_CP_UPDATE = 11,   /* rcp_cp_als: solve, norms, Grams, fit of one mode */
    RCP_KERNEL_COUNT = 12
};
rcp_status rcp_profile(rcp_plan plan, int32_t enable);
rcp_status rcp_profile_read(rcp_plan plan, int32_t kernel_class, int64_t* launches, double* ms,
                            double* bytes, double* flops);

/* ------------------------------------------------------------------------
 * Batches of independent problems.  Algorithms 1 and 2 applied to `count`
 * unrelated tensors (uneven shapes, ranks and seeds) as one unit of work:
 * the compression passes of the problems are spread over a few internal
 * streams forked from and joined back into the batch stream (so small
 * problems' kernels run side by side), then one launch runs CP-ALS for all
 * of them (one workgroup per problem) and one launch the back-projection.
 * The paper treats one tensor at a time; this is the throughput form for
 * many small ones.  Each problem gives exactly the result rcp_decompose
 * gives it alone.
 *
 * rcp_batch_workspace_size: bytes of device workspace for probs[0..count).
 *   RCP_ERR_INVALID_ARG / RCP_ERR_UNSUPPORTED as rcp_init for any problem.
 * rcp_batch_init: binds the workspace (device, 256-byte aligned, at least
 *   rcp_batch_workspace_size bytes) and the stream (hipStream_t as void*,
 *   NULL = the null stream); RCP_ERR_WORKSPACE / RCP_ERR_INVALID_ARG as
 *   rcp_init.
 * rcp_batch_decompose: X[i] (host array of count device pointers to the
 *   C-order float32 tensors), outputs A[i][n] (device, I_n x k_i float32,
 *   row-major; A and A[i] are host arrays), lambda[i] (device, k_i float32)
 *   and info (device array of count rcp_als_info).  The output pointers go
 *   into device argument tables: when they differ from the previous call's,
 *   the call first waits for the batch stream to drain and uploads new
 *   tables in stream order (host blocking only then).  On a non-null stream
 *   the first call records the whole sequence in a HIP graph and launches
 *   it; later calls with the same X pointers relaunch the graph (other X
 *   pointers re-record it).  On the null stream the kernels are enqueued
 *   directly.  Asynchronous otherwise, like every other call; numeric
 *   outcomes land in info[i].  RCP_ERR_INVALID_ARG: a null or misaligned
 *   pointer.  When every problem uses the sequential scheme, compresses
 *   every mode with a generated test matrix and has modes that fit the fused
 *   power kernel and the LDS QR (at most 512 rows), the range finder runs in
 *   phase order: each step (sketch, reduction, QR, power step, mode product)
 *   is one launch over all problems (descriptor tables in the workspace,
 *   rebuilt when X or the launch shape changes); otherwise each problem's
 *   chain runs on the internal streams.  Either way every problem gets the
 *   arithmetic of its single-problem rcp_decompose, bit for bit.
 * rcp_batch_read_status: the status word (rcp_read_status) of problem index.
 * rcp_batch_get_core: rcp_get_core of problem index (the core B of its last
 *   decomposition, l_0 x ... x l_{N-1}, inside the batch workspace; valid
 *   until the next rcp_batch_decompose).
 * rcp_batch_destroy: waits for the batch stream, frees the host-side state
 *   (the graph included). */
typedef struct rcp_batch_t* rcp_batch;
rcp_status rcp_batch_workspace_size(const rcp_problem* probs, int32_t count, size_t* bytes);
rcp_status rcp_batch_init(rcp_batch* batch, const rcp_problem* probs, int32_t count,
                          void* workspace, size_t workspace_bytes, void* hip_stream);
rcp_status rcp_batch_decompose(rcp_batch batch, const float* const* X, float* const* const* A,
                               float* const* lambda, rcp_als_info* info);
rcp_status rcp_batch_read_status(rcp_batch batch, int32_t index, int32_t* status);
rcp_status rcp_batch_get_core(rcp_batch batch, int32_t index, float** core, int64_t* core_dims);
/* Autotuner of the batched launch shape (no counterpart in the paper, which
 * has no batched form).  Times complete batch decompositions of the given
 * inputs into the given outputs (so it also leaves their results there) for
 * candidate shapes, searching one knob at a time with the others at their
 * best so far:
 *   shape[0] internal streams the compressions are spread over: 4, 8, 16
 *            (not searched when every problem takes the grouped form, which
 *            runs each step as one launch over all problems on the batch
 *            stream);
 *   shape[1] workgroups per streaming pass (at most one per tile): 16, 32,
 *            64, 128, one per compute unit;
 *   shape[2] rows per row block of the sketch passes of modes with at most
 *            512 rows, in units of 64: 1, 2, 4, 8.
 * Each candidate is recorded once and timed over two replays with HIP events
 * on the batch stream; it replaces the best so far only if at least 3%
 * faster (the timing noise).  The chosen shape is kept for later calls of this
 * batch (the graph is recorded again on the next call) and written to the
 * host array shape[3]; *best_ms (host) receives its time per call.  Blocks
 * until the timing is done.  Errors: RCP_ERR_INVALID_ARG as
 * rcp_batch_decompose, RCP_ERR_HIP for a failed launch or event call. */
rcp_status rcp_batch_autotune(rcp_batch batch, const float* const* X, float* const* const* A,
                              float* const* lambda, rcp_als_info* info, int32_t* shape,
                              double* best_ms);
rcp_status rcp_batch_destroy(rcp_batch batch);

/* Static description of a status code; any other int value gives
 * "unknown rcp_status". */
const char* rcp_status_string(rcp_status status);

/* Library version string. */
const char* rcp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RCP_H_ */
