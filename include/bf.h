/*
 * bf.h -- C ABI of an MI355X (gfx950) interpolative butterfly apply for the
 * oscillatory matvec g = K f, K(x, xi) = alpha(x, xi) exp(2 pi i Phi(x, xi)).
 *
 * Method: H. Yang, "A Unified Framework for Oscillatory Integral Transforms:
 * When to use NUFFT or Butterfly Factorization?" (arXiv:1803.04128).
 *   - problem statement: Section 4 (potential g(x) = sum_xi K(x, xi) f(xi))
 *     and Section 5, eq. (eqn:1D-FIO) with the grid of eq. (eqn:1D-xandxi);
 *   - amplitude split: eq. (eqn:tg), g = sum_k a_k * BF(b_k * f);
 *   - factors: Algorithm 2 (interpolative low-rank approximation, Section
 *     2.1) on the dyadic trees of Section 4;
 *   - apply: the butterfly algorithm of Section 4 (Algorithm 4.1), with the
 *     precomputed factors kept for many input vectors (Section 1 footnote
 *     on reusing precomputation; Section 4 closing paragraph).
 *
 * Grid (per dimension, 0-based): x_i = i / n, xi_j = j - n/2, n a power of
 * two.  dim = 1: N = n.  dim = 2: N = n * n and a point is addressed by its
 * row-major index i1 * n + i2 (the tree order is internal).
 *
 * Complex data is interleaved single precision (re, im) on the device, and
 * interleaved double precision on the host where stated.
 *
 * Errors: every call returns BF_OK (0) or a negative status; the message of
 * the last failure on the calling thread is returned by bf_last_error().
 * No C++ exception crosses this interface.  Kernel faults surface at the
 * caller's next synchronisation of the stream.
 */
#ifndef BF_H
#define BF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define BF_OK            0
#define BF_EINVAL       -1   /* bad argument (shape, null pointer, aliasing) */
#define BF_ENOMEM       -2   /* device or host allocation failed, or the
                                request exceeds the configured memory cap */
#define BF_EHIP         -3   /* a HIP runtime call failed */
#define BF_EUNSUPPORTED -4   /* valid request this build does not implement */
#define BF_EBUSY        -5   /* resource in use */

/* ---- phase functions (evaluated in FP64 on the device) ------------------ */
/* BF_PHASE_DFT:       Phi = x . xi                                 (no params)
 * BF_PHASE_FIO1D:     Phi = x xi + c(x)|xi|, c(x) = (p0 + p1 sin 2 pi x)/p2
 *                     (Section 5, eq. (eqn:1D-FIO-kernal) with general c)
 * BF_PHASE_FIO1D_WARP: Phi = x xi + c(x) xi with the same c(x) (1D): the
 *                     FIO of the composition example, eq. (eqn:FIOK2); it
 *                     evaluates the Fourier series of its input at
 *                     x + c(x).
 * BF_PHASE_LOWRANK:   Phi(x_i, xi_j) = sum_{k<rank} U[i][k] V[j][k], the
 *                     phase given by real low-rank factors (the input form
 *                     of Algorithm 2), any dim; U and V come in bf_phase.
 * BF_PHASE_RADON2D:   Phi = x . xi + sqrt(c1(x)^2 xi1^2 + c2(x)^2 xi2^2),
 *                     c1 = (p0 + p1 sin 2 pi x1 sin 2 pi x2) / p2,
 *                     c2 = (p3 + p4 cos 2 pi x1 cos 2 pi x2) / p5
 * BF_PHASE_SEPARABLE: Phi = p0 sin(2 pi x1)(1 + x2) + p1 |xi| + p2 |xi|^2/n
 *                     (x2 = 0 in 1D; |xi| Euclidean), additively separable,
 *                     for which the factorization is exact (R = 0 in
 *                     eq. (eqn:RAB)).                                      */
#define BF_PHASE_DFT        0
#define BF_PHASE_FIO1D      1
#define BF_PHASE_RADON2D    2
#define BF_PHASE_SEPARABLE  3
#define BF_PHASE_FIO1D_WARP 4
#define BF_PHASE_LOWRANK    5

/* ---- arithmetic of the apply ------------------------------------------- */
/* BF_FP32:   FP32 complex state and factors, FP32 vector arithmetic.
 * BF_BF16X3: Lagrange matrices and the panel are split x = hi + lo in
 *            bfloat16; the shared-matrix contraction runs on MFMA as
 *            hi*hi + hi*lo + lo*hi with FP32 accumulation; twiddles,
 *            switch blocks and the state stay FP32.
 * BF_FP16X3: as BF_BF16X3 with IEEE half hi/lo parts; each panel column
 *            of a product is scaled by a power of two (exact) so that its
 *            largest magnitude maps into [0.5, 1) before the split.        */
#define BF_FP32    0
#define BF_BF16X3  1
#define BF_FP16X3  2

typedef struct bf_grid {
    int dim;   /* 1 or 2 */
    int n;     /* points per dimension, a power of two, 2 <= n;
                  1D: n <= 2^22, 2D: n <= 2^11 */
} bf_grid;

typedef struct bf_phase {
    int kind;              /* BF_PHASE_* */
    int nparams;           /* number of entries in params (0, 3 or 6) */
    const double* params;  /* host, read during bf_plan only */
    /* BF_PHASE_LOWRANK only (nparams = 0): 1 <= rank <= 64 and the factors,
     * host float64 [N][rank] row-major in user index order (row i of U
     * belongs to x_i, row j of V to xi_j); copied to the device by bf_plan
     * (2 N rank doubles, freed by bf_destroy) and read during applies only
     * by the on-the-fly switch form.  The FP64 sum carries an error of
     * about |Phi| 2^-52 cycles, so FP32-level results need |Phi| below
     * about 2^25 (the built-in kinds reduce their bilinear part exactly). */
    int rank;
    const double* U;
    const double* V;
} bf_phase;

/* Low-rank amplitude alpha(x, xi) = sum_{k<r} a_k(x) b_k(xi) (eq. (eqn:tg)).
 * a, b: host complex128 interleaved, layout [r][N] in user index order; read
 * during bf_plan only.  r = 1 with a = b = NULL means alpha = 1.            */
typedef struct bf_amplitude {
    int r;             /* 1 <= r <= 16 */
    const double* a;
    const double* b;
} bf_amplitude;

typedef struct bf_plan_s* bf_plan_t;

/* Plan and factor construction (synchronous).
 *
 * Builds the dyadic trees (Section 4), the interpolation points of every box
 * (eqs. (eqn:gdA)/(eqn:gdB), read with the ascending Chebyshev node), the
 * box centers, the Lagrange matrices (Section 2.1), and on the device in
 * FP64 the twiddles and switch blocks of Algorithm 4.1 (eqs. (eqn:1),
 * (eqn:2), the switch step and eq. (eqn:3), regrouped into unit-modulus
 * diagonals times one shared real matrix per level and child).  All factor
 * memory stays on the current device until bf_destroy.
 *
 * q: interpolation points per box and dimension, 2 <= q <= 16 (1D) or
 *    2 <= q <= 8 (2D).
 * precision: BF_FP32, BF_BF16X3 or BF_FP16X3.
 * max_nvec: the largest nvec bf_apply will be called with (>= 1); the
 *    default workspace is sized for it (in vector chunks when large).
 * out: receives the plan handle.
 * Returns BF_EINVAL on bad arguments, BF_ENOMEM when device memory (or the
 * cap set by the environment variable BF_MEM_CAP_BYTES) does not suffice.  */
int bf_plan(const bf_grid* grid, const bf_phase* phase,
            const bf_amplitude* amp, int q, int precision, int max_nvec,
            bf_plan_t* out);

/* ---- transposed and conjugate operators ---------------------------------
 * Scenario 2 of Section 1 (iterative solvers and preconditioners built on
 * K) needs K^T and K^H besides K.  K^T(xi_j, x_i) = alpha(x_i, xi_j)
 * exp(2 pi i Phi(x_i, xi_j)) maps vectors on the x grid to vectors on the
 * xi grid; it has the form of eq. (eqn:FIO) with x and xi exchanged, so
 * Algorithm 4.1 factorizes it with the same trees, points and Lagrange
 * matrices, the phase evaluated with its arguments exchanged (and negated
 * for the conjugates), and the amplitude factors swapped: b_k weights the
 * output and a_k the input (conjugated for the conjugates).  The error is
 * of the same order as for K (Section 3 bounds the ranks in both
 * variables).  Index order of both grids is the user order of bf_grid.   */
#define BF_OP_N  0   /* K                         */
#define BF_OP_T  1   /* K^T                       */
#define BF_OP_C  2   /* conj(K), entrywise        */
#define BF_OP_H  3   /* K^H = conj(K)^T           */

/* As bf_plan, for the operator op (BF_OP_*); bf_apply then computes
 * g[v] = op(K) f[v].  bf_plan(...) equals bf_plan_op(..., BF_OP_N, ...).
 * The amplitude pointers keep their meaning (a_k on x, b_k on xi).
 * Returns BF_EINVAL for an unknown op, otherwise as bf_plan.             */
int bf_plan_op(const bf_grid* grid, const bf_phase* phase,
               const bf_amplitude* amp, int q, int precision, int max_nvec,
               int op, bf_plan_t* out);

/* Device bytes bf_plan_op with the same arguments would allocate: the
 * factor arena (twiddles, Lagrange matrices, amplitude factors), the stored
 * switch blocks when the initial execution form reads them, the low-rank
 * phase factors and the default workspace.  Host only: no device is
 * touched, so a caller that admits plans under a memory budget can decide
 * before anything is allocated.  Returns the status bf_plan_op would return
 * for the arguments' checks (BF_EINVAL, BF_EUNSUPPORTED, BF_ENOMEM for the
 * BF_MEM_CAP_BYTES cap); *bytes is 0 on failure.                         */
int bf_plan_footprint(const bf_grid* grid, const bf_phase* phase,
                      const bf_amplitude* amp, int q, int precision,
                      int max_nvec, int op, size_t* bytes);

/* Apply: g[v] = sum_k a_k * BF(b_k * f[v]) for v < nvec (eq. (eqn:tg) with
 * Algorithm 4.1).
 * f, g: device complex64 interleaved, layout [nvec][N], contiguous, owned
 *    by the caller; g must not overlap f.
 * stream: a hipStream_t (NULL = the null stream).  The call is asynchronous
 *    on that stream and allocates nothing; it uses the plan's workspace, so
 *    applies of one plan must not overlap (use bf_apply_ws for that).
 * Returns BF_EINVAL for nvec < 1, nvec > max_nvec, null or overlapping
 * pointers.                                                               */
int bf_apply(bf_plan_t plan, int nvec, const void* f, void* g, void* stream);

/* Allocation-free apply, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): as bf_apply, with the workspace taken from a static device
 * buffer of BF_STATIC_SCRATCH_BYTES that the library holds on every GPU it
 * runs on until the process ends (its address is recorded once per device
 * when the first plan is built there).  The call allocates nothing; vectors
 * are processed in chunks that fit the buffer.  All calls on one GPU share
 * the buffer and leave their intermediate state in it: calls that overlap
 * in time on one GPU (other streams, other threads or plans) race and must
 * be serialized by the caller.  Returns BF_EINVAL when one vector's
 * workspace (bf_workspace_bytes(plan, 1)) exceeds the buffer, otherwise as
 * bf_apply.                                                               */
#define BF_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
int bf_apply_static(bf_plan_t plan, int nvec, const void* f, void* g,
                    void* stream);

/* Chained applies: g = P_{count-1}( ... P_1(P_0 f)) for the plans
 * plans[0 .. count-1] (the same plan may appear more than once), e.g. the
 * composition of two FIOs of eq. (eq:example4): the FIO, then the Fourier
 * coefficients of its output (a BF_OP_H plan of the DFT phase with the
 * constant amplitude 1/N), then the FIO again.  Every plan must have the
 * same N, live on the current device and accept nvec vectors.
 * f, g: device complex64 [nvec][N], g must not overlap f.
 * tmp: device complex64 [nvec][N] owned by the caller, the intermediate
 *    results ping-pong between tmp and g (f is only read); may be NULL for
 *    count == 1, must not overlap f or g.
 * Asynchronous on stream like bf_apply, and each apply uses its plan's
 * own workspace, so chains that share a plan must not overlap in time.
 * Returns BF_EINVAL (checked before anything is launched) for count < 1,
 * an invalid plan, mismatched N, nvec out of a plan's range, or null or
 * overlapping buffers.                                                   */
int bf_apply_chain(const bf_plan_t* plans, int count, int nvec,
                   const void* f, void* g, void* tmp, void* stream);

/* Workspace bytes bf_apply_ws needs for nvec vectors. */
int bf_workspace_bytes(bf_plan_t plan, int nvec, size_t* bytes);

/* As bf_apply with a caller-owned device workspace of ws_bytes bytes
 * (>= bf_workspace_bytes(plan, nvec)); applies of one plan with distinct
 * workspaces may run concurrently on different streams.                   */
int bf_apply_ws(bf_plan_t plan, int nvec, const void* f, void* g, void* ws,
                size_t ws_bytes, void* stream);

/* Releases every device allocation of the plan after synchronising the
 * device work the plan issued.  NULL is accepted.                         */
int bf_destroy(bf_plan_t plan);

typedef struct bf_plan_info {
    int dim, n, L, h, q, r, precision;
    long long N;
    int first_xi_level;    /* first level with an interpolating xi step   */
    int last_x_level;      /* last level with an interpolating x step     */
    int n_steps;           /* computed steps: xi levels + switch + x levels */
    int n_passes;          /* kernel passes per vector chunk              */
    int max_rank;          /* largest number of coefficients per pair     */
    int chunk_nvec;        /* vectors per workspace chunk                 */
    size_t factor_bytes;   /* device bytes of twiddles, blocks, matrices  */
    size_t workspace_bytes;/* default workspace (for chunk_nvec vectors)  */
    double flops_per_column;  /* algorithmic flops per apply column       */
    double factor_stream_bytes; /* factor bytes read per apply            */
    int op;                /* BF_OP_* the plan applies                    */
    int method;            /* 0 butterfly (Section 4), 1 NUFFT by
                              dimension lifting (Section 3)              */
} bf_plan_info;

int bf_query(bf_plan_t plan, bf_plan_info* info);

/* ---- NUFFT by dimension lifting (Section 3) ------------------------------
 * For a kernel whose phase and amplitude are given by real low-rank factors
 * on an N x N grid (1D x and xi), Phi(x_i, xi_j) ~ sum_c U1[i][c] V1[j][c]
 * (rank r1) and alpha(x_i, xi_j) ~ sum_c U2[i][c] V2[j][c] (rank r2), the
 * framework applies K either by the butterfly (bf_plan with
 * BF_PHASE_LOWRANK) or, when the phase minus its leading rank-r part leaves
 * a kernel of small numerical rank, as r_eps r-dimensional type-3 NUFFTs
 * (eq. (eqn:tg3)):
 *   g(x_i) ~ sum_k a_k(x_i) sum_j exp(2 pi i P_i . Q_j) b_k(xi_j) f(xi_j).
 *
 * bf_lift_decide: Algorithm 6 (host, FP64, synchronous, no device use).
 *   1. P Q^T = the rank-r truncated SVD of U1 V1^T (P scaled by the
 *      singular values), by a randomized range finder with the caller's
 *      test matrix omega [N][omega_cols], r1 < omega_cols <= 64;
 *   2. the residual Kres = (U2 V2^T) . exp(2 pi i (U1 V1^T - P Q^T)) at the
 *      columns test_cols[0 .. n_test) (the method's random sample, r_eps q
 *      of them for an oversampling q), and its numerical rank n: the
 *      diagonal entries of R in its pivoted QR above |R(1,1)| eps;
 *   3. y = 1 when n <= r_eps (the printed test compares n with r and
 *      samples r q columns; it is read with r_eps, the rank of the sum in
 *      eq. (eqn:tg3), since r = 1 could otherwise never pass), and then
 *   4. Algorithm 1 factors Kres ~ sum_k a_k b_k^T with rank k <= r_eps:
 *      `rounds` rounds of sampled rows rows_s[round][per_round] and columns
 *      cols_s[round][per_round] (the important columns: pivots of a
 *      pivoted QR of Kres(I, :); the important rows: pivots of a pivoted
 *      LQ of Kres(:, J)), orthonormal bases from them, and the core matrix
 *      on the important plus the extra rows and columns extra_rows,
 *      extra_cols [n_extra].
 * Inputs: U1, V1 [N][r1], U2, V2 [N][r2] real row-major host arrays; 1 <= r
 * < r1, r <= 2; 1 <= r_eps <= 64; indices in [0, N).
 * Outputs: *y, *n_rank; P, Q [N][r] (always); a, b host complex128
 * interleaved [r_eps][N] of which the first *k_out rows are set when y = 1.
 * Returns BF_EINVAL for bad arguments or a phase of numerical rank below r.
 */
int bf_lift_decide(long long N, int r1, const double* U1, const double* V1,
                   int r2, const double* U2, const double* V2, int r,
                   int r_eps, double eps, const double* omega, int omega_cols,
                   const long long* test_cols, int n_test, int rounds,
                   const long long* rows_s, const long long* cols_s,
                   int per_round, const long long* extra_rows,
                   const long long* extra_cols, int n_extra, int* y,
                   int* n_rank, double* P, double* Q, double* a, double* b,
                   int* k_out);

/* bf_plan_lifted: a plan that applies eq. (eqn:tg3) on the current device:
 * g_v(x_i) = sum_{c<k} a_c(x_i) sum_j exp(2 pi i P_i . Q_j) b_c(xi_j)
 * f_v(xi_j), each term an r-dimensional type-3 NUFFT from the sources Q_j
 * to the targets P_i (Gaussian gridding of the shifted sources onto a grid
 * at twice the targets' Nyquist rate, a power-of-two FFT with the positive
 * exponent on a twice-oversampled grid, Gaussian interpolation at the
 * targets; about 1e-7 relative before FP32 rounding).  P, Q: host float64
 * [N][r] (r = 1 or 2); a, b: host complex128 interleaved [k][N] (1 <= k <=
 * 64); copied to the device.  The plan is used with bf_apply, bf_apply_ws,
 * bf_apply_static, bf_apply_chain, the graph calls, bf_query (method = 1)
 * and bf_destroy; it has one execution form (bf_set_config and
 * bf_autotune return BF_EUNSUPPORTED) and no butterfly steps.  The
 * workspace holds k FFT grids per vector chunk.  Returns BF_EINVAL for bad
 * arguments, BF_EUNSUPPORTED when the grid the points need exceeds 2^24
 * points (4096 per dimension for r = 2): the space-bandwidth product of the
 * lifted phase is too large for this path, BF_ENOMEM when memory does not
 * suffice.                                                               */
int bf_plan_lifted(long long N, int r, const double* P, const double* Q,
                   int k, const double* a, const double* b, int max_nvec,
                   bf_plan_t* out);

/* ---- stored factors (diagnostics) ----------------------------------------
 * The computed steps of a plan in apply order (bf_plan_info.n_steps of
 * them): the xi levels, the switch, the x levels of Algorithm 4.1.  Each
 * stored factor entry is exp(2 pi i [Phi(x_0, xi_0) - Phi(x_1, xi_1) -
 * Phi(x_2, xi_2)]), rounded to complex64, over its phase terms (one to
 * three), Phi the phase of the plan's operator (its arguments exchanged for
 * BF_OP_T, negated for BF_OP_C).  Layouts, 0-based, R = 2^dim, pairs and
 * boxes numbered as in Section 4 (2D box coordinates interleaved into
 * Morton order, first coordinate on the odd bits):
 *   xi step at level l: twiddles [u][i][c][s], u = a' R^(L-l) + b with a'
 *     at level l-1 of the x tree, b at level L-l of the xi tree; the entry
 *     W_{A,C}[s] (eq. (eqn:2) regrouped) for A = R a' + i, C = R b + c:
 *     terms (c_A, xi_s^C) and, unless the step reads f, (c_P, xi_s^C);
 *   switch at level h: blocks [p][t][s], p = a R^(L-h) + b:
 *     S_{AB}[t][s] with terms (x_t^A, xi_s^B), then (c_A, xi_s^B) unless
 *     the switch reads f, then (x_t^A, c_B) unless no x step follows;
 *   x step at level l: twiddles [u][i][c][t] (u as above): T_{A,C}[t]
 *     (eq. (eqn:3) regrouped), A = R a' + i, B = b, C = R b + c: terms
 *     (x_t^A, c_C) and, unless the step writes lambda, (x_t^A, c_B).
 * Points are the interpolation points of eqs. (eqn:gdA)/(eqn:gdB) (as
 * bf_points gives them), centers the lower-middle index of a box.        */
typedef struct bf_step_info {
    int kind;             /* 0 xi level, 1 switch, 2 x level              */
    int level;            /* tree level l of the step                     */
    int r_in, r_out;      /* coefficients per input / output pair          */
    int reads_f;          /* the step reads f (exact copy levels below)    */
    int writes_lambda;    /* the step emits lambda (exact sums above)     */
    int side_in, side_out;/* box side (per dimension) of the input-side
                             and output-side point sets                   */
    long long units;      /* units (xi, x) or pairs (switch)              */
    long long tw_entries; /* stored twiddle entries (0: none)             */
    long long S_entries;  /* stored switch block entries (0: none)        */
} bf_step_info;

int bf_step_query(bf_plan_t plan, int step, bf_step_info* info);

/* Reads count stored entries of a step: which = 0 twiddles, 1 switch
 * blocks; idx: host entry indices in the layout above.  Writes, per entry
 * k, host arrays x[3 k + j], xi[3 k + j] (user indices of term j's x and xi
 * arguments, -1 past the entry's terms) and values[2 k], values[2 k + 1]
 * (the stored real and imaginary parts).  Synchronous; allocates a small
 * device buffer.  For tests of the factor construction against an FP64
 * evaluation of the same terms.  Returns BF_EINVAL for a bad step, an index
 * out of range or factors the plan does not store.                       */
int bf_factor_entries(bf_plan_t plan, int step, int which,
                      const long long* idx, int count, long long* x,
                      long long* xi, float* values);

/* ---- execution form ------------------------------------------------------
 * How an apply is issued; every form computes the same Algorithm 4.1 and
 * agrees to FP32 rounding (the split precisions exist on BF_PATH_FUSED only).
 * BF_PATH_FUSED:      level-fused passes, one kernel per group of levels:
 *                     the state of a radix-2^k group of pairs stays in LDS
 *                     across k levels (and the switch), so HBM sees it once
 *                     per pass; 1D plans with r in {1, 2, 4, 8} contract on
 *                     MFMA, the others on the vector ALU.
 * BF_PATH_FUSED_VALU: the same passes on the vector ALU only.
 * BF_PATH_PER_STEP:   one kernel per computed level (state through HBM),
 *                     vector ALU.
 * BF_PATH_PER_STEP_MFMA: one kernel per computed level with the level's
 *                     shared-matrix and switch contractions on MFMA (ranks
 *                     up to 64: the 2D form); optionally with the switch
 *                     blocks generated during the apply (switch_otf), which
 *                     trades the N r^2 complex factor stream and its
 *                     storage for one FP64 phase evaluation and one FP32
 *                     sincospi per block entry.
 * The initial form is BF_PATH_FUSED (1D) or BF_PATH_PER_STEP_MFMA (2D) with
 * the default tile width; the environment variables BF_FUSED=0|1, BF_MFMA=0
 * and BF_TILE_COLS=<w>, read when the plan is built, override it.  A plan
 * whose fused passes do not fit starts with one launch per step.           */
#define BF_PATH_FUSED          0
#define BF_PATH_FUSED_VALU     1
#define BF_PATH_PER_STEP       2
#define BF_PATH_PER_STEP_MFMA  3

typedef struct bf_config {
    int path;            /* BF_PATH_* */
    int tile_cols;       /* columns per fused tile: 0 = default (about 8),
                            else a multiple of r, <= 64; the MFMA passes
                            round it down to a power of two that fits   */
    int tile_cols_used;  /* out (bf_get_config, bf_autotune): the width
                            the passes use for a full chunk; 0 per step */
    int switch_otf;      /* BF_PATH_PER_STEP_MFMA only: 1 = generate each
                            switch block during the apply (FP64 phase
                            reduced modulo 1, FP32 sincospi) instead of
                            reading the stored blocks; a plan whose form
                            never reads them does not store them        */
    int max_pass_levels; /* fused forms: levels per pass at most this many
                            (each half then split into equal passes; a
                            single level left over joins the pass before
                            it); 0 = as many as the LDS holds; 0..12   */
    int twiddle_otf;     /* BF_PATH_PER_STEP_MFMA, FP32 only: 1 = evaluate
                            each twiddle entry during the apply exactly as
                            the plan stores it (FP64 phase reduced modulo
                            1, FP64 sincospi, rounded to complex64)
                            instead of reading it (Section 4: Algorithm
                            4.1 applied without precomputed factors).  A
                            plan built with the environment variable
                            BF_TWIDDLE_OTF=1 (and BF_FUSED=0) stores no
                            twiddles and runs only with twiddle_otf = 1  */
} bf_config;

/* Current execution form of the plan. */
int bf_get_config(bf_plan_t plan, bf_config* cfg);

/* Makes cfg the plan's execution form (synchronous; tile_cols_used is
 * ignored).  Grows the plan's default workspace when the form needs more
 * (bf_workspace_bytes reports the new size).  Returns BF_EINVAL for an
 * unknown path or a bad width, BF_EUNSUPPORTED when the form cannot run
 * this plan (a pass does not fit the LDS, or a split precision off the
 * MFMA passes; the plan is then unchanged), BF_EBUSY while graphs captured
 * from the plan exist.                                                    */
int bf_set_config(bf_plan_t plan, const bf_config* cfg);

/* Autotuner: times every candidate execution form on the caller's buffers
 * (f, g as for bf_apply, nvec vectors, on stream): one warm-up apply, then
 * reps timed applies (hipEvents), and makes the fastest the plan's form.
 * Candidates: BF_PATH_FUSED and BF_PATH_FUSED_VALU at tile widths r * 2^j
 * <= 16, BF_PATH_PER_STEP, and BF_PATH_PER_STEP_MFMA with stored and with
 * on-the-fly switch blocks (the stored blocks are built first if the plan
 * has none), each also with twiddles evaluated in the apply; out (capacity
 * cap) receives one entry per
 * candidate with its mean milliseconds per apply, -1 when the form cannot
 * run the plan, -2 when it resolves to kernels already timed; *count
 * receives the number of candidates.  Synchronous; allocates a temporary
 * workspace; g holds the result of the last timed form.  BF_EBUSY while
 * graphs captured from the plan exist.                                     */
typedef struct bf_tune_entry {
    bf_config config;
    double ms;
} bf_tune_entry;

int bf_autotune(bf_plan_t plan, int nvec, const void* f, void* g, int reps,
                void* stream, bf_tune_entry* out, int cap, int* count);

/* ---- captured applies (HIP graphs) --------------------------------------
 * bf_graph_create records the kernels of bf_apply(plan, nvec, f, g) into an
 * executable HIP graph (captured on a private stream; nothing runs), bound
 * to f, g and the plan's default workspace.  bf_graph_launch replays it on
 * stream: the same computation as bf_apply with one launch call, for small
 * problems where launch overhead dominates.  Replays and bf_apply share the
 * workspace, so they must not overlap.  The graph holds no memset node.
 * While a graph exists the plan cannot be reconfigured or destroyed
 * (BF_EBUSY).  bf_graph_destroy synchronises the device first; NULL is
 * accepted.                                                                */
typedef struct bf_graph_s* bf_graph_t;

int bf_graph_create(bf_plan_t plan, int nvec, const void* f, void* g,
                    bf_graph_t* out);

/* As bf_graph_create for the chain of bf_apply_chain (same arguments and
 * checks): the applies of all plans, ping-ponging between tmp and g, in one
 * graph.  Every plan of the chain holds a reference until bf_graph_destroy
 * (bf_destroy and bf_set_config return BF_EBUSY meanwhile).  For chains of
 * small applies whose launches dominate, e.g. a composition of FIOs.     */
int bf_graph_create_chain(const bf_plan_t* plans, int count, int nvec,
                          const void* f, void* g, void* tmp,
                          bf_graph_t* out);

int bf_graph_launch(bf_graph_t graph, void* stream);
int bf_graph_destroy(bf_graph_t graph);

/* ---- kernel timing (diagnostics) ---------------------------------------
 * bf_profile(plan, 1): every later apply of this plan records a hipEvent
 * pair around each kernel launch it issues, on the apply stream (at most
 * 4096 launches are kept until the next bf_profile_read; later ones are not
 * timed, and launches inside a graph capture never are).  bf_profile(plan, 0)
 * stops recording.  bf_profile_read synchronises the recorded events and
 * returns one entry per kernel class: launches, total milliseconds, the
 * algorithmic bytes (inputs, outputs and factors each counted once) and
 * flops of those launches, and the state bytes they spill through memory;
 * it then clears the records.  stats: caller
 * array of cap entries; *count receives the number of classes.            */
typedef struct bf_kernel_stat {
    char name[48];
    int launches;
    double total_ms;
    double bytes;        /* algorithmic: f, b_k, g, a_k and factors read
                            or written by the launches, each once        */
    double flops;        /* algorithmic (2D: one-dimension-at-a-time
                            contraction of the Kronecker matrices)      */
    double state_bytes;  /* the N r V state (and partial sums) read or
                            written between launches: spills, not part
                            of the algorithmic bytes                     */
} bf_kernel_stat;

int bf_profile(bf_plan_t plan, int enable);
int bf_profile_read(bf_plan_t plan, bf_kernel_stat* stats, int cap,
                    int* count);

/* Message of the last failed call on this thread ("" if none). */
const char* bf_last_error(void);

/* ---- host-only geometry (no device needed) ------------------------------
 * Interpolation offsets of a box of box_size indices with q points
 * (eqs. (eqn:gdA)/(eqn:gdB), ascending-node reading, ties rounded up, all
 * indices when box_size <= q): writes min(q, box_size) 0-based offsets to
 * out (capacity cap) and their count to *count.                          */
int bf_points(int box_size, int q, int* out, int cap, int* count);

/* Lagrange weights M_t(y) of the node set nodes[0..r) at points y[0..m):
 * out[k * r + t] = prod_{j != t} (y_k - x_j) / (x_t - x_j), FP64 (Section
 * 2.1).                                                                   */
int bf_lagrange(const int* nodes, int r, const double* y, int m, double* out);

/* ---- phase recovery under indirect access (Section 3.2) ------------------
 * When K is known only through entry evaluation (Scenario 1 of Table
 * (tab:sc)) or applies of K and K^T (Scenario 2), its samples fix the phase
 * modulo 1 only.  These host routines (FP64, synchronous, no device use)
 * recover a low-rank Psi = U V^T with exp(2 pi i Psi) = exp(2 pi i Phi) for
 * a BF_PHASE_LOWRANK plan.  Phases are in cycles; indices are 0-based.     */

/* Algorithm 3: v (length n) equal to u modulo 1, continued by matching
 * second differences, restarting where 2 pi |second difference| > tau (an
 * angle; the paper uses pi / 2).  disc (capacity cap) receives the restart
 * indices, disc[0] = 0; *ndisc their number (may exceed cap).
 * Returns BF_EINVAL for n < 3, tau <= 0 or NULL pointers.                   */
int bf_unwrap(const double* u, long long n, double tau, double* v,
              long long* disc, int cap, int* ndisc);

/* Algorithm 1 (randomized low-rank factorization) restricted to given
 * samples of a real N x N matrix A: columns cols [nc][N] (cols[k * N + i] =
 * A(i, C[k])) and rows rows [nr][N] (rows[k * N + j] = A(R[k], j)), C and R
 * sorted, distinct, in [0, N), the rows and columns agreeing where they
 * meet.  The important columns and rows are the pivots of pivoted QR / LQ
 * of A(R, C); A ~ U V^T of rank k = *rank_out <= min(rank, cap_rank) (at
 * most the numerical rank of A(R, C)), U, V host [N][cap_rank], columns
 * past k zero.  Used for the amplitude of a kernel known through samples
 * (A = |K|, Section 3.3) and inside bf_recover_phase.  Returns BF_EINVAL
 * for bad arguments or too few samples.                                   */
int bf_lowrank_samples(long long N, const double* cols, const long long* C,
                       int nc, const double* rows, const long long* R, int nr,
                       int rank, int cap_rank, double* U, double* V,
                       int* rank_out);

/* Sampler callback of bf_recover_phase: the phase modulo 1 of count columns
 * (is_row = 0; out [N][count], out[i * count + k] = Phi(i, idx[k])) or rows
 * (is_row = 1; out [count][N], out[k * N + j] = Phi(idx[k], j)).  Returns 0
 * on success.  Scenario 2: the columns of K are K e_j, its rows K^T e_i;
 * the phase is arg(K) / (2 pi) after the amplitude is divided out.        */
typedef int (*bf_phase_sampler)(void* ctx, int is_row, int count,
                                const long long* idx, double* out);

/* Algorithm 5 for a 1D phase: from the sampled columns C (nc indices) and
 * rows R (nr indices), both sorted, distinct, in [0, N) and drawn by the
 * caller (the method's random choice, e.g. rank * oversampling of each),
 * Algorithm 4 recovers unwrapped columns and rows that agree where they
 * meet (sampling the discontinuity rows and columns it detects and each
 * block's first three rows and columns; the detection threshold is tau as
 * in bf_unwrap, none inside a block), then Algorithm 1's factorization
 * restricted to those samples gives Psi ~ U V^T of rank
 * k = *rank_out <= min(rank, cap_rank).  U, V: host [N][cap_rank]
 * row-major, columns past k zero.  Memory: about (nc + nr + 2 k) N doubles
 * of host scratch.  Returns BF_EINVAL for bad arguments, too few samples
 * for the rank, or a failing sampler.                                     */
int bf_recover_phase(long long N, const long long* C, int nc,
                     const long long* R, int nr, int rank, double tau,
                     bf_phase_sampler sample, void* ctx, int cap_rank,
                     double* U, double* V, int* rank_out);

#ifdef __cplusplus
}
#endif
#endif /* BF_H */
