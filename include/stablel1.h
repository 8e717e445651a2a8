/*
 * stablel1 -- Lasso solver with stable safe screening over a sequence of fast
 * approximate dictionaries, for AMD Instinct MI355X (gfx950).
 *
 * Problem (Section I-A, the Lasso): given a dictionary A in R^{N x K}, a signal
 * y in R^N and lambda > 0, find x* = argmin_x 1/2 ||A x - y||^2 + lambda ||x||_1.
 *
 * Method (Algorithm 1, FastL1, with Algorithm 2, SwitchDictionary): FISTA
 * iterations run on a sequence A~^0, ..., A~^I = A of approximations whose atoms
 * are known up to error bounds ||a~_j - a_j||_q <= eps_j (Section III-B; any l_q
 * norm, 1 <= q <= inf, as Lemma 1 and Lemma 2 allow; q = 2 is the usual one).  Each
 * iteration applies the stable GAP Safe sphere test (Table I, last row; Theorem 1)
 * so that rejected atoms are provably inactive for the ORIGINAL problem, and
 * switches to a finer approximation on duality-gap saturation (Section IV-A) or
 * straight to A when the preserved set is small enough (Sections IV-B, IV-C).
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer (memory of the current HIP device)
 *     unless its description says "host".
 *   - Dense matrices are column-major: atom j occupies A[j*N .. j*N+N-1].
 *   - Kronecker atoms: atom j = j1*k2 + j2, row i = i1*n2 + i2 and
 *     (B kron C)[i, j] = B[i1, j1] * C[i2, j2]; term r of B is column-major
 *     n1 x k1 at B + r*n1*k1 (element (i1, j1) at j1*n1 + i1), same for C.
 *   - BF16 arrays hold bfloat16 bit patterns (uint16); FP8 arrays hold OCP FP8
 *     E4M3FN codes (uint8, largest finite value 448).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Return value: 0 = SL1_OK, > 0 = warning (outputs valid), < 0 = error
 *     (outputs untouched or undefined).  Argument checks are synchronous on the
 *     host; errors met on the device are reported through the return value of
 *     the call that waits for them (sl1_solve, sl1_lambda_max, sl1_grad).
 *   - Implementation limits (SL1_ELIMIT): N % 4 == 0; N <= 8192; K <= 262144; Kronecker
 *     factor sizes n1, k1, n2, k2 multiples of 16; at most SL1_MAX_STAGES stages.
 */
#ifndef STABLEL1_H
#define STABLEL1_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SL1_MAX_STAGES 8
#define SL1_TRACE_FIELDS 13

enum sl1_status_code {
    SL1_OK = 0,
    SL1_MAXITER = 1,      /* warning: a signal stopped at max_iter; its gap may exceed tol */
    SL1_EINVAL = -1,      /* bad value: lambda <= 0, non-finite input, eps < 0, NULL pointer, ... */
    SL1_ESHAPE = -2,      /* inconsistent sizes between dictionaries or arguments */
    SL1_EDTYPE = -3,      /* unsupported storage / working precision combination */
    SL1_EHIP = -4,        /* a HIP runtime call failed */
    SL1_ENOMEM = -5,      /* device or host allocation failed */
    SL1_ESINGULAR = -6,   /* singular Gram matrix on the support (sl1_grad) */
    SL1_ELIMIT = -7       /* outside a documented implementation limit */
};

enum sl1_dtype {
    SL1_F64 = 0,
    SL1_F32 = 1,
    SL1_BF16 = 2,
    SL1_FP8_E4M3 = 3
};

/* Immutable dictionary handle (one stage of the sequence). */
typedef struct sl1_dict_s* sl1_dict;

/*
 * sl1_dict_dense -- a dense stage A~ (or the exact A).
 *   dtype      storage type: SL1_F64, SL1_F32, SL1_BF16 or SL1_FP8_E4M3.
 *   N, K       rows (signal length) and atoms.
 *   A          N x K column-major storage, device.  BORROWED: the caller keeps it
 *              alive and unchanged until sl1_dict_free.
 *   col_scale  optional (may be NULL) K floats, device: atom j is
 *              col_scale[j] * decode(A[:, j]).  Copied.
 *   eps        K doubles, device: bounds eps_j >= ||a~_j - a_j||_q against the
 *              exact dictionary (Section III-B; all zero for the exact A).  Copied.
 *              The library adds to each eps_j a bound on its own rounding in the
 *              products with this stage, so the test stays safe (Lemma 1, Lemma 2,
 *              Theorem 1 hold with the enlarged bounds).
 *   q          the norm of the bounds, 1 <= q <= inf (INFINITY accepted); 2 for l2
 *              bounds.  The dual scaling and the test pair eps with ||z||_{q*},
 *              1/q + 1/q* = 1 (Lemma 1 with an l_q zone, Lemma 2), and Theorem 1
 *              uses the l2 column bound N^((1/2 - 1/q)_+) eps_j (the Hoelder
 *              constant of the Appendix).  Stages with q != 2 run in the grid engine:
 *              SL1_ENGINE_WG refuses them with SL1_ELIMIT, and the hybrid engine
 *              keeps the grid kernels throughout when the last stage has q != 2.
 * Errors: SL1_EINVAL (NULL A/eps, N or K < 1, q < 1 or NaN), SL1_EDTYPE, SL1_ELIMIT,
 * SL1_EHIP, SL1_ENOMEM.
 */
int sl1_dict_dense(sl1_dict* out, int dtype, int64_t N, int64_t K, const void* A,
                   const float* col_scale, const double* eps, double q, void* stream);

/*
 * sl1_dict_kron -- a structured stage A~ = sum_{r<R} B_r kron C_r (the SuKro model
 * of Section V-A), N = n1*n2, K = k1*k2.
 *   dtype      SL1_F64, SL1_F32, SL1_BF16 or SL1_FP8_E4M3 (factor storage).  FP8
 *              factors are decoded exactly to BF16 for the BF16 matrix-core products
 *              (FP32 accumulation), so they carry the BF16 rounding allowance; stages
 *              with FP8 factors run in the grid engine (SL1_ENGINE_WG refuses them
 *              with SL1_ELIMIT; the automatic choice never picks it for them).
 *   B, C       R*n1*k1 and R*n2*k2 elements, device, layout in the header comment.
 *              Copied (the factors are small).  A non-finite entry is SL1_EINVAL.
 *   eps, q     as for sl1_dict_dense (eps copied).
 * Errors: SL1_EINVAL, SL1_EDTYPE, SL1_ELIMIT, SL1_EHIP, SL1_ENOMEM.
 */
int sl1_dict_kron(sl1_dict* out, int dtype, int R, int n1, int k1, int n2, int k2,
                  const void* B, const void* C, const double* eps, double q, void* stream);

/*
 * sl1_dict_faust -- a structured stage A~ = S_1 S_2 ... S_J, a product of sparse
 * factors (the FAuST model cited in Section I-D, used for the MEG operator of
 * Section V-G and Table V).  S_l has dims[l-1] x dims[l] entries (0-based: S_l
 * is factor l-1 below), dims[0] = N, dims[J] = K.
 *   dtype      SL1_F64 or SL1_F32 (factor values; products accumulate in FP64).
 *   J          number of factors, 1 .. 8.
 *   dims       host, J+1 sizes: N (multiple of 4, <= 1024), inner sizes <= 1024, K.
 *   nnz        host, J entry counts.
 *   row_ptr    host, CSR row pointers of every factor, concatenated (dims[l] + 1
 *              entries for factor l, starting at 0 and ending at nnz[l]).
 *   col_idx    host, CSR column indices, concatenated (nnz[l] for factor l;
 *              strictly increasing within a row).
 *   val        host, values in dtype, concatenated like col_idx.
 *   eps, q     as for sl1_dict_dense.
 * Everything is copied; the transposed factors, ||a~_j|| and the rounding allowance
 * of the chain's FP64 sums are formed here.  FAuST stages run in the grid engine
 * (SL1_ENGINE_WG refuses them with SL1_ELIMIT).
 * Errors: SL1_EINVAL (malformed CSR, non-finite values, bad eps), SL1_EDTYPE,
 * SL1_ELIMIT, SL1_EHIP, SL1_ENOMEM.
 */
int sl1_dict_faust(sl1_dict* out, int dtype, int J, const int64_t* dims, const int64_t* nnz,
                   const int32_t* row_ptr, const int32_t* col_idx, const void* val, const double* eps,
                   double q, void* stream);

/* Releases a handle; NULL is accepted and ignored. */
int sl1_dict_free(sl1_dict d);

/*
 * sl1_dict_info -- host outputs (any may be NULL): sizes, the largest bound
 * max_j eps_j as given, and the relative-complexity model of the stage
 * (1 for dense full precision, bytes per element / 4 for BF16 and FP8 storage,
 * R (1/n1 + 1/k2) for Kronecker sums, nonzeros / (N K) for FAuST chains;
 * Section IV-B and Table IV).
 */
int sl1_dict_info(sl1_dict d, int64_t* N, int64_t* K, double* eps_max, double* rc_model);

/* Solver options (sl1_opts_default fills the defaults given in brackets). */
typedef struct {
    double Gamma;        /* [0.5] gap-ratio switching threshold (Section IV-A; Section V-C) */
    double tol;          /* [1e-6] stop once on A with conventional duality gap < tol */
    double margin;       /* [1e-12] reject atom j iff its test value < 1 - margin */
    int32_t max_iter;    /* [100000] iteration cap per signal */
    int32_t y_dtype;     /* [SL1_F32] storage type of the signals y: SL1_F64 or SL1_F32 */
    int32_t chunk;       /* [16] grid engine: iterations enqueued between two convergence polls
                            (rounded up to even); whole-solve engine: at most 256*chunk
                            iterations per launch */
    int32_t flags;       /* [0] SL1_FLAG_* */
    double* trace;       /* [NULL] optional device buffer, batch x trace_cap x SL1_TRACE_FIELDS
                            doubles: per iteration t, stage, |A_t|, |A_t+1|, K_t, G(x,theta'|A~),
                            G(x,theta~|A~), delta, radius of the test's sphere (R' for stable GAP
                            Safe, ||theta'-y/lambda|| for stable Dynamic Safe), gamma, ||x_t||_1,
                            P(x_t|A~), ||x_t||_0 */
    int32_t trace_cap;   /* [0] rows per signal in `trace` */
    int32_t screen_every;/* [1] reject atoms only at iterations t with t % screen_every == 0 (the
                            variation of Algorithm 1 that screens at regular intervals); dual
                            points, gaps and K_t are still formed every iteration; 0 = 1 */
    int32_t gemm_signals;/* [64] grid engine: the batched correlation product (SL1_FLAG_NO_GEMM)
                            runs in a chunk of iterations when at least this many signals
                            qualified at the end of the previous chunk (and in the first chunk
                            when the batch has this many); 0 = 64 */
    const double* x0;    /* [NULL] optional device buffer, batch x K doubles: the initial iterate
                            (warm start, e.g. the solution at the previous lambda of a path --
                            the sequential setting of Section I-D). The preserved set still starts
                            with every atom and the first step has no momentum, so the test stays
                            safe for any x0; a non-finite entry makes that signal SL1_EINVAL.
                            NULL: x_0 = 0 (Algorithm 1) */
} sl1_opts;

#define SL1_FLAG_NO_GRAPH 1   /* launch iterations directly instead of replaying a hipGraph */
#define SL1_FLAG_PROFILE 2    /* direct launches bracketed by HIP events; see sl1_last_solve_profile */
#define SL1_FLAG_ENGINE_GRID 4    /* force the per-iteration grid engine throughout */
#define SL1_FLAG_ENGINE_WG 8      /* force the whole-solve engine (SL1_ELIMIT if its LDS need exceeds 159 KB) */
#define SL1_FLAG_ENGINE_HYBRID 16 /* grid engine, then the tail kernel (SL1_ELIMIT if a dense last stage's
                                     tail layout exceeds 159 KB; the grid engine alone when the last
                                     stage is not dense) */
#define SL1_FLAG_TAIL_COLUMNS 32  /* the tail kernel forms every iteration's products from the stored
                                     columns (no Gram mode) */
#define SL1_FLAG_HYBRID_GRID_FIRST 1024 /* hybrid engine: run the Kronecker approximations on the grid
                                     kernels too (by default they run in the whole-solve kernel) */
#define SL1_FLAG_GRID_SPLIT_STEP 2048   /* grid engine: chip-wide forward and update launches throughout
                                     (by default, for batches of at least 128 signals, while every live
                                     signal can only be on dense stages and without l_q bounds or the
                                     dome rule, one launch per iteration does the update and the next
                                     forward, one block per signal) */
#define SL1_FLAG_GRID_STEP 4096         /* grid engine: those per-signal step launches for any batch size
                                     (not together with SL1_FLAG_GRID_SPLIT_STEP: SL1_EINVAL) */
#define SL1_FLAG_PARK_ALL 8192          /* hybrid engine: the grid kernels start only once every live signal
                                     has left the whole-solve phase on the Kronecker approximations (by
                                     default, for batches of at least 128 signals with a dense last stage
                                     and step launches, they start once at most batch / 128 are still on
                                     the approximations, and those go on in a whole-solve launch on a
                                     second stream until they reach A, then join) */
#define SL1_FLAG_ISTA 64          /* ISTA update x_{t+1} = ST(x_t + A~^T rho~_t / L) (Section I-B)
                                     instead of FISTA */
#define SL1_FLAG_NO_GEMM 256      /* grid engine: correlations of every signal stream its own preserved
                                     columns (by default, signals on the exact dense stage with
                                     |A_t| >= max(4 a ceil(K/64), K/8), a = 2 for N <= 1024 else 1,
                                     share one FP64 matrix-core product A^T Z over tiles of 64 atoms
                                     x 64 signals; see gemm_signals) */
#define SL1_FLAG_RULE_DST 128     /* stable Dynamic Safe test (Table I, fourth row) instead of stable
                                     GAP Safe: sphere B(y/lambda, ||theta'_t - y/lambda||) tested with
                                     a_j^T y formed once on the exact dictionary (footnote to Table I;
                                     the solve first runs one correlation pass of seq[n_stages-1] over
                                     all atoms, which must be dense: SL1_ELIMIT otherwise) */
#define SL1_FLAG_RULE_DOME 512    /* stable GAP Safe sphere intersected with the GAP dome of the same dual
                                     point theta'_t: the ball with diameter [theta'_t, y/lambda] (theta*
                                     is the projection of y/lambda, Section II-C) cut by the half-space
                                     that keeps theta* at distance >= sqrt(||y||^2 - 2(P(x|A~) +
                                     delta(x)))/lambda from y/lambda (weak duality with Theorem 1's
                                     bound); the dome region the paper names as an extension (Section
                                     I-E), tested over Lemma 1's zone.  An atom is kept when the smaller
                                     of the two tests is >= 1 - margin.  Needs a_j^T y like
                                     SL1_FLAG_RULE_DST (dense exact stage; not together with it:
                                     SL1_EINVAL); grid engine only (SL1_FLAG_ENGINE_WG: SL1_ELIMIT;
                                     the hybrid engine keeps the grid kernels) */

/* Engines (at most one SL1_FLAG_ENGINE_* flag; none = automatic):
 *   SL1_ENGINE_GRID    five persistent launches per iteration covering every live
 *                      signal (any size within the limits; captured in hipGraph chunks);
 *   SL1_ENGINE_WG      one 512-thread workgroup per signal runs the whole solve in one
 *                      launch (per-signal z and the current stage's Kronecker factors in
 *                      LDS); launches are bounded and repeated while signals remain;
 *   SL1_ENGINE_HYBRID  when every stage before the last is a Kronecker stage (and the
 *                      whole-solve layout fits), those stages run in the whole-solve
 *                      kernel, each signal stopping there on reaching the last stage;
 *                      then (or from the start, for other sequences) the grid engine
 *                      until, after a chunk, every live signal is on the last (dense)
 *                      stage and its preserved set holds at most ~2 MiB of columns
 *                      or fits the Gram capacity (up to 128 atoms); the remaining
 *                      iterations then run in a tail kernel, one workgroup per
 *                      signal with the preserved set's state in LDS.
 *                      Once a signal's |A_t| fits the Gram capacity, the tail kernel
 *                      forms G = A_t^T A_t and A_t^T y once (FP64) and iterates on
 *                      them (g = A_t^T y - G x, ||y - Ax||^2 and y^T(y - Ax) from the
 *                      same forms), with the FP64 rounding of these forms bounded and
 *                      added to the test and to delta (SL1_FLAG_TAIL_COLUMNS: never).
 * Automatic choice: whole-solve when its LDS need fits and N*K <= 2^20, hybrid when the
 * last stage is dense and N*K is larger, grid otherwise.  All compute every per-element
 * quantity with the same expressions; results differ only by the order of FP64
 * reductions (and, in Gram mode, by the Gram forms of the same products). */
#define SL1_ENGINE_GRID 1
#define SL1_ENGINE_WG 2
#define SL1_ENGINE_HYBRID 3

int sl1_opts_default(sl1_opts* o);

/*
 * sl1_solve -- Algorithm 1 on a batch of independent signals sharing the
 * dictionary sequence seq[0..n_stages-1]; seq[n_stages-1] must be the exact A
 * (eps = 0; Algorithm 1 input).  Stages must share N and K.
 *   L          host, n_stages doubles: step-size constants L_i >= ||A~^i||_2^2.
 *   rc         host, n_stages doubles: relative complexities RC(A~^i) used by the
 *              speed criterion (Section IV-B); rc[n_stages-1] is ignored.
 *   atom_norm  K doubles: ||a_j||_2 of the exact atoms (restricted zone, Lemma 1).
 *   batch      number of signals (>= 1).
 *   y          batch x N in opt->y_dtype (signal b at y + b*N).
 *   lambda     batch doubles, each > 0.
 *   x          out, batch x K doubles: the solution, zero on screened atoms.
 * Precision: iterates, residuals, correlations, gaps and tests are FP64; each
 * stage's products read its own storage type (FP64 / FP32 / BF16 / FP8) with
 * FP64 accumulation, except FP32 and BF16 Kronecker products, which run on the
 * matrix cores with FP32 accumulation (their rounding is covered by eps).
 *   gap        out, batch doubles: conventional duality gap G(x, theta|A) at x.
 *   gap_cert   out (may be NULL), batch doubles: G(x, theta'|A~) + delta(x) at x, an
 *              upper bound of the gap of the exact problem (Theorem 1).
 *   screened   out (may be NULL), batch x K bytes: 1 = atom rejected by the test.
 *   iters      out (may be NULL), batch int32: iterations performed.
 *   stage      out (may be NULL), batch int32: index of the final stage.
 * The stop test precedes the screening step of its iteration (Algorithm 1), so
 * `screened` holds the atoms rejected before the stop.  For lambda >= lambda'_max of
 * seq[0] the first test rejects every atom except near-ties; for lambda_max <= lambda <
 * lambda'_max the solve returns x = 0 on A with the atoms rejected until then.
 * The call orders itself after prior work on `stream`, polls convergence and
 * returns once every signal has converged or reached max_iter; the outputs are
 * then complete.  Internally it runs on the workspace's own stream and, in a hybrid
 * solve of 128 signals or more, on a second stream of the workspace for a few late
 * signals (see SL1_FLAG_PARK_ALL); both are joined before the call returns.  Concurrent calls with identical shapes on one device are
 * serialised internally; calls with other shapes use other workspaces and may run
 * concurrently (a cached workspace is released only when no call holds it).
 * Returns SL1_OK, SL1_MAXITER, SL1_EINVAL (bad lambda / non-finite y detected on
 * the device), SL1_ESHAPE, SL1_EDTYPE, SL1_ELIMIT, SL1_EHIP or SL1_ENOMEM.
 */
int sl1_solve(const sl1_dict* seq, int n_stages, const double* L, const double* rc,
              const double* atom_norm, int64_t batch, const void* y, const double* lambda,
              const sl1_opts* opt, double* x, double* gap, double* gap_cert, uint8_t* screened,
              int32_t* iters, int32_t* stage, void* stream);

/*
 * sl1_solve_noalloc -- sl1_solve for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, checks, kernels and results as sl1_solve, with
 * the workspace laid out in a fixed device array of 64 MiB that the library holds
 * on each device it runs on until the process ends.  It calls no hipMalloc,
 * hipFree or other allocating routine: it launches on `stream` itself (no library
 * stream, events or graphs; iterations are launched directly, which gives results
 * bit-identical to the replayed graphs of sl1_solve) and clears the array with a
 * fill kernel at the start of each call.  The caller still passes every input and
 * output.  The dictionary handles are made beforehand with the sl1_dict_* calls.
 *   Limit: the workspace of (batch, N, K) must fit 64 MiB; it takes about
 *   batch * (89 K + 8 N + 9 KiB) bytes plus 16 MiB for the batched product's tiles,
 *   and batch * (8 K + 8) more with SL1_FLAG_RULE_DST or SL1_FLAG_RULE_DOME (e.g.
 *   up to ~130 signals at N = 1024, K = 4096).  Larger requests return SL1_ELIMIT
 *   before any device work.  SL1_FLAG_PROFILE is refused (SL1_EINVAL); the
 *   sl1_last_solve_* queries do not see these solves.
 *   Concurrency: every call on one device shares that device's array, which keeps
 *   the last call's contents.  Calls from host threads are serialised by the
 *   library; calls that overlap on the device in any other way (e.g. the same
 *   graph-captured call replayed on two streams at once) race and give undefined
 *   results.
 * Returns as sl1_solve, plus SL1_ELIMIT for a workspace beyond the array.
 */
int sl1_solve_noalloc(const sl1_dict* seq, int n_stages, const double* L, const double* rc,
                      const double* atom_norm, int64_t batch, const void* y, const double* lambda,
                      const sl1_opts* opt, double* x, double* gap, double* gap_cert, uint8_t* screened,
                      int32_t* iters, int32_t* stage, void* stream);

/*
 * sl1_lambda_max -- out[b] = max_j (|a~_j^T y_b| + eps_j ||y_b||_{q*}), the stable
 * lambda'_max of Section III-C for the stage's bound norm q (equal to
 * lambda_max = ||A^T y_b||_inf when eps = 0).
 *   y    batch x N in y_dtype;  out  batch doubles.  Includes the library's own
 *        rounding allowance, so it is an upper bound.  Synchronous.
 */
int sl1_lambda_max(sl1_dict d, int64_t batch, const void* y, int y_dtype, double* out,
                   void* stream);

/*
 * sl1_dict_adjoint -- out[b*K + j] = a~_j^T z_b for every atom j, computed by the
 * solver's own correlation kernel for this stage (the adjoint product of
 * Algorithm 1's update, A~^T rho~).  z_b is y_b as the solver stores it: y_b
 * itself, or its FP32 / BF16 rounding for FP32 / BF16 Kronecker stages (written
 * to z_used, batch x N doubles, when z_used is not NULL).
 *   y    batch x N in y_dtype;  out  batch x K doubles.  Synchronous.
 */
int sl1_dict_adjoint(sl1_dict d, int64_t batch, const void* y, int y_dtype, double* out,
                     double* z_used, void* stream);

/*
 * sl1_grad -- implicit adjoint of the Lasso solution map on the support
 * S_b = {j : x_b[j] != 0}: from the optimality conditions (Section II),
 * A_S^T A_S x_S = A_S^T y - lambda sign(x_S), so for a loss L(x*):
 *   dL/dy      = A_S (A_S^T A_S)^{-1} (dL/dx)_S
 *   dL/dlambda = -sign(x_S)^T (A_S^T A_S)^{-1} (dL/dx)_S
 *   A          the exact dictionary (dense stage).
 *   x, dx      batch x K doubles (solution and incoming gradient).
 *   y          batch x N in y_dtype (unused by the formula; kept for symmetry).
 *   dy         out, batch x N in y_dtype;  dlambda  out, batch doubles.
 * Returns SL1_ESINGULAR if a support Gram matrix is not positive definite,
 * SL1_ELIMIT if a support exceeds 1024 atoms or N.  Synchronous.  Its device
 * memory is kept per device, grown to the largest call and held until the
 * process ends; calls on one device are serialised.
 */
int sl1_grad(sl1_dict A, int64_t batch, const double* x, const void* y, const double* lambda,
             const double* dx, void* dy, double* dlambda, int y_dtype, void* stream);

/*
 * sl1_measure_rc -- measured relative complexity of each stage: the device
 * time of one iteration's products with seq[i] divided by that of the last
 * stage with every atom preserved (Section IV-B, Section V-A measures RC
 * instead of using the model).  rc_out: host, n_stages doubles.  Synchronous.
 */
int sl1_measure_rc(const sl1_dict* seq, int n_stages, int64_t batch, double* rc_out,
                   void* stream);

/*
 * sl1_tune_kron -- the autotuner of the Kronecker correlation tile shape.  Every
 * Kronecker stage of seq is timed with each usable item shape kt2 x kt1 (atoms j2 x j1
 * per item, kt2, kt1 in {16, 32, 64, 128} dividing k2 and k1, at least two 16 x 16
 * output tiles, the item's intermediate within 96 KB of LDS) on `batch` synthetic
 * signals, and the fastest shape is recorded in the stage's handle; later solves,
 * lambda and adjoint calls use it.  Other stages are left as they are.
 *   shape_out  host, 2 n_stages int32 (may be NULL): (kt2, kt1) chosen per stage, 0 0
 *              for stages that are not Kronecker sums.
 *   ms_out     host, n_stages doubles (may be NULL): the chosen shape's launch time.
 * The shape changes the order of the FP32 sums only (within the stage's rounding
 * allowance).  A handle's shape is the one property that changes after creation: do
 * not tune handles that a concurrent call is using.  Synchronous.
 */
int sl1_tune_kron(const sl1_dict* seq, int n_stages, int64_t batch, int32_t* shape_out, double* ms_out,
                  void* stream);

/*
 * sl1_dict_kron_tile -- sets the correlation tile shape of a Kronecker stage by hand
 * (kt2 x kt1 atoms per item, multiples of 16 dividing k2 and k1, the item's
 * intermediate within 96 KB; the tuner's candidates are a subset).  SL1_EINVAL for
 * another kind of stage or an unusable shape.  Same caveat as sl1_tune_kron.
 */
int sl1_dict_kron_tile(sl1_dict d, int kt2, int kt1);

/*
 * sl1_last_solve_clock -- device wall-clock stamps of the most recent
 * sl1_solve with these shapes on the current device: out[2b] = start of signal
 * b, out[2b+1] = iteration at which its gap first fell below tol (0 if never).
 * out: host, 2*batch int64; rate_khz: host, clock rate.  For time-to-gap.
 */
int sl1_last_solve_clock(int64_t batch, int64_t N, int64_t K, long long* out, double* rate_khz);

/*
 * sl1_last_solve_profile -- per-kernel device time of the grid kernels in the
 * most recent sl1_solve with SL1_FLAG_PROFILE and these shapes: ms[k] total
 * milliseconds and launches[k] launch count of k = 0 forward/residual, 1 dense
 * correlations, 2 Kronecker correlations, 3 scalar block + test/update/compaction,
 * 4 batched dense correlations, 5 the pass that finishes row-split product tiles,
 * 6 the per-signal step (update of one iteration and forward of the next; see
 * SL1_FLAG_GRID_SPLIT_STEP) (host arrays of 7).
 */
int sl1_last_solve_profile(int64_t batch, int64_t N, int64_t K, double* ms, long long* launches);

/*
 * sl1_last_solve_phases -- engine that ran the most recent sl1_solve with these
 * shapes (*engine = SL1_ENGINE_GRID, _WG or _HYBRID) and, when it was run with
 * SL1_FLAG_PROFILE, for its whole-solve part: phase_ms[0..3] (host, 11 doubles,
 * may be NULL) workgroup milliseconds summed over signals of forward/residual,
 * dense correlations, Kronecker correlations (hybrid tail: Gram-mode
 * correlations and scalars) and test/update/compaction,
 * phase_ms[4] the elapsed milliseconds of the whole-solve launches and
 * *wg_launches (may be NULL) their number; for a hybrid solve whose Kronecker
 * approximations ran in the whole-solve kernel, phase_ms[5] the elapsed
 * milliseconds of those launches (part of phase_ms[4]), phase_ms[6..9] their
 * four phase sums (not part of phase_ms[0..3]) and phase_ms[10] their number (a
 * launch beside the grid kernels for late signals included; its time overlaps
 * theirs); *gram_cap (may be NULL) the Gram
 * capacity (atoms) of the hybrid tail, 0 when no tail ran or it had no Gram mode:
 * a signal's tail iterations with |A_t| <= *gram_cap ran in the Gram form;
 * *gemm_min (may be NULL) the |A_t| from which a grid iteration of a signal on the
 * exact dense stage went through the batched correlation product (0: never).
 * sl1_last_solve_profile covers the grid kernels.
 */
int sl1_last_solve_phases(int64_t batch, int64_t N, int64_t K, int32_t* engine, double* phase_ms,
                          long long* wg_launches, int32_t* gram_cap, int32_t* gemm_min);

const char* sl1_status_str(int status);
const char* sl1_version(void);

#ifdef __cplusplus
}
#endif
#endif /* STABLEL1_H */
