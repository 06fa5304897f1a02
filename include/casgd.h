/*
 * casgd.h -- C ABI of libcasgd: s-step (communication-avoiding) mini-batch SGD
 * for L2-regularised logistic regression (and the linear and Poisson models
 * of the same paper) on AMD Instinct MI355X (gfx950).
 *
 * Method: "Mixed-Precision Communication-Avoiding SGD for Generalized Linear
 * Models on GPUs". One outer iteration (Algorithm 1) samples s blocks of b
 * rows Y = X[I,:], forms the margins r = Y x and the strict block-lower part
 * of the Gram matrix G = Y Y^T, runs the s dependent residual corrections
 * (Algorithm 1, inner loop) and applies one update x += (eta/b) Y^T delta.
 * The L2 term (lambda/2)||x||^2, which the paper does not have, is folded in
 * as the per-step decay beta = 1 - eta*lambda:
 *     z_j   = beta^j r_j + (eta/b) sum_{i<j} beta^(j-1-i) G_{j,i} delta_i
 *     delta_j = y_{I_j} / (1 + exp(y_{I_j} z_j))      (= y (1 - sigma(y z)), Sec. 3.1)
 *     x    <- beta^s x + (eta/b) Y^T c,   c_i = beta^(s-1-i) delta_i.
 * This is exactly s plain SGD steps on the same samples (Sec. 5.1,
 * Assumption 6: the exact block is the composition of s mini-batch steps).
 *
 * Sampling (Algorithm 1, first step: i.i.d. uniform with replacement; the
 * paper does not fix a generator): sample number t of stream `seed` is
 * SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) output t, i.e.
 * mix(seed + (t+1) * 0x9E3779B97F4A7C15), mapped to a row by the high 64 bits
 * of its 128-bit product with m. Outer iteration h uses samples
 * h*s*b ... (h+1)*s*b - 1 and block j of it the b samples starting at
 * h*s*b + j*b, so plain SGD (s = 1) visits the same rows in the same order
 * for every s.
 *
 * Conventions for every entry point:
 *  - Pointers marked (device) are device memory of the current HIP device;
 *    pointers marked (host) are host memory. The caller owns every buffer;
 *    the library never allocates or frees device memory. Scratch memory comes
 *    from the caller's workspace `ws` (device, 256-byte aligned), sized by the
 *    matching *_workspace_size call, and is only valid for the problem shape
 *    it was sized for.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work
 *    is enqueued and the call returns without waiting.
 *  - Argument errors are reported synchronously by the return value, with a
 *    message from casgd_last_error() (per thread). Device-side conditions
 *    (non-finite values, a grid barrier that did not complete) are recorded
 *    in the workspace and reported by casgd_check() after the stream has been
 *    synchronised. No C++ exception crosses this interface.
 *  - Calls on distinct workspaces may run concurrently; calls sharing one
 *    workspace must be ordered on one stream.
 *  - Results are bitwise reproducible for a fixed (problem, b, s, seed,
 *    launch configuration); reductions use fixed orders, never atomics on
 *    floating-point data.
 */
#ifndef CASGD_H
#define CASGD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t casgd_status;
enum {
    CASGD_OK = 0,
    CASGD_EINVAL = -1,       /* invalid argument */
    CASGD_EUNSUPPORTED = -2, /* valid but not supported (shape, dtype, limit) */
    CASGD_ENOMEM = -3,       /* workspace too small */
    CASGD_EDEVICE = -4,      /* HIP runtime error */
    CASGD_ENONFINITE = -5,   /* a margin, residual or weight became NaN/Inf */
    CASGD_ETIMEOUT = -6      /* a grid barrier of the fused kernel timed out */
};

/* Storage formats of X (Table 1 storage slot u_A). */
enum {
    CASGD_F32 = 0,      /* IEEE binary32 */
    CASGD_BF16 = 1,     /* bfloat16 bits (uint16) */
    CASGD_F16 = 2,      /* IEEE binary16 */
    CASGD_FP8E4M3 = 3   /* OCP FP8 E4M3 (bias 7, max 448, no Inf); needs row_scale */
};

/* Losses of the generalized linear model (Sec. 2.1) with their residuals
 * delta = -dL/dz at the margin z = a^T x (Sec. 3.1):
 *   LOGISTIC  L = log(1 + exp(-y z)), y in {-1, +1}   delta = y / (1 + exp(y z))
 *   LINEAR    L = (z - y)^2 / 2, y real               delta = y - z
 *   POISSON   L = exp(z) - y z, y >= 0 (counts)       delta = y - exp(z)
 * Only the residual formula of the s-step recurrence and the evaluated loss
 * depend on it; sampling, Gram, margins and update are the same kernels. */
enum { CASGD_LOSS_LOGISTIC = 0, CASGD_LOSS_LINEAR = 1, CASGD_LOSS_POISSON = 2 };

/* Matrix layouts. */
enum { CASGD_DENSE = 0, CASGD_CSR = 1 };

/*
 * A feature matrix X with m rows (samples) and n columns (features).
 * DENSE: `values` (device) holds m rows of `ld` elements of `dtype`, row i at
 *   values + i*ld; ld >= n, ld*elementsize a multiple of 16 bytes and the base
 *   16-byte aligned. Columns n..ld-1 are never read.
 * CSR: `row_ptr` (device, int64, m+1), `col_idx` (device, int32, nnz, strictly
 *   increasing within each row, < n) and `values` (device, FP32, nnz); dtype must be
 *   CASGD_F32; ld is ignored.
 * `row_scale` (device, FP32, m) or NULL: the stored row i represents
 *   row_scale[i] * values[i,:]. Required for CASGD_FP8E4M3, optional otherwise.
 */
typedef struct {
    int64_t m, n, ld;
    int32_t dtype;
    int32_t layout;
    const void *values;
    const float *row_scale;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    int64_t nnz;
} casgd_matrix;

/* Execution options; a NULL pointer means all defaults (zeros). */
typedef struct {
    /* Precision of the inner residual corrections (slot u_c, Sec. 5.2):
     * 0 = automatic (FP64 when s*b >= 512, else FP32), 32 = FP32, 64 = FP64. */
    int32_t recur_prec;
    /* 0 = automatic (fused), 1 = one fused persistent launch for the whole
     * fit, 2 = one launch per phase, stream ordered. With b = 16, 32, 64 or
     * 128 the recurrence runs on one chain workgroup plus helper workgroups
     * that add the older column blocks (stream ordered always; fused from
     * s = 4 on, as fused variant 3); otherwise on one workgroup. Forms that
     * sum the recurrence in different orders agree to rounding; each is
     * bitwise reproducible. */
    int32_t exec_mode;
    /* Snapshots: when > 0, after every `snapshot_every` outer iterations the
     * current x is copied to x_history (device, FP32, row k = snapshot k,
     * n_outer / snapshot_every rows of n) and, if t_history (device, int64)
     * is not NULL, the device wall clock (100 MHz ticks) to t_history[k]. */
    int64_t snapshot_every;
    float *x_history;
    int64_t *t_history;
    /* Spin limit of every bounded wait on the device (the fused kernel's
     * grid barrier, the recurrence workgroups' exchange; 0 = default, about
     * 2 s). */
    int64_t spin_limit;
    /* Tuning knobs of the fused kernel (0 = automatic):
     * fused_variant 1 = every update workgroup runs the recurrence itself
     *   (one grid barrier per outer iteration; for small s*b),
     * fused_variant 2 = one workgroup runs the recurrence while the others
     *   compute the next outer iteration's Gram (two barriers);
     * fused_variant 3 = the multi-workgroup recurrence (chain + helpers, as
     *   in exec_mode 2) runs while the other workgroups compute the next
     *   Gram; two grid barriers (b = 16, 32, 64, 128);
     * grid_blocks = number of workgroups of the fused launch (capped at the
     *   number that can be resident). */
    int32_t fused_variant;
    int32_t grid_blocks;
    /* Phase clock of the fused kernel (measurement support; NULL = off):
     * device, int64, 8 words per outer iteration for the first
     * phase_trace_outer outer iterations, device wall clock (100 MHz ticks)
     * when, in outer iteration k, [8k+0] workgroup 0 starts the first phase,
     * [8k+1] workgroup 0 finishes it (its recurrence), [8k+2] the first
     * Gram workgroup and [8k+6] the last workgroup finish it, [8k+3]
     * workgroup 0 leaves the following barrier, [8k+4] finishes its update
     * slices, [8k+5] leaves the next barrier, [8k+7] the last workgroup
     * finishes its second-phase work. Words of phases a variant lacks stay
     * untouched. */
    int64_t *phase_trace;
    int64_t phase_trace_outer;
    /* CSR lambda path (casgd_fit_path): workgroups that share the
     * recurrence of one group of four lanes, splitting the rows of every
     * block; a power of two dividing b (0 = automatic). */
    int32_t rec_split;
    /* CASGD_LOSS_* (0 = logistic). */
    int32_t loss;
    /* End-to-end low-precision baseline (the paper's all-BF16 and all-FP16
     * recipes, Table 3 columns I and H; dense X only): 0 = off, 1 = BF16
     * (X stored in BF16), 2 = FP16 (X stored in FP16). Every slot's output is
     * rounded to the format, round to nearest even: G, r, the correction sum
     * a_j, z_j = fl(beta^j r_j + alpha a_j), delta_j, c_j, the gradient
     * g = Y^T c and x <- fl(beta^s x + alpha g); sums inside a kernel
     * accumulate in FP32 (CDNA has no FP16-accumulate matrix instruction, so
     * the FP16 recipe's accumulate-in-FP16 slots are not emulated). The
     * corrections run in FP32 (recur_prec 64 is rejected). */
    int32_t e2e;
    /* Gram work units (0 = automatic): 64 = 64 x 64 (or 32 x 64) tiles whose
     * four waves split K and read their operands directly; 128 = 128 x 128
     * tiles with both row panels staged through LDS (more reuse per byte,
     * fewer and larger units). Automatic: 128 when there are at least half
     * as many such tiles as compute units (as many for FP32 storage; the
     * group's workgroups in a batched launch). Results of the two agree to
     * rounding. */
    int32_t gram_tile;
} casgd_opts;

const char *casgd_status_string(casgd_status st);
/* Message of the last failing call on this thread ("" if none). */
const char *casgd_last_error(void);
/* Library version as 10000*major + 100*minor + patch. */
int32_t casgd_version(void);

/* ------------------------------------------------------------ one problem */

/* Workspace bytes for casgd_step / casgd_fit on X with these b, s. */
casgd_status casgd_workspace_size(const casgd_matrix *X, int32_t b, int32_t s,
                                  size_t *bytes);

/* Clear the device flags in a workspace (non-finite, timeout). Enqueued. */
casgd_status casgd_reset(void *ws, size_t ws_bytes, void *stream);

/*
 * One outer iteration (Algorithm 1 with L2 decay) at index `outer_iter`,
 * updating x (device, FP32, n) in place. y (device, FP32, m) holds +-1 labels.
 * eta > 0, lambda >= 0, b >= 1, s >= 1, s*b <= 4096. Stateless: the sample
 * set comes from (seed, outer_iter), so a sequence of calls with increasing
 * outer_iter equals one casgd_fit.
 */
casgd_status casgd_step(const casgd_matrix *X, const float *y, float *x, double eta,
                        double lambda, int32_t b, int32_t s, uint64_t seed,
                        uint64_t outer_iter, const casgd_opts *opts, void *ws,
                        size_t ws_bytes, void *stream);

/* Outer iterations outer_begin .. outer_begin + n_outer - 1. */
casgd_status casgd_fit(const casgd_matrix *X, const float *y, float *x, double eta,
                       double lambda, int32_t b, int32_t s, uint64_t seed,
                       uint64_t outer_begin, int64_t n_outer, const casgd_opts *opts,
                       void *ws, size_t ws_bytes, void *stream);

/*
 * casgd_fit without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, serving loops, harnesses that
 * forbid hipMalloc). Dense X only. The workspace lives in a static device
 * array of 64 MiB that the library holds on every device it runs on until
 * the process ends; problems whose casgd_workspace_size exceeds it are
 * rejected with CASGD_EUNSUPPORTED. No device memory is allocated or freed.
 * The array is shared by every call on a device and keeps the last call's
 * contents: each call clears what must start at zero, and calls that overlap
 * on one device (other streams, other threads) race and give undefined
 * results. status_out (device, one int32, or NULL) receives, in stream order
 * after the fit, CASGD_OK, CASGD_ENONFINITE or CASGD_ETIMEOUT (the checks
 * casgd_check makes on a workspace). Other arguments as for casgd_fit.
 */
casgd_status casgd_fit_noalloc(const casgd_matrix *X, const float *y, float *x, double eta,
                               double lambda, int32_t b, int32_t s, uint64_t seed,
                               uint64_t outer_begin, int64_t n_outer, const casgd_opts *opts,
                               int32_t *status_out, void *stream);

/* Reports the device flags of a workspace after synchronising `stream`:
 * CASGD_OK, CASGD_ENONFINITE, CASGD_ETIMEOUT, or CASGD_EUNSUPPORTED when a
 * sparse tail bucket overflowed. */
casgd_status casgd_check(const void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------- CSR X and lambda lanes */

/*
 * A CSR X is split once per (X, b, s) into dense "head" columns (the most
 * frequent ones, at most 512, expected to occur at least once per outer block)
 * and sparse "tail" columns. The head panel's Gram runs on MFMA; tail
 * intersections are accumulated per G row in a fixed order. Tail columns may
 * occur at most 64 times in one outer block of sampled rows; more raises a
 * device flag reported by casgd_check as CASGD_EUNSUPPORTED.
 */

/* Workspace bytes for a CSR X with these b, s and up to `lanes` lanes (a
 * dense X is not supported here). Reads row_ptr (synchronous). b must be a
 * multiple of 4. */
casgd_status casgd_path_workspace_size(const casgd_matrix *X, int32_t b, int32_t s,
                                       int32_t lanes, size_t *bytes);

/* Prepare a workspace for a CSR X: column frequencies, head/tail split,
 * cleared buckets. Synchronous. Required once per (X, b, s, workspace) before
 * casgd_fit / casgd_step / casgd_fit_path on that CSR X; `lanes` is the largest
 * lane count that will be used. Its cost is not part of any iteration. The
 * decisions (X's pointers and shape, b, s, lanes, the head split) are stored
 * in the workspace itself; the library keeps no host state. A CSR fit reads
 * that record back with a small synchronous device-to-host copy before it
 * enqueues its launch. */
casgd_status casgd_sparse_prepare(const casgd_matrix *X, int32_t b, int32_t s, int32_t lanes,
                                  void *ws, size_t ws_bytes, void *stream);

/*
 * Regularisation path: L lanes (1 <= L <= 64) with strengths lambdas (host,
 * L doubles, >= 0) share the sampled rows, the gathered block and the Gram
 * matrix of every outer iteration; each lane runs its own residual
 * corrections and update (beta_l = 1 - eta*lambda_l). x_lanes (device, FP32,
 * n x L, lane fastest) is updated in place; lane l equals a casgd_fit with
 * lambda_l on the same seed. CSR X only. One fused launch.
 */
casgd_status casgd_fit_path(const casgd_matrix *X, const float *y, float *x_lanes,
                            const double *lambdas, int32_t L, double eta, int32_t b, int32_t s,
                            uint64_t seed, uint64_t outer_begin, int64_t n_outer,
                            const casgd_opts *opts, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------ many problems */

/* One problem of a batched launch. X dense (all problems of a batch share
 * one storage dtype); the other fields as for casgd_fit; ws/ws_bytes is this
 * problem's own workspace (casgd_workspace_size). groups = workgroups given to
 * this problem (0: chosen by the library from a cost model); variant and
 * recur_prec as casgd_opts.fused_variant / recur_prec (0 = automatic). */
typedef struct {
    casgd_matrix X;
    const float *y;
    float *x;
    double eta, lambda;
    int32_t b, s;
    uint64_t seed;
    uint64_t outer_begin;
    int64_t n_outer;
    void *ws;
    size_t ws_bytes;
    int32_t groups;
    int32_t variant;
    int32_t recur_prec;
    int32_t loss;        /* CASGD_LOSS_* */
    /* snapshots of this problem, as casgd_opts.snapshot_every / x_history /
     * t_history (0 / NULL = none); the device clock is this problem's own */
    int64_t snapshot_every;
    float *x_history;
    int64_t *t_history;
    int32_t gram_tile;   /* as casgd_opts.gram_tile (0 = automatic for this problem's group) */
    int32_t reserved;
} casgd_problem;

/* Bytes of the device table workspace of a batch of `count` problems. */
size_t casgd_batch_table_size(int32_t count);

/*
 * Fit `count` independent dense problems (probs: host array) in one
 * cooperative launch: each problem runs its whole fit (all of its outer
 * iterations, as casgd_fit would) on its own group of workgroups with its own
 * grid barrier, so short and long problems proceed concurrently. Problems
 * whose automatic form is fused variant 3 keep it when every problem's
 * recurrence group fits on the device at once; otherwise those with the
 * smallest modelled gain fall back to variant 2. On success the workgroups
 * and the fused variant each problem runs with are written back to its
 * `groups` and `variant` fields. The problem
 * table is uploaded to `table` (device, casgd_batch_table_size bytes) with a
 * synchronous copy before the launch. spin_limit as in casgd_opts (0 =
 * default). Results equal casgd_fit per problem for the same variant and
 * Gram unit kind (gram_tile); the automatic kind may differ between a
 * problem's group and the whole device, and the two kinds agree to rounding.
 */
casgd_status casgd_fit_batch(casgd_problem *probs, int32_t count, int64_t spin_limit,
                             void *table, size_t table_bytes, void *stream);

/* ------------------------------------------------- pieces of the iteration */

/* Sample rows (Algorithm 1, first step): out[q] = row of sample t0+q. */
casgd_status casgd_sample_indices(uint64_t seed, uint64_t t0, int64_t count, int64_t m,
                                  int64_t *out, void *stream);

/*
 * Margins and Gram of outer iteration `outer_iter` (Algorithm 1, margin and
 * Gram steps): r (device, FP32, s*b) = Y x and G (device, FP32, s*b x s*b,
 * row-major) with the strict block-lower entries G[t][u] = Y_t . Y_u,
 * block(u) < block(t), written; other entries are left untouched. x and r
 * may both be NULL to compute the Gram alone. opts (may be NULL): gram_tile
 * selects the Gram unit kind as for a fit (automatic: 128 x 128 tiles when
 * there are at least as many as compute units). With a workspace of
 * casgd_gram_workspace_size bytes, 128 x 128 tiles are split along K over
 * several workgroups when the device holds more workgroups than there are
 * tiles (or than the tiles left after whole rounds), for rows of 8 KB or
 * more: a cooperative launch; the pieces' sums are added in a fixed order,
 * so the result is reproducible. The automatic kind is then the split
 * 128 x 128 tiles for rows of 16 KB or more. With casgd_workspace_size
 * bytes no tile is split.
 */
casgd_status casgd_gram_workspace_size(const casgd_matrix *X, int32_t b, int32_t s,
                                       size_t *bytes);
/* casgd_gram_workspace_size: workspace bytes of casgd_gram_margin (and of
 * stream-ordered fits, exec_mode 2) that include the exchange region of the
 * K-split Gram: casgd_workspace_size plus, when the split applies to this
 * shape, an epoch line and one 128 x 128 slot of 64-bit words per piece. Each
 * launch tags its words with a new epoch; the library clears the region when
 * its marker word is not set (first use, or a workspace that held other data),
 * which costs one extra pass over it. Dense X only. */
casgd_status casgd_gram_margin(const casgd_matrix *X, const float *x, int32_t b,
                               int32_t s, uint64_t seed, uint64_t outer_iter, float *G,
                               float *r, const casgd_opts *opts, void *ws, size_t ws_bytes,
                               void *stream);

/*
 * The s residual corrections (Algorithm 1, inner loop, with decay) from
 * device inputs G (FP32 s*b x s*b row-major, strict block-lower part read),
 * r (FP32 s*b) and labels yI (FP32 s*b); writes c (device, FP32, s*b) with
 * c_t = beta^(s-1-j) delta_t for t in block j, and delta (device, FP32, s*b)
 * if not NULL. prec: 0 auto, 32, 64 as casgd_opts.recur_prec; loss:
 * CASGD_LOSS_*. form selects the execution form the fits use:
 *   0 = automatic (2 when b is 16, 32, 64 or 128 and s > 1, else 1),
 *   1 = one workgroup streams the whole strict block-lower part,
 *   2 = a chain workgroup plus s - 3 helper workgroups (s - 2 for b = 128)
 *       that add the older column blocks and exchange tagged words (the form
 *       of the fused fit from s = 4 on); b must be 16, 32, 64 or 128.
 * ws (device, 256-byte aligned, casgd_recurrence_workspace_size bytes) holds
 * the exchange words and device flags; it may be NULL for form 1. Flags are
 * reported by casgd_check(ws) as for a fit.
 */
size_t casgd_recurrence_workspace_size(int32_t b, int32_t s);
casgd_status casgd_recurrence(const float *G, const float *r, const float *yI, int32_t b,
                              int32_t s, double eta, double lambda, int32_t prec, int32_t loss,
                              int32_t form, float *c, float *delta, void *ws, size_t ws_bytes,
                              void *stream);

/* x <- beta^s x + (eta/b) Y^T c for outer iteration `outer_iter` (Algorithm 1,
 * gradient and update steps, fused). c: device FP32 s*b (row scales are
 * applied by the library). ws as for casgd_step. */
casgd_status casgd_update(const casgd_matrix *X, float *x, const float *c, int32_t b,
                          int32_t s, uint64_t seed, uint64_t outer_iter, double eta,
                          double lambda, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------ precision selection */

/*
 * Thm. 5.1 (mixed-precision local error of one outer iteration) as a
 * run-time precision selector. The theorem bounds the forward error of one
 * outer iteration by nine additive terms E_slot = coef_slot * u_slot, one per
 * precision slot (storage of X u_A, margin GEMV u_r, Gram GEMM u_G, inner
 * corrections u_c, residual nonlinearity u_sigma, gradient GEMV u_g, weights
 * u_x, and the two all-reduce slots, which vanish on one device), plus a
 * remainder at most C_loc * Omega * sum E (C_loc = 2), valid while
 * Omega <= 1/2. The coefficients depend on the sampled rows Y, x and the
 * exact residual history d through ||Y||_2, K_s = ||(I - L_sigma alpha
 * |G_L|)^-1||_2, ||H_L||_2 and the source quantities T_g, T_r, T_G, T_c.
 * Constants: L_sigma = 1/4 (logistic), 1 (linear), exp(max z) over the block
 * (Poisson); C_delta = 8; D_delta = 1 (logistic) or max |d| (linear,
 * Poisson). Slots of this library: u_r = u_G = 2 u_A + gamma_n(u32) for
 * low-precision storage (FP32 accumulation; gamma_n(u32) for FP32 storage),
 * u_g = 2 u_A + gamma_sb(u32), u_sigma = u_c, u_x = u32. Nominal unit
 * roundoffs: FP8-E4M3 2^-4, BF16 2^-8, FP16 2^-11, FP32 storage of an FP32
 * master copy 0; corrections FP32 2^-24 or FP64 2^-53.
 */
enum { CASGD_SLOT_A = 0, CASGD_SLOT_R, CASGD_SLOT_G, CASGD_SLOT_C, CASGD_SLOT_SIGMA,
       CASGD_SLOT_GRAD, CASGD_SLOT_X, CASGD_SLOTS };

typedef struct {
    int32_t dtype;        /* storage format of X (CASGD_F32 .. CASGD_FP8E4M3) */
    int32_t recur_prec;   /* 32 or 64 (slot u_c) */
    int32_t valid;        /* Omega <= 1/2 and (s-1) b u_c < 1 */
    int32_t reserved;
    double u[CASGD_SLOTS]; /* unit roundoff or Higham factor of each slot */
    double E[CASGD_SLOTS]; /* the leading terms E_slot = coef_slot * u_slot */
    double sum, Omega, bound, rel_bound;  /* bound = (1 + 2 Omega) sum; rel_bound = bound / ||x^(s)|| */
} casgd_precision_candidate;

typedef struct {
    double alpha, norm_Y, K_s, norm_HL, T_g, T_r, T_G, T_c, norm_x_next, L_sigma, D_delta;
    double coef[CASGD_SLOTS];
    int32_t ncand;        /* candidates evaluated (storage formats x {FP32, FP64} corrections) */
    int32_t chosen;       /* index into cand */
    int32_t dtype;        /* the chosen storage format */
    int32_t recur_prec;   /* the chosen correction precision (casgd_opts.recur_prec) */
    int32_t meets_budget; /* 0: no valid candidate met rel_budget; the most accurate valid one is chosen */
    int32_t reserved;
    casgd_precision_candidate cand[8];
} casgd_precision_report;

/* Workspace bytes of casgd_select_precision (X dense FP32). */
size_t casgd_precision_workspace_size(const casgd_matrix *X, int32_t b, int32_t s);

/*
 * Evaluate Thm. 5.1 on outer iteration `outer_iter` of (X, y, seed) from x
 * (all device; X the FP32 master copy) with step eta (the theorem's setting
 * has no L2 term, so lambda = 0) and the given loss, and choose the cheapest
 * assignment -- storage FP8-E4M3, BF16, FP16, FP32 in that order (those set in
 * the bit mask `allowed`, bit = dtype; 0 = all), corrections FP32 before
 * FP64 -- whose relative bound bound / ||x^(s)|| is at most rel_budget and
 * which is valid. FP16 is skipped when a sampled entry is outside its range.
 * The gather, Gram, margins and exact residual history run on the GPU (ws,
 * casgd_precision_workspace_size bytes); the norms and the selection run on
 * the host in FP64. Synchronous (a planning call, not part of any fit).
 * Fills out (host) with every candidate's terms and the choice.
 */
casgd_status casgd_select_precision(const casgd_matrix *X, const float *y, const float *x,
                                    double eta, int32_t b, int32_t s, uint64_t seed,
                                    uint64_t outer_iter, int32_t loss, double rel_budget,
                                    uint32_t allowed, casgd_precision_report *out, void *ws,
                                    size_t ws_bytes, void *stream);

/* ------------------------------------------------------- storage formats */

/*
 * Convert an FP32 matrix (device, m x ld_src) to storage `dtype`
 * (Table 1, storage precision u_A): dst (device, m x ld_dst elements of dtype).
 * BF16 and F16 round to nearest even; FP8-E4M3 uses per-row scales
 * scale_i = amax_i / 448 (FP32), stores e4m3(x * (448 / amax_i)) rounded to
 * nearest even with saturation at +-448, and writes row_scale (device, m);
 * an all-zero row gets scale 1. BF16, F16 and F32 are not scaled: row_scale
 * may be NULL, and if it is not it is filled with 1. Columns n..ld_dst-1 of
 * dst are set to zero.
 */
casgd_status casgd_quantize(const float *src, int64_t m, int64_t n, int64_t ld_src,
                            int32_t dtype, void *dst, int64_t ld_dst, float *row_scale,
                            void *stream);

/* Same as casgd_quantize of the column-scaled matrix X diag(col_scale)
 * (col_scale: device, FP32, n), each product rounded to FP32 first. Used to
 * apply a diagonal preconditioner d as X diag(sqrt(d)). */
casgd_status casgd_quantize_scaled(const float *src, int64_t m, int64_t n, int64_t ld_src,
                                   const float *col_scale, int32_t dtype, void *dst,
                                   int64_t ld_dst, float *row_scale, void *stream);

/* ------------------------------------------------ learned preconditioner */

/*
 * A 4 -> 64 -> 2 MLP maps per-column statistics of X to a per-feature step
 * scale and a step size (not part of the paper). Parameters (device, FP32,
 * 450 floats): W1[64][4], b1[64], W2[2][64], b2[2]; for input row f:
 * pre = W1 f + b1, h = relu(pre), out = W2 h + b2. out[0] predicts log d_k,
 * out[1] is averaged over a problem's columns into its log step size. Every
 * reduction runs in a fixed order.
 */
#define CASGD_MLP_PARAMS 450

/* feats (device, N x 4) = (log(1 + |stats|) - norm[0:4]) / norm[4:8];
 * stats (device, N x 4) as written by casgd_colstats; norm (device, 8). */
casgd_status casgd_mlp_features(const float *stats, int64_t N, const float *norm, float *feats,
                                void *stream);

/* Feature normalisation over N training rows (device): norm[c] = mean_k
 * log(1 + |stats[k][c]|), norm[4 + c] = max(sample standard deviation, 1e-6),
 * c = 0..3, accumulated in FP64 in a fixed order. N >= 1. */
casgd_status casgd_mlp_feature_norm(const float *stats, int64_t N, float *norm, void *stream);

/* out (device, N x 2); pre (device, N x 64, the hidden pre-activations kept
 * for the backward pass) may be NULL. */
casgd_status casgd_mlp_forward(const float *params, const float *feats, int64_t N, float *out,
                               float *pre, void *stream);

/* Applies a forward output (device, N x 2) for one problem of N columns: the
 * step scale d_k = exp(clamp(out[k][0] - mean_j out[j][0], -20, 20)) is
 * returned as the column scale q_k = sqrt(d_k) (device, N), and
 * eta[0] = exp(mean_j out[j][1]) (device, 1 float). N >= 1. The scaled problem
 * X~ = X diag(q) is built with casgd_quantize_scaled; a fit of X~ gives x~ and
 * x = q * x~ (X~ x~ = X x, so losses of x~ on X~ equal those of x on X). */
casgd_status casgd_mlp_apply(const float *out, int64_t N, float *q, float *eta, void *stream);

/* Workspace of casgd_mlp_loss_grad / casgd_mlp_backward for N rows, P problems. */
size_t casgd_mlp_workspace_size(int64_t N, int32_t P);

/*
 * Training loss over P problems whose rows are seg_off[p] .. seg_off[p+1]-1
 * (seg_off: device, int64, P+1):
 *   L = mean_rows (out0 - t_d)^2 + w_eta * mean_p (mean_{rows of p} out1 - t_eta[p])^2
 * loss (device, FP64, 1) and g_out = dL/dout (device, N x 2).
 */
casgd_status casgd_mlp_loss_grad(const float *out, const int64_t *seg_off, int32_t P, int64_t N,
                                 const float *t_d, const float *t_eta, float w_eta, double *loss,
                                 float *g_out, void *ws, size_t ws_bytes, void *stream);

/* grad (device, 450) = dL/dparams given g_out, from feats and pre of the forward. */
casgd_status casgd_mlp_backward(const float *params, const float *feats, const float *pre,
                                const float *g_out, int64_t N, int32_t P, float *grad, void *ws,
                                size_t ws_bytes, void *stream);

/* One Adam step (Kingma and Ba, 2015) with bias correction, t >= 1:
 * m1 = b1 m1 + (1-b1) g; m2 = b2 m2 + (1-b2) g^2;
 * params -= lr (m1/(1-b1^t)) / (sqrt(m2/(1-b2^t)) + eps). All device arrays. */
casgd_status casgd_adam_step(float *params, const float *grad, float *m1, float *m2,
                             int32_t count, int64_t t, float lr, float beta1, float beta2,
                             float eps, void *stream);

/* Diagonal of the Hessian of the mean logistic loss plus lambda at x:
 * hdiag_k = m^-1 sum_i s(z_i)(1 - s(z_i)) X_ik^2 + lambda, z_i = X_i . x
 * (device, FP32, n). Dense X. ws (device) of casgd_hess_diag_workspace_size. */
size_t casgd_hess_diag_workspace_size(const casgd_matrix *X);
casgd_status casgd_hess_diag(const casgd_matrix *X, const float *x, double lambda, float *hdiag,
                             void *ws, size_t ws_bytes, void *stream);

/* Training target of the per-feature scale from a Hessian diagonal h (device,
 * n, positive): t_d = -log h_k + mean_j log h_j (device, n), the log of a
 * Jacobi preconditioner normalised to unit geometric mean, and, when q is not
 * NULL, the column scale q = exp(t_d / 2) (device, n). n >= 1. */
casgd_status casgd_jacobi_target(const float *hdiag, int64_t n, float *t_d, float *q,
                                 void *stream);

/* --------------------------------------------------- measurement support */

/*
 * Mean logistic loss m^-1 sum_i log(1 + exp(-y_i a_i^T x)) (Sec. 2.1) for
 * `count` weight vectors x_k = xs + k*x_stride (device, FP32, n each);
 * out (device, FP64, count). Dense X (any dtype, row scales applied) or CSR.
 * Margins accumulate in FP32, the loss terms and their sum in FP64, in a fixed
 * order. ws (device) must hold casgd_logloss_workspace_size() bytes.
 */
size_t casgd_logloss_workspace_size(int64_t count);
casgd_status casgd_logloss(const casgd_matrix *X, const float *y, const float *xs,
                           int64_t count, int64_t x_stride, double *out, void *ws,
                           size_t ws_bytes, void *stream);

/* Mean loss m^-1 sum_i L(a_i^T x, y_i) of any of the three losses of Sec. 2.1
 * (loss = CASGD_LOSS_*); otherwise as casgd_logloss, with the same workspace
 * size. The Poisson terms may overflow to +Inf for huge margins. */
casgd_status casgd_loss(const casgd_matrix *X, const float *y, const float *xs, int64_t count,
                        int64_t x_stride, int32_t loss, double *out, void *ws, size_t ws_bytes,
                        void *stream);

/*
 * Per-column statistics (device, FP32, n x 4 row-major): mean, population
 * variance, fraction of nonzeros and max |value| over the m rows, with row
 * scales applied. Dense X (any dtype) or CSR. ws (device) must hold
 * casgd_colstats_workspace_size(X) bytes.
 */
size_t casgd_colstats_workspace_size(const casgd_matrix *X);
casgd_status casgd_colstats(const casgd_matrix *X, float *stats, void *ws, size_t ws_bytes,
                            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CASGD_H */
