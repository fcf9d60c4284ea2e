/*
 * snect.h -- C ABI of the MI355X (gfx950) SNeCT engine.
 *
 * SNeCT (Choi & Sael, arXiv:1711.08095) fits a Tucker model (Eq. 2)
 *     x(i,j,k) ~ sum_{a,b,c} G[a,b,c] A[i,a] B[j,b] C[k,c]
 * to the observed cells of a sparse patient x gene x platform tensor, with an
 * L2 penalty (Eq. 3) and a gene-network Laplacian penalty on B (Eq. 4), by
 * stochastic gradient descent over the nonzeros (Algorithm 1, gradients of
 * Eq. 5).  This library runs that SGD on one GPU with a deterministic
 * stratified schedule in place of the paper's lock-free random order:
 *
 *   plan  seeded permutations split patients and genes into P blocks each;
 *         block (p,q) lists its nonzeros in ascending (k, i, j) and cuts them
 *         into tiles of at most T entries that never straddle a change of k;
 *   epoch (a) network step: B <- B - (lr lambda_g / n_sub) L B, n_sub times,
 *             n_sub = max(1, ceil(2 lr lambda_g d_max)), L = D - W;
 *         (b) for each of P strata (seeded order), the blocks (p, (p+s) mod P)
 *             run concurrently; inside a block the tiles run in order and every
 *             nonzero of a tile reads the factor rows from before the tile:
 *               e = x - a_i . (H_k b_j),  H_k = G x3 c_k (frozen per stratum)
 *               a_i += lr * sum_t (e_t H_k b_j - lambda / n1[i] a_i)
 *               b_j += lr * sum_t (e_t H_k^T a_i - lambda / n2[j] b_j)
 *             then C and G take one step with the stratum's mean gradient,
 *             step lr * core_lr_scale;
 *         (c) f_opt and training RMSE at the end-of-epoch factors.
 *
 * Conventions
 *   - Indices are 0-based (the paper's are 1-based).  All matrices are
 *     row-major float32: A is I1 x J1, B is I2 x J2, C is I3 x J3, and G is
 *     J1 x J2 x J3 with flat index (a*J2 + b)*J3 + c.
 *   - Status codes: 0 on success, a negative SNECT_E_* value on failure.
 *     No exception or abort crosses this interface.  After a failure,
 *     snect_last_error() describes it.  Every input is validated before any
 *     device work starts.
 *   - Ownership: the caller owns every buffer it passes.  The library only
 *     borrows them for the duration of the call.  Memory the library
 *     allocates (the device-resident plan, scratch) belongs to the context
 *     or problem object and is released by the matching destroy call.
 *   - Streams: all device work is issued on the stream given to
 *     snect_create (NULL = the device's default stream).  Every call that
 *     returns host-visible results synchronises that stream before returning.
 *   - Threads: one context per host thread; contexts are independent.
 */
#ifndef SNECT_H
#define SNECT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SNECT_OK 0
#define SNECT_E_ARG -1         /* bad scalar argument or NULL pointer        */
#define SNECT_E_INDEX -2       /* a coordinate or edge endpoint out of range */
#define SNECT_E_DUPLICATE -3   /* the same (i,j,k) given twice               */
#define SNECT_E_RANK -4        /* core size outside what the kernels support */
#define SNECT_E_OOM -5         /* host or device allocation failed           */
#define SNECT_E_HIP -6         /* a HIP runtime call failed                  */
#define SNECT_E_DIVERGED -7    /* the epoch loss became non-finite           */
#define SNECT_E_BUSY -8        /* the serving pool has no free slot/memory   */
#define SNECT_E_UNSUPPORTED -9 /* valid input outside this build's limits   */

#define SNECT_PRECISION_FP32 0 /* FP32 contractions                          */
#define SNECT_PRECISION_BF16 1 /* BF16 MFMA contractions, FP32 masters       */

/* Limits of this build. */
#define SNECT_MAX_RANK 32      /* J1, J2, J3 <= 32                           */
#define SNECT_MAX_TILE 64      /* T <= 64: one tile is one wavefront         */

typedef struct snect_ctx snect_ctx;
typedef struct snect_problem snect_problem;

/* Sparse tensor X over its observed cells Omega_X (Section 2.2, Table 2).
 * Host memory.  nnz may be 0.  Coordinates must be distinct. */
typedef struct {
    int32_t I1, I2, I3;       /* patients, genes, platforms                 */
    int64_t nnz;              /* number of observed cells, < 2^31           */
    const int32_t *i, *j, *k; /* [nnz] 0-based coordinates                   */
    const float *x;           /* [nnz] values, finite                        */
} snect_tensor;

/* Gene network Y (Section 2.1.2, Eq. 4): undirected edges, each listed once
 * in either orientation; repeated pairs add their weights.  Host memory. */
typedef struct {
    int64_t E;                /* number of edges (may be 0)                  */
    const int32_t *u, *v;     /* [E] gene endpoints, u != v                  */
    const float *w;           /* [E] weights >= 0, or NULL for all ones      */
} snect_graph;

typedef struct {
    int32_t J1, J2, J3;       /* core size, 1..SNECT_MAX_RANK               */
    double lambda;            /* L2 weight (Eq. 3), >= 0                     */
    double lambda_g;          /* network weight (Eq. 4), >= 0                */
    double lr;                /* learning rate eta of Algorithm 1, > 0       */
    double core_lr_scale;     /* C and G step = lr * core_lr_scale, >= 0     */
    int32_t strata_P;         /* blocks per mode, 1 <= P <= min(I1, I2)      */
    int32_t tile_T;           /* tile size, 1 <= T <= SNECT_MAX_TILE         */
    int32_t precision;        /* SNECT_PRECISION_*                           */
    uint64_t seed;            /* plan seed (permutations, stratum orders)    */
} snect_params;

/* Factor set: device pointers (row-major float32, sizes as above). */
typedef struct {
    float *A, *B, *C, *G;
} snect_factors;

/* Per-problem figures, for reporting and roofline accounting. */
typedef struct {
    int64_t nnz, ntiles, edges_csr;
    int32_t P, T, rows1_max, rows2_max;
    int32_t bits_i, bits_j;   /* widths of the row fields of a packed record */
    int32_t n_sub;            /* network sub-steps per epoch                 */
    double d_max;             /* largest weighted gene degree                */
    int64_t device_bytes;     /* device memory held by the problem           */
    double plan_seconds;      /* host planning time                          */
    double upload_seconds;    /* host-to-device copy time                    */
} snect_info;

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t, or NULL for the default stream).  *ctx receives the
 * handle.  Errors: E_ARG, E_HIP. */
int snect_create(snect_ctx **ctx, int device, void *hip_stream);

/* Release a context.  All problems created on it must be destroyed first;
 * otherwise the call fails with E_BUSY and the context stays valid. */
int snect_destroy(snect_ctx *ctx);

/* Message for the last failure on this context ("" if none).  The string is
 * owned by the context and valid until its next call. */
const char *snect_last_error(const snect_ctx *ctx);

/* Validate the inputs, build the plan on the host (slice counts, seeded
 * permutations, block-sorted packed nonzeros, tiles, the symmetric CSR of
 * the network Laplacian) and upload it.  The tensor and graph arrays are
 * only read during the call.  Errors: E_ARG, E_INDEX, E_DUPLICATE, E_RANK,
 * E_UNSUPPORTED (a block's rows do not fit on chip), E_OOM, E_HIP. */
int snect_problem_create(snect_ctx *ctx, const snect_tensor *X, const snect_graph *Y,
                         const snect_params *params, snect_problem **prob);

/* Free a problem and its device memory. */
int snect_problem_destroy(snect_problem *prob);

/* Figures about a problem. */
int snect_problem_info(const snect_problem *prob, snect_info *info);

/* Run `epochs` epochs numbered start_epoch, start_epoch+1, ... (the epoch
 * number selects the stratum order, so a run split into pieces reproduces
 * one long run).  The factors in `f` (device pointers) are read as the
 * starting point and overwritten in place.  loss[e] and rmse[e] (host
 * arrays of length `epochs`, either may be NULL) receive f_opt and the
 * training RMSE after each epoch.  If an epoch's loss is not finite the call
 * stops, leaves the factors of the last finite epoch in `f` and returns
 * E_DIVERGED.  Errors: E_ARG, E_HIP, E_DIVERGED. */
int snect_train(snect_problem *prob, snect_factors *f, int32_t start_epoch, int32_t epochs,
                double *loss, double *rmse);

/* f_opt (Eq. 3 + lambda_g Eq. 4, L2 over the observed rows) and the RMSE of
 * the given factors, without changing them.  Errors: E_ARG, E_HIP. */
int snect_evaluate(snect_problem *prob, const snect_factors *f, double *loss, double *rmse);

/* One-shot form of Algorithm 1 (REQUIRE: X, Y, ranks, lambda, lambda_g,
 * eta; ENSURE: A, B, C, G): create the problem, set the starting factors in
 * `out` (device buffers), train `epochs` epochs from start_epoch, destroy
 * the problem.  loss and rmse are as in snect_train.
 *
 * init != NULL: the starting factors are copied from `init` (device
 * buffers; init and out may be the same).
 * init == NULL: Algorithm 1 starts from random factors.  This library draws
 * every entry of A, B, C and G (in that order, each row-major) i.i.d. from
 * N(0, sigma^2) with sigma = (mean of x^2 / (J1 J2 J3))^(1/8), so that the
 * model values start at the scale of the data (sigma = 1 when nnz = 0 or
 * every x is 0).  The normals come from the Box-Muller transform
 * (Box & Muller 1958) of pairs of uniforms (u1, u2) in (0, 1), each
 * u = (floor(r / 2^11) + 1/2) 2^-53 for a 64-bit draw r of the SplitMix64
 * stream 2^40 of params->seed (the same stream construction as the plan);
 * a pair gives sqrt(-2 ln u1) cos(2 pi u2), then sqrt(-2 ln u1)
 * sin(2 pi u2).  The draw runs on the host in double precision and is
 * rounded once to float.  The same seed gives the same factors.
 * Errors: those of snect_problem_create and snect_train. */
int snect_decompose(snect_ctx *ctx, const snect_tensor *X, const snect_graph *Y,
                    const snect_params *params, const snect_factors *init, snect_factors *out,
                    int32_t start_epoch, int32_t epochs, double *loss, double *rmse);

/* Algorithm 1's last step: for n = 1, 2, 3, U(n) = Q R with R upper
 * triangular and a positive diagonal, U(n) <- Q and G <- G x_n R, so the
 * model values are unchanged and every factor gets orthonormal columns.
 * Device factors in place (A is I1 x J1 and so on); the arithmetic is FP64
 * (CholeskyQR2: Gram matrix, Cholesky, triangular solve, twice).  Needs
 * J_n <= I_n.  Errors: E_ARG (also a rank-deficient factor), E_RANK, E_OOM,
 * E_HIP.  Allocates and frees its own scratch; synchronises the stream. */
int snect_orthonormalize(snect_ctx *ctx, int32_t I1, int32_t I2, int32_t I3, int32_t J1, int32_t J2, int32_t J3,
                         snect_factors *f);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * orthonormalisation as snect_orthonormalize, with the same kernels and
 * bit-identical results, but no allocation of any kind.  Its FP64 scratch
 * (256 partial 32 x 32 Gram matrices, the triangular factors, a 32^3 core
 * and the status words: 2,392,320 bytes) is a fixed array in device memory
 * that every device the library runs on holds until the process ends; its
 * address is looked up once per device by the first snect_create on it.
 * Limit: J1, J2, J3 <= 32 (the capacity of that array; larger ranks give
 * E_RANK), J_n <= I_n.  All calls on one device share the array, so calls
 * that overlap on a device (two streams or two contexts at once) race and
 * must be serialised by the caller; each call leaves its last mode's data in
 * the array and clears its status words before use.  Synchronises the
 * stream.  Errors: E_ARG (also a rank-deficient factor), E_RANK, E_HIP. */
int snect_orthonormalize_noalloc(snect_ctx *ctx, int32_t I1, int32_t I2, int32_t I3, int32_t J1, int32_t J2,
                                 int32_t J3, snect_factors *f);

/* The plan's seeded draws, for cross-checks: perm1[I1] and perm2[I2] (the
 * row at each position of the patient / gene permutation; block of position
 * r is floor(r P / I)), strata[P] (stratum order of `epoch`).  Any pointer
 * may be NULL.  Host memory. */
int snect_plan_export(const snect_problem *prob, int32_t epoch, int32_t *perm1, int32_t *perm2,
                      int32_t *strata);

/* The plan exactly as the stratum kernels read it, copied back from the
 * device (the random order of Algorithm 1 replaced by the seeded plan), for
 * bit-exact cross-checks of the index work.  Host buffers, any may be NULL:
 *   word[nnz], x[nnz]  the packed nonzero records in plan order: block
 *                      (p, q) = (b / P, b % P) for b = 0 .. P*P-1 in turn,
 *                      inside a block ascending (k, i, j).  word holds, from
 *                      bit 0 up, the patient row inside its block (bits_i
 *                      bits; the row's position in perm1 minus
 *                      ceil(p I1 / P)), the gene row inside its block
 *                      (bits_j bits, likewise with perm2 and q) and 6 bits of
 *                      slot: the record's rank in its tile when the tile is
 *                      stably ordered by that gene row.  x is the value.
 *   tile_off[ntiles+1] first record of each tile (and nnz at the end);
 *   tile_k[ntiles]     platform of each tile (a tile never spans two);
 *   blk_tile[P*P+1]    first tile of each block (and ntiles at the end).
 * bits_i, bits_j and ntiles are in snect_info.  Synchronises the stream.
 * Errors: E_ARG, E_HIP. */
int snect_plan_layout(const snect_problem *prob, uint32_t *word, float *x, int32_t *tile_off, int32_t *tile_k,
                      int32_t *blk_tile);

/* Device time of the last snect_train call (milliseconds, summed over its
 * epochs), measured with HIP events on the library stream: [0] network step,
 * [1] strata (all stratum work), [2] loss, [3] the stratum kernels alone
 * (per-launch events, only with per-launch timing on) and [4] the number of
 * stratum-kernel launches timed for [3]. */
int snect_last_timing(const snect_problem *prob, double *ms5);

#define SNECT_PATH_AUTO 0       /* persistent kernel when it can be resident */
#define SNECT_PATH_PERSISTENT 1 /* one cooperative launch per epoch           */
#define SNECT_PATH_MULTI 2      /* one launch per stratum + a core-step launch */

/* Execution choices; they never change results: every sum of the stratum
 * kernels is taken in an order fixed by the problem alone, so both drivers
 * and every record-chunk size give bit-identical factors and losses.  per_launch_timing records a pair of HIP events around
 * every stratum-kernel launch (no extra host synchronisation); path selects
 * the stratum driver; waves and rec_cap shape the stratum workgroups;
 * wait_limit bounds the persistent kernel's waits (the factors are undefined
 * after an epoch that failed that way).
 * SNECT_PATH_PERSISTENT fails with E_UNSUPPORTED at snect_train if the P
 * workgroups cannot all be resident.  Errors: E_ARG, E_HIP. */
typedef struct {
    int32_t per_launch_timing;
    int32_t path;
    int32_t waves;   /* wavefronts per stratum workgroup: 0 or 8 (the only size) */
    int32_t rec_cap; /* nonzero records staged in LDS per chunk: 0 (the largest
                        that fits) or a power of two from 64 up to that */
    int32_t wait_limit; /* poll rounds after which a workgroup of the persistent
                           kernel stops waiting for another one and the epoch
                           fails with E_HIP: 0 (the default, 2^25 rounds, far
                           longer than any stratum) or a positive count; a
                           small one forces that failure path (tests) */
} snect_exec;

int snect_set_exec(snect_problem *prob, const snect_exec *exec);

/* Sweep: trains n independent problems of one context together (the
 * rank and lambda_g grids of Section 3.1), each following exactly the
 * schedule snect_train would run for it, so its factors and losses are
 * bit-identical to snect_train's (Algorithm 1 per problem, as read in
 * snect_train).  fs[i] are problem i's factors (device, caller owned);
 * loss and rmse (host, may be NULL) receive n * epochs values,
 * problem-major.  The problems must share a precision.
 *
 * In this build every problem runs on a stream of its own, created for the
 * call, with the multi-launch driver (a block-step launch and a core-step
 * launch per stratum, the code of its own core size, workgroups of eight
 * wavefronts, the record chunk snect_sweep_autotune chose up to the
 * problem's own), the problems' epochs queued side by side so that they
 * run concurrently; the streams start after the work already queued on the
 * context's stream, and the call waits for them before it returns.  The
 * single cooperative launch per epoch for all problems (problem i on P_i
 * workgroups with its own exchange words) is switched off until the cause of
 * a GPU memory fault seen in its kernel is established.
 *
 * Errors: E_ARG, E_OOM, E_HIP, E_DIVERGED (the message names the problem;
 * that problem's factors are rolled back to the start of the failing
 * epoch, the others end after it; later loss entries are undefined). */
int snect_sweep_train(snect_ctx *ctx, int32_t n, snect_problem *const *probs, snect_factors *fs,
                      int32_t start_epoch, int32_t epochs, double *loss, double *rmse);

/* Execution autotuner.  Times `trials` epochs (the best one counts) of
 * every execution choice -- both stratum drivers (the persistent one where
 * its workgroups can be resident), record chunks from
 * the largest that fits down to 256 in powers of two -- on scratch copies
 * of the factors f (device; f itself is not changed), keeps the fastest on
 * the problem (as snect_set_exec would) and reports it in *best (may be
 * NULL) with its epoch time in ms (*best_ms, may be NULL).  Results never
 * depend on the choice.  Allocates device scratch for the copies.
 * Errors: E_ARG, E_OOM, E_HIP, E_DIVERGED (f diverges in one epoch). */
int snect_autotune(snect_problem *prob, const snect_factors *f, int32_t trials, snect_exec *best,
                   double *best_ms);

/* Autotuner of a sweep: times `trials` sweep epochs on scratch
 * copies of fs for every problem's record chunk scaled by 1, 1/2 and 1/4
 * (not below 256) and keeps the fastest for later snect_sweep_train calls
 * on these problems; *best_ms (may be NULL) receives its epoch time.
 * Errors: those of snect_sweep_train, E_OOM. */
int snect_sweep_autotune(snect_ctx *ctx, int32_t n, snect_problem *const *probs, const snect_factors *fs,
                         int32_t trials, double *best_ms);

/* The stratum driver the next snect_train call will use (SNECT_PATH_*). */
int snect_exec_path(const snect_problem *prob);

/* ------------------------------------------------------------------------
 * Fold-in and top-k search for new patients (Section 3.2.1, Eq. 6) with
 * continuous batching.  With B, C, G fixed, a new patient's observed cells
 * (j_t, k_t, x_t) give rows w_t = G x2 b_{j_t} x3 c_{k_t}; the server finds
 *     u = argmin 1/2 |x - W u|^2 + lambda/2 |u|^2
 * (Eq. 6 with a ridge term): the rows w, Q = W^T W + lambda I and r = W^T x
 * in FP32 (fixed-order sums), pg_iters projected-gradient steps from u = 0
 * with step 1/|Q|_F in FP32, then one refinement u <- u + Q^{-1}(r - Q u) in
 * FP64 (residual, Cholesky factorisation of Q and the two triangular solves),
 * which gives the minimiser of the FP32-formed system.  It then returns the
 * topk rows of A with the largest cosine similarity to u (FP32; rows of zero
 * norm excluded, ties to the lower row index; missing entries are -1 with
 * score -inf).
 *
 * Requests are admitted while a slot (one HIP stream each) and room in the
 * device request pool (12 bytes per cell, 256-byte aligned) are free; each
 * runs on its own stream, so requests overlap on the device.  A request's
 * result does not depend on the others in flight.
 * ---------------------------------------------------------------------- */
typedef struct snect_server snect_server;

typedef struct {
    int32_t max_slots;   /* requests in flight at once, 1..64              */
    int64_t pool_bytes;  /* device memory for request cells (>= 4096)      */
    int32_t pg_iters;    /* projected-gradient steps before the refinement */
    int32_t topk;        /* neighbours returned, 1..64 (<= I1)             */
    double lambda;       /* ridge weight, >= 0                             */
} snect_server_config;

/* A, B, C, G: device factors (row-major FP32, A is I1 x J1, ...).  The
 * server precomputes the rows w for every (gene, platform) cell, the row
 * norms of A and a transposed copy of A before it returns, and reads the
 * factors no more: later changes to them are not seen by the server.
 * Errors: E_ARG, E_RANK, E_OOM, E_HIP. */
int snect_server_create(snect_ctx *ctx, int32_t I1, int32_t I2, int32_t I3, int32_t J1, int32_t J2, int32_t J3,
                        const snect_factors *f, const snect_server_config *cfg, snect_server **srv);

/* Waits for requests in flight and frees the server. */
int snect_server_destroy(snect_server *srv);

/* Admit one request: nnz cells j[], k[] (0-based gene and platform) and
 * values x[] (host memory, copied before the call returns).  *ticket
 * identifies it for snect_server_poll.  Errors: E_BUSY (no free slot or no
 * room in the pool now: try again after a completion), E_UNSUPPORTED (the
 * request needs more than the whole pool: 3 * 4 * nnz bytes, each array
 * rounded up to 256), E_INDEX, E_ARG (bad or non-finite input), E_OOM, E_HIP.  A failed submit changes
 * nothing. */
int snect_server_submit(snect_server *srv, int64_t nnz, const int32_t *j, const int32_t *k, const float *x,
                        int64_t *ticket);

/* 0 while the request runs; 1 when it is done, with u[J1], idx[topk] and
 * score[topk] filled (any may be NULL) and the ticket retired; E_ARG if
 * the fold-in system was not positive definite (lambda = 0 and too few
 * cells) or the ticket is unknown; E_HIP. */
int snect_server_poll(snect_server *srv, int64_t ticket, double *u, int32_t *idx, double *score);

/* Open-loop replay of a request stream in native code: request r arrives
 * arrival_s[r] seconds after the start (non-decreasing) and has the cells
 * offsets[r] .. offsets[r+1]-1 of j, k, x.  Requests are submitted as they
 * arrive and as slots and pool room free up, completions are polled, and
 * latency_s[r] = completion - arrival.  u [nreq*J1], idx and score
 * [nreq*topk] and status [nreq] (SNECT_OK or the request's error) may be
 * NULL.  *wall_s receives the total time.  If gpu_busy_s is not NULL, each
 * request's kernels are bracketed with timing events and *gpu_busy_s
 * receives the time during which at least one request's kernels ran (the
 * union of those windows; uploads and downloads not included).  Errors:
 * E_ARG, E_HIP (timing events); a request's own error goes to status. */
int snect_server_replay(snect_server *srv, int64_t nreq, const double *arrival_s, const int64_t *offsets,
                        const int32_t *j, const int32_t *k, const float *x, double *latency_s, double *u,
                        int32_t *idx, double *score, int32_t *status, double *wall_s, double *gpu_busy_s);

#ifdef __cplusplus
}
#endif
#endif /* SNECT_H */
