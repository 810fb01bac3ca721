/*
 * nomad.h -- C ABI of the MI355X NOMAD library (libnomad.so).
 *
 * NOMAD (Yun, Yu, Hsieh, Vishwanathan, Dhillon) fits A ~ W H^T on the observed entries
 * Omega of a sparse m x n rating matrix by stochastic gradient descent
 * (section 2.3, eqs. w_update / h_update) on the objective J(W,H) of eq. (obj_fcn).
 * The rows are split into p disjoint sets I_1..I_p with about the same number of
 * ratings each (section 3.1 and its footnote); worker q owns and alone updates w_i for
 * i in I_q.  Every item vector h_j is owned by exactly one worker at a time and moves
 * between workers ("nomadic" variables, section 3.1, Algorithm 1), so no two concurrent
 * updates touch the same parameter.  Here a worker is one workgroup of a persistent
 * kernel on one GPU (normally one per CU), the hybrid layout of section 3.4: its rows are
 * split again among its compute wavefronts, each item visits them in ascending order
 * through LDS, and a memory wavefront takes items over from other workers and hands
 * them on.
 *
 * Conventions for every entry point
 *   - Returns a nomad_status; nothing aborts or throws across the ABI.  On failure the
 *     message is available from nomad_last_error(ctx) (or nomad_last_error(NULL) for
 *     failures that leave no context, such as nomad_init).
 *   - Pointers named d_* are device pointers (HIP global memory on the current device);
 *     h_* pointers are host memory.  Arrays are dense, row-major, 0-based.
 *   - Input arrays are read during the call only and stay owned by the caller.  The
 *     context owns every allocation it makes; nomad_destroy frees them.
 *   - All device work is ordered on the HIP stream given to nomad_init (NULL = the
 *     default stream) and every entry point synchronises that stream before returning.
 *   - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef NOMAD_H
#define NOMAD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nomad_ctx nomad_ctx;

typedef enum {
    NOMAD_OK = 0,
    NOMAD_EINVAL = 1,   /* bad argument: sizes, k, index out of range, duplicate (i,j) */
    NOMAD_ENOMEM = 2,   /* device or host allocation failed */
    NOMAD_EDEVICE = 3,  /* a HIP call failed, or the workers cannot all be resident */
    NOMAD_ESTATE = 4,   /* call not valid in the context's state (e.g. NULL context) */
    NOMAD_ENOTIMPL = 5  /* an option combination the library does not provide */
} nomad_status;

/* Order in which items travel between workers.
 *   RING: fixed token-passing order.  Item j starts at worker g(j) (its uniformly random
 *     initial queue, Algorithm 1); in sub-step s of an epoch worker q processes the items
 *     with g(j) = (q+s) mod p in ascending j; items then pass from q to q-1.  Every
 *     rating is updated once per epoch and the result is one fixed serial order of
 *     updates, independent of timing.
 *   PERM: asynchronous (Algorithm 1 with the random-permutation circulation of section
 *     3.4).  Every worker has a lock-free inbound queue of items and takes them in arrival
 *     order.  In epoch e item j visits its nh holders (the workers holding its ratings,
 *     ranked 0..nh-1 in ascending worker order) in the order rank = pi(0), pi(1), ...,
 *     pi(nh-1) of a keyed bijection pi of [0, nh): with b the bits of nh - 1, lo = b/2,
 *     key = lowbias32(lowbias32(r ^ j) ^ e*0x9E3779B9), x split into L = x >> lo and
 *     R = x mod 2^lo, eight steps, L ^= H(R, key + s*0x9E3779B9) then
 *     R ^= H(L, key + (s+1)*0x9E3779B9) for s = 0, 2, 4, 6 (H(v, c) = lowbias32(v ^ c)
 *     reduced to the half's bits; 32-bit arithmetic), map x to (L << lo) | R, repeated
 *     until the value is below nh; r = 0x6a09e667 ^ the two 32-bit halves of
 *     nomad_config.seed.  A fresh pseudo-random permutation every epoch, so every rating
 *     is updated once per epoch and t = epochs done.  At the start of a call every item is queued at its first worker
 *     (each queue in ascending item order).  The serial order depends on timing
 *     (record_trace gives it); with one worker it is the ring order.  Not available in
 *     batches.
 *   UNIFORM: asynchronous, Algorithm 1 as printed: after a visit an item goes to a worker
 *     drawn uniformly from all p (move v of item j: lowbias32(lowbias32(r ^ 0x2545F491 ^ j)
 *     + v*0x9E3779B9) scaled to [0, p)), also to workers holding none of its ratings,
 *     which pass it on.  t = the number of earlier visits of the item to the worker (kept
 *     across calls).  A call of E epochs stops moving items once E * nnz updates are done;
 *     visits already under way complete, so nomad_stats.updates can exceed E * nnz. */
typedef enum { NOMAD_SCHED_RING = 0, NOMAD_SCHED_PERM = 1, NOMAD_SCHED_UNIFORM = 2 } nomad_sched;

/* Per-rating loss l(r, d) of a rating r at prediction d = <w_i, h_j> (section 2: the method
 * takes any separable loss; the paper works with the square loss).  The updates of section
 * 2.3 use the residual e = -dl/dd in place of r - d:
 *   SQUARE    l = (r - d)^2 / 2, e = r - d;
 *   LOGISTIC  l = log(1 + exp(-r d)) for labels r = +-1, e = r / (1 + exp(r d)) (computed in
 *             FP32 with the fast exponential).
 * nomad_eval_rmse's objective J sums l + lambda/2 (|w_i|^2 + |h_j|^2) over the ratings; its
 * RMSE is that of d against r whatever the loss. */
typedef enum { NOMAD_LOSS_SQUARE = 0, NOMAD_LOSS_LOGISTIC = 1 } nomad_loss;

/* Storage type of W in device memory (H is always held in FP32); arithmetic is always
 * FP32.  NOMAD_BF16: W is rounded to bfloat16 once at nomad_init (nearest-even) and every
 * updated w_i is rounded to bfloat16 before it is stored, by the nomad_round rule:
 *   RNE         nearest, ties to even;
 *   STOCHASTIC  the FP32 result's 16 low bits plus 16 random bits, truncated (the magnitude
 *               rounds up with probability equal to the discarded fraction).  The random
 *               bits of element l of the update of rating (i, j) in epoch t are the low
 *               (l even) or high (l odd) half of lowbias32(c + l/2), with
 *               c = lowbias32(s ^ i*0x9E3779B1 ^ j*0x85EBCA77 ^ t*0xC2B2AE3D) in 32-bit
 *               arithmetic, s = the low 32 bits of nomad_config.seed, lowbias32 = C. Wellons'
 *               integer hash (x ^= x>>16; x *= 0x7feb352d; x ^= x>>15; x *= 0x846ca68b;
 *               x ^= x>>16).
 * nomad_get_factors returns W widened to FP32 (exact). */
typedef enum { NOMAD_FP32 = 0, NOMAD_BF16 = 1 } nomad_dtype;
typedef enum { NOMAD_ROUND_RNE = 0, NOMAD_ROUND_STOCHASTIC = 1 } nomad_round;

typedef struct {
    int32_t k;          /* latent dimension, 1..256 */
    float lambda;       /* regularisation of eq. (obj_fcn), >= 0 */
    float alpha, beta, gamma; /* step size s_t = alpha / (1 + beta t^gamma), eq. (stepsize_method);
                           t = number of earlier updates of the (i,j) pair = epochs done */
    int32_t sched;      /* nomad_sched */
    int32_t dtype;      /* nomad_dtype */
    int32_t rounding;   /* nomad_round, used when dtype = NOMAD_BF16 */
    int32_t workers;    /* p, number of workers (workgroups, all resident at once);
                           0 = one per compute unit */
    int32_t waves_per_worker; /* compute wavefronts of a worker, 1..15 (1..8 under the asynchronous
                                 schedules); 0 = 8 (ring), 4 (asynchronous; 6 when some row holds
                                 more than half of a four-wave share of the ratings, i.e. its
                                 degree exceeds nnz / (8 x workers)) */
    int32_t item_slots;  /* items a worker holds in LDS at once: a power of two, 1..64;
                            0 = as many as LDS allows, up to 64 */
    int32_t window;      /* rows a compute wave keeps in flight: 8, 16 or 32 (other values in
                            1..32 are rounded up); 0 = as many as LDS allows, up to 32 */
    int32_t record_trace;    /* 1 = record every (worker, item) visit for replay */
    int32_t collect_stats;   /* 1 = time the phases of every worker (nomad_get_worker_stats);
                                counts are always collected */
    int32_t debug_ownership; /* 1 = check the ownership invariant of section 3.1 while training
                                (nomad_stats.violations): every item has one holder word, which
                                a worker claims when it takes the item over (it must find the
                                item free) and frees when it passes the item on (it must find
                                its own claim), and every rating a compute wave updates must be
                                of a row the wave owns (the ring order checks a wave's ratings
                                once per launch, before its update loop, and counts a violation
                                per epoch).  Costs two atomics per visit. */
    int32_t t_source;        /* what t counts in s_t: 0 = earlier updates of the same (i,j) pair
                                (section 5.1; the default), 1 = all updates applied before the
                                visit since nomad_init, in the run's serial order (the global
                                count; every rating of a visit uses the count at the visit's
                                start).  Not available in batches. */
    int32_t balance;         /* 1 = dynamic load balancing (section 3.3) under the asynchronous
                                schedules: a worker's load is the number of items waiting in its
                                queue.  UNIFORM: the next worker is the less loaded of two drawn
                                uniformly (the second draw hashes r ^ 0x5BD1E995 in place of r;
                                the first on a tie).  PERM: two holders not yet visited in the
                                epoch are candidates, the one held over from the item's last
                                choice (if any, else the next of the visiting order) and the next
                                of the visiting order; the less loaded goes next (the first on a
                                tie) and the other is held over, so every holder is still visited
                                once per epoch.  ENOTIMPL under RING. */
    int32_t transpose;       /* 1 = make the row factors nomadic instead (the symmetry noted in
                                section 3.1): the library runs NOMAD on the transposed matrix, so
                                the columns of A are partitioned among the workers, h_j stay
                                with their worker, and the w_i travel.  Every argument and result
                                of the calls keeps A's orientation (nomad_init's m, n, d_row,
                                d_col, d_W0, d_H0; nomad_get_factors' d_W, d_H; the evaluation's
                                rows and columns); what is transposed is reported by
                                nomad_get_partition (bounds of column blocks), nomad_get_trace
                                (the travelling index is the row i) and the BF16 storage form
                                (the resident factor, H, is the one stored in bfloat16; W is then
                                FP32).  Pays off when rows are fewer than columns.  ENOTIMPL in
                                batches. */
    int32_t loss;            /* nomad_loss; batches use NOMAD_LOSS_SQUARE (ENOTIMPL otherwise) */
    uint64_t seed;      /* initial item placement g(j) = splitmix64(seed ^ j) mod p, routing,
                           stochastic rounding */
} nomad_config;

typedef struct {
    double seconds;        /* device time of the training kernel launches of the call (HIP events
                              around each launch; seeding kernels and resets excluded) */
    uint64_t updates;      /* SGD updates applied by the call */
    uint64_t epochs_done;  /* epochs completed since nomad_init */
    double layout_seconds; /* device time spent by nomad_init building the layout */
    uint64_t hops;         /* hand-offs of an item from one worker to the next during the call:
                              queue pushes under the asynchronous schedules (pass-through
                              visits of uniform routing included); under the ring order,
                              passes to a later visit of the same call */
    uint64_t violations;   /* ownership violations seen by debug_ownership (always 0 when
                              the invariant holds; 0 when the checks are off) */
} nomad_stats;

/* Default values of nomad_config (k = 0 means "caller must set"). */
void nomad_config_default(nomad_config *cfg);

/* Build a context for one problem: validates the training ratings, partitions the rows
 * (section 3.1 footnote: equal numbers of ratings), lays the ratings out per worker in
 * processing order, and copies W0/H0 into the context.
 *   m, n      matrix size (m, n >= 1, each < 2^31); nnz >= 0 training ratings (< 2^32).
 *   d_row, d_col, d_val  device COO, nnz entries each: int32 row in [0,m), int32 column in
 *             [0,n), float rating.  Omega is a set: a repeated (i,j) is EINVAL.
 *   d_W0      device m x k FP32 initial user factors, row-major (row stride k).
 *   d_H0      device n x k FP32 initial item factors, row-major.
 *   hip_stream  hipStream_t to order all work on (NULL = default stream).
 * On success *out holds a new context; on failure *out is NULL. */
nomad_status nomad_init(nomad_ctx **out, const nomad_config *cfg, int64_t m, int64_t n, int64_t nnz,
                        const int32_t *d_row, const int32_t *d_col, const float *d_val,
                        const float *d_W0, const float *d_H0, void *hip_stream);

/* Run `epochs` >= 0 epochs of NOMAD SGD (every training rating updated once per epoch),
 * continuing the step-size counter from earlier calls.  `out` may be NULL. */
nomad_status nomad_train_epochs(nomad_ctx *ctx, int32_t epochs, nomad_stats *out);

/* Test RMSE sqrt(sum (A_ij - <w_i,h_j>)^2 / nnz) (section 5.1) over the given device COO,
 * with FP64 dot products and a deterministic compensated (Neumaier) sum.  If
 * objective_out is not NULL it also receives
 * J = 1/2 sum [ (A_ij - <w_i,h_j>)^2 + lambda (|w_i|^2 + |h_j|^2) ] over the same entries
 * (eq. obj_fcn in its per-rating form), or with the logistic loss (nomad_config.loss)
 * J = sum [ log(1 + exp(-A_ij <w_i,h_j>)) + lambda/2 (|w_i|^2 + |h_j|^2) ].  nnz = 0 gives
 * NaN.  Indices are checked. */
nomad_status nomad_eval_rmse(nomad_ctx *ctx, int64_t nnz, const int32_t *d_row, const int32_t *d_col,
                             const float *d_val, double *rmse_out, double *objective_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): nomad_eval_rmse with every temporary in
 * a fixed scratch array the library keeps on each device (about 512 KB, held until the
 * process ends).  Nothing is allocated, cleared with a memset, or synchronised: the work
 * is only queued on the context's stream.  Results go to d_out, a device array of three
 * doubles: [0] the RMSE (NaN when nnz = 0), [1] J as nomad_eval_rmse defines it, [2] 1.0
 * if some entry's index was out of range (the sums then skip it), else 0.0.
 *   nnz       0 .. 134,217,728 (the scratch holds one partial sum per 8,192 entries, at
 *             most 16,384 of them); larger is EINVAL.
 * Every call on one device shares that device's scratch: calls whose work overlaps on a
 * device (other streams, other threads, other contexts) race and give undefined results.
 * ESTATE for a batch, a failed context or NULL; EINVAL for bad arguments; EDEVICE if a HIP
 * launch fails. */
nomad_status nomad_eval_rmse_noalloc(nomad_ctx *ctx, int64_t nnz, const int32_t *d_row, const int32_t *d_col,
                                     const float *d_val, double *d_out);

/* Copy the current factors out as FP32: d_W m x k, d_H n x k (device, row-major). */
nomad_status nomad_get_factors(nomad_ctx *ctx, float *d_W, float *d_H);

/* Row partition: h_row_start[0..p] (host, p+1 int64), worker q owns rows
 * [h_row_start[q], h_row_start[q+1]).  *p_out receives p. */
nomad_status nomad_get_partition(nomad_ctx *ctx, int32_t *p_out, int64_t *h_row_start, int64_t cap);

/* The configuration the context runs with: the one given to nomad_init with the library's
 * choices filled in (workers, waves_per_worker, item_slots, window).  *h_cfg: host.  For a
 * batch: its shared configuration (workers = the total). */
nomad_status nomad_get_config(nomad_ctx *ctx, nomad_config *h_cfg);

/* Visit trace of the last nomad_train_epochs call with record_trace = 1.  Each record is
 * four int32: (worker q, item j, step index t, visit sequence number of item j since
 * nomad_init), one per visit of an item at a worker, written when the worker takes the
 * item over.  Records of one worker appear in that worker's execution order.  With
 * h_buf = NULL only *len is set; otherwise up to `cap` records are copied to h_buf
 * (host). */
nomad_status nomad_get_trace(nomad_ctx *ctx, int64_t *len, int32_t *h_buf, int64_t cap);

/* Per-worker counters of the last nomad_train_epochs call: p rows of sixteen int64 in
 * h_stats (host, cap >= 16p).  Times are ticks of the device's 100 MHz constant clock and
 * are only collected with collect_stats = 1; counts are always collected.
 *   0 memory wave: time in the kernel            5 compute waves: time waiting for items
 *   1 memory wave: rounds of its loop              (sum over the waves)
 *   2 visits taken over                          6 ratings updated
 *   3 polls of an item not yet free              7 row reads served from an update still in
 *   4 compute waves: time in the kernel            a wave's prefetch window
 *     (sum over the waves)                       8 compute waves: longest time in the kernel
 *                                                9 memory wave: waiting for its loads/stores
 *   10 asynchronous schedules: the XCD (accelerator complex die, 0..7 on MI355X) the worker
 *      ran on, read from the hardware's XCC_ID register
 *   asynchronous schedules, memory wave, sums over the rounds of its loop:
 *   11 free item slots                          14 visits passed on (a total, not per round)
 *   12 items waiting in its queue (collect_stats 15 visits held: taken over, not yet passed
 *      = 1 only)                                   on
 *   13 rounds in which the next queue entry was not yet written while a later one was
 *   (the ring order leaves 10..15 zero) */
nomad_status nomad_get_worker_stats(nomad_ctx *ctx, int64_t *h_stats, int64_t cap);

/* One problem of a batch (nomad_init_batched): the arguments of nomad_init that differ
 * between problems.  Arrays as in nomad_init (device, caller-owned, read during the call). */
typedef struct {
    int64_t m, n, nnz;
    const int32_t *d_row, *d_col;
    const float *d_val;
    const float *d_W0, *d_H0;  /* m x k and n x k FP32, row-major */
    int32_t k;                 /* 1..256; the batch stores every problem at the largest padded k */
    float lambda, alpha, beta, gamma;
} nomad_problem_desc;

/* Several independent problems trained together: every nomad_train_epochs call on the
 * returned batch context runs all of them, each in its own ring order (section 3.1,
 * Algorithm 1) exactly as it would alone with the same worker count, in one launch.
 * `common` gives the fields the problems share (schedule, storage type, rounding, waves,
 * item slots, window, seed, collect_stats); its k, lambda, alpha, beta and gamma are ignored
 * and its `workers` is the total (0 = as many as can be resident; window 0 means 8 here,
 * which lets more workers share a compute unit).  Problem b gets
 * max(1, about workers * nnz_b / sum nnz) workers (largest remainders).  EINVAL if a
 * problem is invalid (the message names it) or there are more problems than workers;
 * ENOTIMPL with record_trace.  Problems are read back through nomad_batch_problem. */
nomad_status nomad_init_batched(nomad_ctx **out, int32_t nprob, const nomad_problem_desc *descs,
                                const nomad_config *common, void *hip_stream);

/* The context of problem b of a batch, for nomad_eval_rmse, nomad_get_factors,
 * nomad_get_partition and nomad_get_worker_stats (owned by the batch: nomad_destroy on it
 * does nothing, nomad_train_epochs on it is ESTATE).  Those calls on the batch itself are
 * ESTATE.  Callers that keep it must not use it after the batch is destroyed. */
nomad_status nomad_batch_problem(nomad_ctx *batch, int32_t b, nomad_ctx **problem);

/* Capture a batch's launch sequence for `epochs` epochs into a HIP graph owned by the
 * batch: kernels that clear the problems' abort words, diagnostics and statistics (no
 * memset nodes), then per launch of up to 64 epochs a kernel that sets the problems'
 * epoch counts and the batched worker launch.  Later nomad_train_epochs calls on the batch
 * with exactly `epochs` epochs upload the problems' launch arguments (their epochs done so
 * far) and replay the graph on the batch's stream; other epoch counts launch directly.
 * Results are those of direct launches.  epochs = 0 drops the graph.  ESTATE if `batch` is
 * not a batch; EINVAL if epochs < 0; EDEVICE if the capture fails. */
nomad_status nomad_batch_graph(nomad_ctx *batch, int32_t epochs);

/* Called by nomad_tune_batched after each candidate: its config, NOMAD_OK and the
 * seconds of its faster epoch, or the status that ruled it out (seconds 0). */
typedef void (*nomad_tune_progress)(const nomad_config *candidate, nomad_status status, double seconds,
                                    void *user);

/* Launch-shape autotuner for a batch: builds the batch (nomad_init_batched) with each
 * candidate shape — workers = 1 or 2 per CU times 4 or 8 compute waves; a field of
 * `common` that is set (> 0) stays fixed, the row window is common's — trains each for two
 * epochs from the problems' initial factors (the caller's arrays are only read), reports
 * each to `progress` if not NULL, and writes the config of the fastest epoch into *best
 * (and its seconds into *best_seconds if not NULL).  Every candidate costs a layout of the
 * whole batch.  Shapes that do not fit the device are skipped; EDEVICE if none fits, with
 * the last reason. */
nomad_status nomad_tune_batched(int32_t nprob, const nomad_problem_desc *descs, const nomad_config *common,
                                void *hip_stream, nomad_tune_progress progress, void *user, nomad_config *best,
                                double *best_seconds);

/* Free every resource of the context (of a batch: of all its problems).  NULL, and a
 * problem of a batch, are ignored. */
void nomad_destroy(nomad_ctx *ctx);

/* Message of the last failure on ctx, or of the last failure of the calling thread
 * when ctx is NULL.  Never NULL; the string stays valid until the next call. */
const char *nomad_last_error(const nomad_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* NOMAD_H */
