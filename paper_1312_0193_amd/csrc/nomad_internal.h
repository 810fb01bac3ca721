// Internal declarations shared by the HIP translation units of libnomad.so.
//
// Workers and their data (section 3.1, Algorithm 1; the hybrid layout of section 3.4):
//   * A worker is one workgroup of the persistent training kernel, normally one per CU.
//     Rows are cut into p contiguous blocks with about equal numbers of ratings (section
//     3.1 footnote); worker q owns rows [row_start[q], row_start[q+1]).
//   * Inside a worker the rows are cut again, by the same rule, among its compute
//     wavefronts ("waves"): wave w of worker q owns rows
//     [wave_start[q*nw + w], wave_start[q*nw + w + 1]).  A wave alone reads and writes
//     those rows.
//   * Items are split into p groups, g(j) = splitmix64(seed ^ j) mod p (the uniformly
//     random initial queue of Algorithm 1).  In the fixed ring order worker q processes,
//     in sub-step s = 0..p-1 of an epoch, the items of group (q + s) mod p in ascending
//     j, each over its ratings in ascending row i.  One such (worker, item) run is a
//     "visit"; visits of worker q are numbered x = 0, 1, ... in that order.
//   * Inside a visit the item passes through the worker's waves in ascending order
//     (rows ascending), through LDS.  A visit of item j at worker q may start once every
//     earlier visit of j in the ring order has finished; a per-item counter of finished
//     visits records that.
//   * Each wave reads its ratings as one stream in processing order: 16-byte records
//     (row, rating, visit information, and where the row is used again inside the
//     wave's window of rows in flight).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nomad {

constexpr int kMaxK = 256;          // largest latent dimension
constexpr int kMaxWaves = 15;       // compute waves per worker (plus one memory wave)
constexpr int kMaxWavesAsync = 8;   // the same under the asynchronous schedules (their kernel is
                                    // built for nine waves, so that each may use 168 registers)
constexpr int kDefaultWaves = 8;
// Asynchronous schedules: fewer compute waves per worker leave the SIMDs to the waves that
// carry the long runs of heavy items (on a Zipf workload 4 waves beat 8 by a fifth).
constexpr int kDefaultWavesAsync = 4;
// The default under the asynchronous schedules when a row holds more than half of a
// four-wave share of the ratings: such rows make some workers host a visit from nearly every
// item, and more waves spread those workers' other rows (measured on the Yahoo-shaped
// workload: 0.65 s per epoch with four waves, 0.52 s with six, 0.54 s with eight).
constexpr int kDenseWavesAsync = 6;
constexpr int kMaxItemSlots = 64;   // items a worker holds in LDS at once
constexpr int kMaxWorkers = 4096;
constexpr int kMaxEpochsPerLaunch = 64;  // a call runs longer epoch counts as several launches
constexpr int kMaxWindow = 32;           // rows a compute wave keeps in flight

// Visit information of a rating record.
constexpr uint32_t kInfoXBits = 23;                       // visit index x within the epoch
constexpr uint32_t kInfoXMask = (1u << kInfoXBits) - 1u;
constexpr uint32_t kInfoFirst = 1u << 23;                 // first rating of the wave in the visit
constexpr uint32_t kInfoLast = 1u << 24;                  // last rating of the wave in the visit
constexpr uint32_t kInfoPrevShift = 25;                   // 1 + wave that precedes it in the visit,
constexpr uint32_t kInfoPrevMask = 15u;                   // 0 = first wave of the visit

// A rating of a wave's stream.  fwd: distance (in the stream, cyclically) to the next
// rating of the same row if it is less than the window D, else 0 (bits 0-7), and the same
// for the previous rating of the row (bits 8-15).
struct alignas(16) RatingRec {
    int32_t row;
    float r;
    uint32_t info;
    uint32_t fwd;
};

// One visit of a worker (16 bytes), in processing order.
struct alignas(16) VisitRec {
    int32_t j;       // item
    uint32_t v;      // ordinal of this visit among the item's visits in one epoch
    uint32_t nvis;   // visits of the item per epoch
    int32_t lastw;   // last wave of the worker holding ratings of the item
};

static_assert(sizeof(RatingRec) == 16, "RatingRec layout");
static_assert(sizeof(VisitRec) == 16, "VisitRec layout");

// Per-worker counters of a training call (100 MHz constant-clock ticks unless a count).
enum WStat {
    kWStatMemTotal = 0,    // memory wave: time in the kernel
    kWStatMemIters = 1,    // memory wave: rounds of its loop
    kWStatVisits = 2,      // visits taken over
    kWStatPollMiss = 3,    // polls of an item that was not yet free
    kWStatCompTotal = 4,   // compute waves: time in the kernel (sum over waves)
    kWStatItemWait = 5,    // compute waves: time waiting for an item (sum over waves)
    kWStatRatings = 6,     // ratings updated
    kWStatForwarded = 7,   // row reads served from an update still in the prefetch window
    kWStatCompMax = 8,     // compute waves: longest time in the kernel
    kWStatMemWait = 9,     // memory wave: time waiting for its loads and stores
    kWStatXcd = 10,        // the accelerator complex die (XCD) the worker ran on
    kWStatRoom = 11,       // memory wave: free item slots, summed over its rounds
    kWStatQueueLen = 12,   // memory wave: items waiting in its queue, summed over rounds (timed)
    kWStatBlocked = 13,    // memory wave: rounds whose next queue entry was not yet written
                           // while a later one was
    kWStatPassed = 14,     // memory wave: visits passed on
    kWStatHeld = 15,       // memory wave: visits held (taken, not yet passed on), summed over rounds
    kWStatCount = 16
};

// Counter-based mixing function splitmix64 (Steele, Lea, Flood 2014).
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__host__ __device__ inline int32_t item_group(uint64_t seed, int64_t j, int32_t p) {
    return (int32_t)(splitmix64(seed ^ (uint64_t)j) % (uint64_t)p);
}

// Device-resident layout of one problem.
struct Plan {
    int64_t m = 0, n = 0, nnz = 0;
    int32_t p = 0;                  // workers
    int32_t nw = 0;                 // compute waves per worker
    int64_t *row_start = nullptr;   // p + 1
    int64_t *wave_start = nullptr;  // p * nw + 1 row boundaries
    int64_t *rbase = nullptr;       // p * nw + 1: wave (q, w) reads records [rbase, rbase + 1)
    RatingRec *recs = nullptr;      // nnz
    int64_t *vbase = nullptr;       // p + 1: worker q's visits are [vbase[q], vbase[q+1])
    VisitRec *visits = nullptr;
    int64_t nvisits = 0;            // (worker, item) visits per epoch
    int64_t max_worker_visits = 0;
    int64_t max_row_degree = 0;     // ratings of the densest row
    // Asynchronous schedules (build_async_tables).  A worker's "local item" x is the item of
    // its visit vbase[q] + x; the ring order's record streams are grouped by local item.
    int32_t *hold = nullptr;   // nvisits holder entries, grouped by item (workers ascending): the worker
    int32_t *hx = nullptr;     //   the item's local index at that worker
    int32_t *hitem = nullptr;  //   the item
    int32_t *hcnt = nullptr;   //   the worker's ratings of the item
    int64_t *hoff = nullptr;   // n + 1: item j's holder entries are [hoff[j], hoff[j+1])
    int32_t *xoff = nullptr;   // nvisits * nw: first record of local item x in wave w's stream, relative to
                               //   the stream start (the end is the next local item's entry, or the stream end)
    int64_t active = 0;        // items with at least one rating
    // Options (built on demand).
    int64_t *vstart = nullptr;  // per visit: ratings before it in an epoch of the ring order
    int32_t *hmap = nullptr;    // uniform routing: p x n, holder entry of (worker, item) or -1
};

// Arguments of the training kernel.
// Launch shape of a worker, shared by every problem of a batched launch.
struct Shape {
    int32_t kp, nw, slots, window;
    int32_t maxw;          // workers that can be resident at once with this shape
    int32_t cus, max_lds;  // device figures
};

struct TrainArgs {
    int64_t m, n, nnz;
    void *W;                    // m x kp, FP32 or bfloat16 (wbytes per element)
    float *H;                   // n x kp
    const RatingRec *recs;
    const int64_t *rbase;
    const VisitRec *visits;
    const int64_t *vbase;
    uint32_t *tok_done;         // n: completed visits of each item (across calls)
    uint32_t *abort_flag;       // 0 = running; 1 = a wait timed out; 2 = malformed layout
    float *dummy;               // p x kMaxWaves words: target of placeholder stores
    int32_t *diag;              // 8 words: the first wait that ran out of time (see train.hip)
    int32_t kp;
    int32_t wbytes;             // 4: W in FP32; 2: W in bfloat16
    int32_t rounding;           // bfloat16 stores: 0 nearest-even, 1 stochastic
    uint32_t sr_seed;           // stochastic rounding: seed of the counter hash
    int32_t p;                  // workers
    int32_t nw;                 // compute waves per worker
    int32_t slots;              // item slots per worker (<= 64)
    int32_t window;             // D: rows a compute wave keeps in flight (8, 16 or 32)
    int32_t epoch0, epochs;     // epochs done before the launch, epochs of the launch
    int32_t wg0;                // first workgroup of this problem in a batched launch (else 0)
    float lambda;
    double alpha, beta, gamma;  // step size s_t = alpha / (1 + beta t^gamma), eq. (stepsize_method)
    int64_t *wstats;            // per worker kWStatCount counters
    bool timing;                // also time the phases (costs clock reads)
    // Asynchronous schedules (sched 1): the plan's holder and offset tables, the inbound
    // queues and the items' state.
    int32_t sched;              // 0 ring, 1 random permutation per epoch, 2 uniform routing (both asynchronous)
    const int32_t *hold, *hx, *hitem;
    const int64_t *hoff;
    const int32_t *xoff;
    uint64_t *queue;            // permutation: nvisits, worker q's inbound queue is [vbase[q], vbase[q+1]);
                                // uniform routing: p * n, worker q's is [q n, (q + 1) n)
    int32_t *tvis;              // uniform routing: per holder entry, visits so far (t of the next one)
    const int32_t *hcnt;        // per holder entry: the worker's ratings of the item
    unsigned long long *upd;    // uniform routing: updates applied in the call
    unsigned long long budget;  // uniform routing: updates after which items stop moving
    uint32_t *qtail;            // p: pushes into each queue during the launch
    uint32_t *qhead;            // p: entries each worker has taken from its queue (published for
                                // the load-balanced choice; queue length = qtail - qhead)
    int32_t balance;            // 1: section 3.3's dynamic load balancing of the next worker
    int32_t loss;               // per-rating loss: 0 square, 1 logistic (the kernels are compiled per loss)
    int32_t *istate;            // n x 4: state of each item, written by its holder before it moves on:
                                //   [0] permutation: epoch of the next visit; uniform: moves so far
                                //   [1] permutation: positions of the epoch's visiting order used
                                //       (the next visit's included)
                                //   [2] visits of the item (that updated something) since nomad_init
                                //   [3] permutation with load balancing: the holder rank held over
                                //       as a candidate for the next choice, or -1
    const int32_t *hmap;        // uniform routing: p x n, holder entry of (worker, item) or -1
    uint32_t *parked;           // items that finished the launch's epochs
    int64_t active;             // items with at least one rating
    uint32_t route_seed;
    const int64_t *wave_start;  // p * nw + 1 row boundaries of the compute waves
    const int64_t *vstart;      // ring order, gstep: per visit, ratings before it in an epoch
    uint32_t *owner;            // ownership checks (NULL = off): n words, the worker holding each
                                // item or 0xFFFFFFFF
    unsigned long long *counters;  // [0] ownership violations, [1] hops, [2] global update count
    int32_t gstep;              // 1: t = global count of updates before the visit (step-size option)
    int32_t keep_rows;          // asynchronous schedules: some compute wave owns a single row (its
                                // single-rating visits keep that row in LDS; see train.hip)
    int32_t *trace;             // optional: 4 ints per visit
    int64_t *trace_len;         // optional counter
    int64_t trace_cap;
};

// Host-side entry points of the translation units (all stream-ordered).

// layout.hip: the ratings of the densest row (stream-ordered, then synchronous).
hipError_t max_row_degree(const int32_t *d_row, int64_t nnz, int64_t m, hipStream_t stream, int64_t *out);
// layout.hip: build the layout; err_code receives 0 or a nomad_status value.
hipError_t build_plan(Plan *plan, int64_t m, int64_t n, int64_t nnz, const int32_t *d_row,
                      const int32_t *d_col, const float *d_val, int32_t p, int32_t nw, int32_t window,
                      uint64_t seed, hipStream_t stream, int *err_code, char *msg, size_t msg_len);
void free_plan(Plan *plan);
// The tables of the asynchronous schedules, from a built plan.
hipError_t build_async_tables(Plan *plan, hipStream_t stream);
// Per visit, the number of ratings before it in one epoch of the ring order (the global
// update count option of the step size).
hipError_t build_visit_starts(Plan *plan, uint64_t seed, hipStream_t stream);
// Uniform routing's holder map (after build_async_tables).
hipError_t build_holder_map(Plan *plan, hipStream_t stream);

// train.hip
size_t train_lds_bytes(int32_t kp, int32_t nw, int32_t slots, int32_t window, int32_t wbytes);
hipError_t launch_train(const TrainArgs &a, hipStream_t stream);
// Asynchronous schedules: queue every item at the first worker of its visiting order for
// epoch a.epoch0 (each worker's queue in ascending item order); scratch: 5 n words at
// `scratch` plus the sort's temporary storage.  Then run the launch.
hipError_t seed_train_async(const TrainArgs &a, void *scratch, size_t scratch_bytes, hipStream_t stream);
hipError_t launch_train_async(const TrainArgs &a, hipStream_t stream);
size_t async_scratch_bytes(int64_t n, int32_t p);
// Several problems in one launch: d_descs[b] describes problem b (its wg0 = first
// workgroup), d_wg_prob[g] = the problem of workgroup g; `shape` gives the launch shape
// shared by all (kp, storage type, nw, slots, window).
hipError_t launch_train_batch(const TrainArgs &shape, int32_t workgroups, const TrainArgs *d_descs,
                              const int32_t *d_wg_prob, hipStream_t stream);
// Kernels a captured batch launch uses in place of memsets (a HIP graph records no memset
// nodes here): clear every problem's abort word, diagnostics and worker statistics; set
// every problem's launch epoch count to `epochs` after advancing its epoch0 by `advance`.
hipError_t launch_batch_reset(const TrainArgs *d_descs, int32_t nprob, hipStream_t stream);
hipError_t launch_batch_epochs(TrainArgs *d_descs, int32_t nprob, int32_t epochs, int32_t advance,
                               hipStream_t stream);
// Workers of `nw` compute waves that can be resident at once on the device.
// `batch`: for the batched kernel (several problems in one launch).
hipError_t train_max_workers(int32_t kp, int32_t nw, int32_t slots, int32_t window, int32_t wbytes,
                             int32_t *max_workers, bool async = false, int32_t loss = 0, bool batch = false);
// The row window the asynchronous kernel's LDS layout is built for (its rows are in
// registers; the layout keeps the ring kernel's shape).
constexpr int kAsyncWindow = 8;
// Row stride of the factors for k: a whole number of 16-byte pieces per lane of a wave.
inline int32_t padded_k(int32_t k) { return k <= 64 ? 64 : (k <= 128 ? 128 : 256); }

// eval.hip: FP64 RMSE / objective with a deterministic compensated sum.
hipError_t eval_sums(const void *W, int32_t wbytes, const float *H, int32_t k, int32_t kp, int64_t m, int64_t n,
                     int64_t nnz, const int32_t *row, const int32_t *col, const float *val,
                     double lambda, int32_t loss, double *h_sq_err, double *h_obj, int *h_bad_index,
                     void *scratch, size_t scratch_bytes, hipStream_t stream);
// FP32 rows (width k) to bfloat16 rows (width kp; nearest-even), and back (exact).
hipError_t to_bf16(const float *src, int32_t k, uint16_t *dst, int32_t kp, int64_t rows, hipStream_t st);
hipError_t from_bf16(const uint16_t *src, int32_t kp, float *dst, int32_t k, int64_t rows, hipStream_t st);
size_t eval_scratch_bytes();
// Allocation-free evaluation: the partial and final sums live in a file-scope device array
// (one per device); its device address comes from noalloc_scratch_address, called with
// that device current.  Results go to d_out (device: RMSE, J, bad-index flag); nothing is
// allocated, set with a memset or synchronised.
int64_t noalloc_max_nnz();
size_t noalloc_scratch_bytes();
hipError_t noalloc_scratch_address(void **ptr);
hipError_t eval_sums_noalloc(const void *W, int32_t wbytes, const float *H, int32_t k, int32_t kp, int64_t m,
                             int64_t n, int64_t nnz, const int32_t *row, const int32_t *col, const float *val,
                             double lambda, int32_t loss, void *scratch_ptr, double *d_out, hipStream_t stream);

}  // namespace nomad
