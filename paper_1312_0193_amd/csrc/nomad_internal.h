// Internal declarations shared by the HIP translation units of libnomad.so.
//
// Data layout produced by the layout step (one-time, inside nomad_init):
//   * Rows are cut into p contiguous blocks with about equal numbers of ratings
//     (section 3.1 footnote).  Worker q owns rows [row_start[q], row_start[q+1]).
//   * Items are split into p groups, g(j) = splitmix64(seed ^ j) mod p (the uniformly
//     random initial queue of Algorithm 1).  A "block" (q, g) is every rating of worker
//     q on an item of group g.  Items pass between workers one at a time: a visit of item
//     j at worker q (its ratings in block (q, g(j))) may start once every earlier visit of
//     j in the ring order has finished, which a per-item counter of finished visits
//     records.
//   * Each worker's ratings are ordered by (ring sub-step s = (g - q) mod p, item j,
//     row i) and cut into "chunks" of at most 64 ratings that never straddle a block.
//     A worker keeps S vectors (rows w_i and items h_j) in LDS slots.  The plan says, per
//     chunk, which vectors to load into which slot (and which row that slot held before,
//     to be written back first), which items leave after the chunk (their visit ends),
//     and, at the end of an epoch, which rows are still in LDS.  Rows stay in LDS while
//     they are used again soon (the victim of a load is the row whose next use is
//     farthest, among rows unused for a few chunks, so the loads of a chunk can be
//     staged while the chunks before it are being computed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nomad {

constexpr int kMaxK = 256;           // largest latent dimension
constexpr int kMaxRatingsPerChunk = 64;
constexpr int kMaxEventsPerChunk = 64;  // loads + item releases of one chunk
constexpr int kMaxSlots = 256;       // slot ids are 8 bits
constexpr int kRing = 4;             // chunks staged ahead of the compute wave (ring entries)
constexpr int kLookahead = 2;        // preferred age (chunks) of a row evicted by a load

// Vectors one chunk may load (one event record per lane of the memory wave).
__host__ __device__ inline int max_loads_per_chunk(int kp) {
    (void)kp;
    return kMaxEventsPerChunk;
}

// Per-worker counters of a training call (100 MHz constant-clock ticks unless a count).
enum WStat {
    kWStatTotal = 0,     // compute wave: time in the kernel
    kWStatAcquire = 1,   // memory wave: time waiting for items to be passed on
    kWStatMemWait = 2,   // memory wave: time waiting for loads and stores to complete
    kWStatChunks = 3,
    kWStatSgd = 4,       // compute wave: time in the rating updates
    kWStatSlotWait = 5,  // memory wave: time waiting for the compute wave to free slots
    kWStatRatings = 6,
    kWStatStarve = 7,    // compute wave: time waiting for a chunk to be staged
    kWStatMemTotal = 8,  // memory wave: time in the kernel
    kWStatCommit = 9,    // memory wave: write-backs of evicted rows, LDS stores, ring entry
    kWStatRetire = 10,   // memory wave: passing on items outside of waits
    kWStatIssue = 11,    // memory wave: prefetch, polls, records
    kWStatLoads = 12,    // vectors loaded
    kWStatLate = 13,     // vectors loaded without prefetch (first chunk of an epoch, busy items)
    kWStatCount = 16
};

// Events of a chunk, in this order: loads (row or item into a slot), releases (items
// whose visit ends with the chunk), and for the last chunk of an epoch the rows still
// in LDS (written back at the end of the epoch).
enum EvKind : uint32_t { kEvLoadRow = 0, kEvLoadItem = 1, kEvRelease = 2, kEvFlush = 3 };

struct alignas(16) EvRec {
    int32_t id;      // row or item id
    uint32_t sk;     // slot | kind << 8
    int32_t evict;   // loads: row written back from the slot before the load, or -1
    uint32_t vis;    // items: v | nvis << 16, the visit may start once the item has
                     // completed epoch * nvis + v visits (v = ordinal of this visit
                     // among the item's visits in one epoch of the ring order)
};

// One chunk of a worker's plan (32 bytes).
struct alignas(16) ChunkRec {
    int64_t rat;        // first rating record (global index)
    int64_t ev;         // first event record (global index)
    uint16_t nrat, nload, nrel, nflush;
    int32_t need_done;  // the chunk's loads may overwrite their slots once the compute
                        // wave has completed this many chunks of the epoch
    uint32_t flags;
};

// A rating inside a chunk (8 bytes): row slot, item slot and the rating value.
struct RatingRec {
    uint32_t slots;  // row slot | item slot << 8
    float r;
};

static_assert(sizeof(ChunkRec) == 32, "ChunkRec layout");
static_assert(sizeof(EvRec) == 16, "EvRec layout");
static_assert(sizeof(RatingRec) == 8, "RatingRec layout");

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

// Device-resident plan of one problem.
struct Plan {
    int64_t m = 0, n = 0, nnz = 0;
    int32_t p = 0;          // workers
    int32_t kp = 0;         // padded row stride (multiple of 4)
    int32_t slots = 0;      // S, LDS vector slots per worker
    int32_t loads = 0;      // max vectors loaded per chunk
    int64_t nchunks = 0, nevents = 0;
    int64_t *row_start = nullptr;  // p + 1
    int64_t *wck = nullptr;        // p + 1: worker q's chunks are [wck[q], wck[q+1])
    ChunkRec *chunks = nullptr;
    EvRec *events = nullptr;
    RatingRec *ratings = nullptr;  // nnz, in processing order
    int64_t nvisits = 0;           // (worker, item) visits per epoch
    int64_t nloads = 0;            // vectors loaded per epoch (rows and items)
};

// Arguments of the training kernel.
struct TrainArgs {
    int64_t m, n;             // bounds of row / item ids (plan validation)
    float *W;                 // m x kp
    float *H;                 // n x kp
    const int64_t *wck;
    const ChunkRec *chunks;
    const EvRec *events;
    const RatingRec *ratings;
    uint32_t *tok_done;       // n: completed visits of each item (across calls)
    int32_t kp;
    int32_t slots;            // S
    int32_t p;                // workers
    int32_t group;            // workers per workgroup (1, 2 or 4)
    int32_t epoch0, epochs;
    float lambda;
    double alpha, beta, gamma;
    int64_t *wstats;          // per worker kWStatCount counters
    bool timing;              // also time the phases (costs clock reads)
    int32_t *trace;           // optional: 4 ints per visit
    int64_t *trace_len;       // optional counter
    int64_t trace_cap;
};

// Host-side entry points of the translation units (all stream-ordered).

// layout.hip: build the plan; err_code receives 0 or a nomad_status value.
hipError_t build_plan(Plan *plan, int64_t m, int64_t n, int64_t nnz, const int32_t *d_row,
                      const int32_t *d_col, const float *d_val, int32_t p, int32_t kp, int32_t slots,
                      int32_t loads, uint64_t seed, hipStream_t stream, int *err_code, char *msg,
                      size_t msg_len);
void free_plan(Plan *plan);

// train.hip
size_t train_lds_bytes(int32_t kp, int32_t slots);  // per worker
int32_t train_group(int32_t kp, int32_t slots, size_t max_lds_per_block);
hipError_t launch_train(const TrainArgs &a, int32_t p, uint32_t *abort_flag, hipStream_t stream);
hipError_t train_max_workers(int32_t kp, int32_t slots, int32_t group, int32_t *max_workers);

// eval.hip: FP64 RMSE / objective with a deterministic compensated sum.
hipError_t eval_sums(const float *W, const float *H, int32_t k, int32_t kp, int64_t m, int64_t n,
                     int64_t nnz, const int32_t *row, const int32_t *col, const float *val,
                     double lambda, double *h_sq_err, double *h_obj, int *h_bad_index,
                     void *scratch, size_t scratch_bytes, hipStream_t stream);
size_t eval_scratch_bytes();

}  // namespace nomad
