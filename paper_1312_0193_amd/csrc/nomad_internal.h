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
//     row i) and cut into "chunks": runs of at most R distinct rows, T distinct items
//     and 64 ratings that never straddle a block.  A chunk is the unit a worker stages
//     in LDS; for each staged row / item the plan gives its LDS slot, whether it must be
//     read from global memory or is still in that slot from the previous chunk, and
//     whether it stays there for the next chunk instead of being written back.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nomad {

constexpr int kMaxK = 256;          // largest latent dimension
constexpr int kMaxRatingsPerChunk = 64;
constexpr int kMaxSlots = 64;       // R + T <= 64 (one slot record per lane)
// Register staging of the next chunk: 16-byte pieces per lane for its rows / items, so
// R * k_padded / 4 <= 64 * kRowPiecesPerLane and T * k_padded / 4 <= 64 * kItemPiecesPerLane.
constexpr int kRowPiecesPerLane = 12;
constexpr int kItemPiecesPerLane = 6;

enum ChunkFlags : uint32_t { kFirstOfBlock = 1u, kLastOfBlock = 2u };

// Per-worker counters of a training call (100 MHz constant-clock ticks unless a count):
// time in the kernel, time blocked acquiring a group, time waiting at the top of an
// iteration for the previous iteration's memory traffic, chunks processed, time in the
// updates, time issuing memory traffic, ratings processed, time staging into LDS.
enum WStat {
    kWStatTotal = 0,
    kWStatAcquire = 1,
    kWStatMemWait = 2,
    kWStatChunks = 3,
    kWStatSgd = 4,    // time in the rating updates
    kWStatIssue = 5,  // time issuing write-backs, prefetches and polls
    kWStatRatings = 6,
    kWStatStage = 7,  // time writing staged vectors to LDS and carrying
    kWStatCount = 8
};

// One chunk of a worker's plan (32 bytes).
struct alignas(16) ChunkRec {
    int64_t rat;    // first rating record (global index into the rating array)
    int64_t slot;   // first slot record (rows first, then items)
    uint32_t info;  // nrat | nr << 8 | nt << 16 | flags << 24
    int32_t group;  // item group g of the block (ring sub-step s = (g - q) mod p)
    int32_t pad0, pad1;
};

// A staged row or item (16 bytes): global id; physical LDS slot (rows and items have
// separate slot ranges); flags: kSlotNew = read it from global memory (otherwise the
// previous chunk left it in this slot), kSlotKeep = the next chunk uses it again (no
// write back, keep the slot); for items, the visit's ordinal v among the item's visits
// in one epoch of the ring order and the item's number of visits per epoch nvis, so that
// this visit may start once the item has completed epoch * nvis + v visits.
enum SlotFlags : uint16_t { kSlotNew = 1, kSlotKeep = 2 };
struct SlotRec {
    int32_t id;
    int16_t phys;
    uint16_t flags;
    int32_t v;
    int32_t nvis;
};

// A rating inside a chunk (8 bytes): row slot, item slot and the rating value.
struct RatingRec {
    uint32_t slots;  // row slot | item slot << 8
    float r;
};

static_assert(sizeof(ChunkRec) == 32, "ChunkRec layout");
static_assert(sizeof(SlotRec) == 16, "SlotRec layout");
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
    int32_t k = 0, kp = 0;  // latent dimension and padded row stride (multiple of 4)
    int32_t rmax = 0, tmax = 0;
    int64_t nchunks = 0, nslots = 0;
    int64_t *row_start = nullptr;  // p + 1
    int64_t *wck = nullptr;        // p + 1: worker q's chunks are [wck[q], wck[q+1])
    ChunkRec *chunks = nullptr;
    SlotRec *slots = nullptr;
    RatingRec *ratings = nullptr;  // nnz, in processing order
    uint32_t *nvis = nullptr;      // n: visits per epoch of each item
    int64_t nvisits = 0;           // (worker, item) visits per epoch
};

// Arguments of the training kernel.
struct TrainArgs {
    int64_t m, n;             // bounds of row / item ids (plan validation)
    float *W;                 // m x kp
    float *H;                 // n x kp
    const int64_t *wck;
    const ChunkRec *chunks;
    const SlotRec *slots;
    const RatingRec *ratings;
    uint32_t *tok_done;       // n: completed visits of each item (across calls)
    int32_t kp;
    int32_t rmax, tmax;       // slot capacity of a buffer: rows then items
    int32_t epoch0, epochs;
    float lambda;
    double alpha, beta, gamma;
    int64_t *wstats;          // optional: per worker 4 counters (see kWStat*)
    int32_t *trace;           // optional: 4 ints per visit
    int64_t *trace_len;       // optional counter
    int64_t trace_cap;
};

// Host-side entry points of the translation units (all stream-ordered, return hipError_t
// or a negative NOMAD error code via the out-parameter conventions below).

// layout.hip: build the plan; err_code receives 0 or a nomad_status value.
hipError_t build_plan(Plan *plan, int64_t m, int64_t n, int64_t nnz, const int32_t *d_row,
                      const int32_t *d_col, const float *d_val, int32_t p, int32_t kp, int32_t rmax,
                      int32_t tmax, uint64_t seed, hipStream_t stream, int *err_code, char *msg,
                      size_t msg_len);
void free_plan(Plan *plan);

// train.hip
size_t train_lds_bytes(int32_t kp, int32_t rmax, int32_t tmax);
hipError_t launch_train(const TrainArgs &a, int32_t p, uint32_t *abort_flag, hipStream_t stream);
hipError_t train_max_workers(int32_t kp, int32_t rmax, int32_t tmax, int32_t *max_workers);
bool train_chunk_fits(int32_t kp, int32_t rmax, int32_t tmax);

// eval.hip: FP64 RMSE / objective with a deterministic compensated sum.
hipError_t eval_sums(const float *W, const float *H, int32_t k, int32_t kp, int64_t m, int64_t n,
                     int64_t nnz, const int32_t *row, const int32_t *col, const float *val,
                     double lambda, double *h_sq_err, double *h_obj, int *h_bad_index,
                     void *scratch, size_t scratch_bytes, hipStream_t stream);
size_t eval_scratch_bytes();

}  // namespace nomad
