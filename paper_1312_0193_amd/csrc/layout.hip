// Layout of a problem for the NOMAD workers (runs once inside nomad_init).
//
//   1. check indices, count ratings per row;
//   2. exclusive scan -> rowptr;
//   3. row partition: row_start[q] = min{ i : rowptr[i] >= ceil(q * nnz / p) } (the
//      "same number of ratings" split of section 3.1, footnote);
//   4. order the ratings by (worker q, ring sub-step s = (g(j) - q) mod p, item j, row i)
//      with two stable radix sorts (first by (j, i), then by (q, s)); a repeated (i, j)
//      is rejected (Omega is a set);
//   5. number the visits of every item (its runs of ratings at one worker) in ring order,
//      i.e. by sub-step s, and count each item's visits per epoch;
//   6. cut each worker's ratings into chunks (see nomad_internal.h) in two passes: count,
//      then fill; finally link the last chunk of an epoch with the first one of the next.
#include <hipcub/hipcub.hpp>

#include <cstdio>
#include <cstring>
#include <vector>

#include "nomad_internal.h"

namespace nomad {
namespace {

constexpr int kThreads = 256;

inline int grid_for(int64_t n, int threads = kThreads, int cap = 65536) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

__global__ void k_check_degree(const int32_t *row, const int32_t *col, int64_t nnz, int64_t m,
                               int64_t n, unsigned long long *deg, int32_t *err) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t i = row[e], j = col[e];
        if (i < 0 || i >= m || j < 0 || j >= n) {
            atomicOr(err, 1);
            continue;
        }
        atomicAdd(&deg[i], 1ull);
    }
}

__global__ void k_partition(const int64_t *rowptr, int64_t m, int64_t nnz, int32_t p,
                            int64_t *row_start) {
    int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q > p) return;
    if (q == 0) { row_start[0] = 0; return; }
    if (q == p) { row_start[p] = m; return; }
    int64_t target = ((int64_t)q * nnz + p - 1) / p;
    int64_t lo = 0, hi = m;  // smallest i in [0, m] with rowptr[i] >= target
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (rowptr[mid] >= target) hi = mid; else lo = mid + 1;
    }
    row_start[q] = lo;
}

__device__ inline int32_t worker_of_row(const int64_t *row_start, int32_t p, int64_t i) {
    int32_t lo = 0, hi = p - 1;  // largest q with row_start[q] <= i
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (row_start[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void k_key_ji(const int32_t *row, const int32_t *col, int64_t nnz, int64_t m,
                         uint64_t *key, uint32_t *idx) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        key[e] = (uint64_t)col[e] * (uint64_t)m + (uint64_t)row[e];
        idx[e] = (uint32_t)e;
    }
}

__global__ void k_check_dup(const uint64_t *key, int64_t nnz, int32_t *err) {
    for (int64_t e = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (key[e] == key[e - 1]) atomicOr(err, 2);
    }
}

__global__ void k_key_qs(const uint32_t *idx, const int32_t *row, const int32_t *col, int64_t nnz,
                         const int64_t *row_start, int32_t p, uint64_t seed, uint32_t *key) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t x = idx[e];
        int32_t q = worker_of_row(row_start, p, row[x]);
        int32_t g = item_group(seed, col[x], p);
        int32_t s = (g - q + p) % p;
        key[e] = (uint32_t)q * (uint32_t)p + (uint32_t)s;
    }
}

__global__ void k_gather(const uint32_t *idx, const int32_t *row, const int32_t *col,
                         const float *val, int64_t nnz, int32_t *srow, int32_t *scol, float *sval) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t x = idx[e];
        srow[e] = row[x];
        scol[e] = col[x];
        sval[e] = val[x];
    }
}

// Block boundaries from the sorted (q, s) keys: blocks are [bfirst[b], bend[b]).
__global__ void k_block_bounds(const uint32_t *key, int64_t nnz, int64_t *bfirst, int64_t *bend) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t b = key[e];
        if (e == 0 || key[e - 1] != b) bfirst[b] = e;
        if (e == nnz - 1 || key[e + 1] != b) bend[b] = e + 1;
    }
}

// Visits: maximal runs of one (worker, item) in the (q, s, j, i) order.
__global__ void k_visit_start(const uint32_t *key2, const int32_t *scol, int64_t nnz, uint32_t *is_start) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        is_start[e] = (e == 0 || key2[e] != key2[e - 1] || scol[e] != scol[e - 1]) ? 1u : 0u;
}

// For each visit (at its first rating e): sort key (item, sub-step) and the visit id.
__global__ void k_visit_keys(const uint32_t *is_start, const uint32_t *vid, const uint32_t *key2,
                             const int32_t *scol, int64_t nnz, int32_t p, uint64_t *vkey, uint32_t *vidx,
                             uint32_t *nvis) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (!is_start[e]) continue;
        const uint32_t v = vid[e];
        const uint32_t s = key2[e] % (uint32_t)p;
        vkey[v] = (uint64_t)scol[e] * (uint64_t)p + s;
        vidx[v] = v;
        atomicAdd(&nvis[scol[e]], 1u);
    }
}

// Visit ordinal within its item: position in the (item, sub-step) order minus the
// item's first position.
__global__ void k_visit_ordinal(const uint64_t *vkey_sorted, const uint32_t *vidx_sorted, const uint32_t *seg,
                                int64_t nv, int32_t p, uint32_t *vord) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nv;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t j = vkey_sorted[t] / (uint64_t)p;
        vord[vidx_sorted[t]] = (uint32_t)(t - seg[j]);
    }
}

struct ChunkerArgs {
    const int32_t *srow, *scol;
    const float *sval;
    const int64_t *bfirst, *bend;
    const uint32_t *vid;   // exclusive count of visit starts before each rating
    const uint32_t *is_start;
    const uint32_t *vord;  // visit ordinal within its item, per visit id
    const uint32_t *nvis;  // visits per epoch of each item
    int32_t p, rmax, tmax;
    int32_t *rowmap;       // m entries, -1 initially: (chunk << 8) | slot of the row's last chunk
    int64_t *ck_count;     // pass 1 output: chunks per worker
    int64_t *sl_count;     // pass 1 output: slots per worker
    const int64_t *ck_off; // pass 2 input: first chunk of each worker
    const int64_t *sl_off; // pass 2 input: first slot of each worker
    ChunkRec *chunks;      // pass 2 output
    SlotRec *slots;
    RatingRec *ratings;
};

// One thread per worker walks its ratings in processing order and cuts chunks.  A row
// (item) that the next chunk uses again stays in LDS at the same physical slot; the
// other rows and items of a chunk take free physical slots, so a worker needs a single
// staging buffer and never copies within LDS.  Chunks do not carry anything across an
// epoch boundary.
template <bool kFill>
__global__ void k_chunker(ChunkerArgs a) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.p) return;
    const int32_t p = a.p;
    int32_t rid[kMaxSlots], rphys[kMaxSlots], prev_rphys[kMaxSlots];
    int32_t tid[kMaxSlots], tphys[kMaxSlots], tv[kMaxSlots];
    uint8_t rcar[kMaxSlots], tcar[kMaxSlots];
    uint8_t lrs[kMaxRatingsPerChunk], lts[kMaxRatingsPerChunk];
    int64_t c = 0;                   // local index of the open chunk
    const int64_t ck_base = kFill ? a.ck_off[q] : 0;
    int64_t sl_pos = kFill ? a.sl_off[q] : 0;  // next free slot record (global)
    int64_t nslots_local = 0;
    int64_t prev_slot_base = -1;     // slot records of the previous chunk (global index)
    int32_t prev_nr = 0;
    int32_t prev_last_tok = -1, prev_last_tok_slot = -1, prev_last_tok_phys = -1;
    bool prev_same_block = false;
    int32_t nr = 0, nt = 0, nrat = 0;
    int64_t rat0 = 0;
    uint32_t flags = 0;
    int32_t g = 0;
    int32_t cur_tok = -1;

    auto assign = [](int32_t *phys, const uint8_t *car, int32_t count) {
        uint64_t used = 0;
        for (int32_t x = 0; x < count; ++x)
            if (car[x]) used |= 1ull << phys[x];
        for (int32_t x = 0; x < count; ++x) {
            if (car[x]) continue;
            const int32_t slot = __builtin_ctzll(~used);
            phys[x] = slot;
            used |= 1ull << slot;
        }
    };
    auto close_chunk = [&](bool last_of_block) {
        const uint32_t f = flags | (last_of_block ? kLastOfBlock : 0u);
        assign(rphys, rcar, nr);
        assign(tphys, tcar, nt);
        if (kFill) {
            ChunkRec r;
            r.rat = rat0;
            r.slot = sl_pos;
            r.info = (uint32_t)nrat | ((uint32_t)nr << 8) | ((uint32_t)nt << 16) | (f << 24);
            r.group = g;
            r.pad0 = r.pad1 = 0;
            a.chunks[ck_base + c] = r;
            for (int32_t x = 0; x < nr; ++x) {
                SlotRec s;
                s.id = rid[x];
                s.phys = (int16_t)rphys[x];
                s.flags = rcar[x] ? 0 : kSlotNew;
                s.v = 0;
                s.nvis = 0;
                a.slots[sl_pos + x] = s;
            }
            for (int32_t x = 0; x < nt; ++x) {
                SlotRec s;
                s.id = tid[x];
                s.phys = (int16_t)tphys[x];
                s.flags = tcar[x] ? 0 : kSlotNew;
                s.v = tv[x];
                s.nvis = (int32_t)a.nvis[tid[x]];
                a.slots[sl_pos + nr + x] = s;
            }
            for (int32_t x = 0; x < nrat; ++x) {
                RatingRec rr;
                rr.slots = (uint32_t)rphys[lrs[x]] | ((uint32_t)tphys[lts[x]] << 8);
                rr.r = a.sval[rat0 + x];
                a.ratings[rat0 + x] = rr;
            }
        }
        for (int32_t x = 0; x < nr; ++x) prev_rphys[x] = rphys[x];
        prev_slot_base = sl_pos;
        prev_nr = nr;
        prev_last_tok = nt > 0 ? tid[nt - 1] : -1;
        prev_last_tok_slot = nt - 1;
        prev_last_tok_phys = nt > 0 ? tphys[nt - 1] : -1;
        prev_same_block = !last_of_block;
        sl_pos += nr + nt;
        nslots_local += nr + nt;
        ++c;
    };
    auto open_chunk = [&](int64_t first_rating, uint32_t f) {
        nr = nt = nrat = 0;
        rat0 = first_rating;
        flags = f;
        cur_tok = -1;
    };

    for (int32_t s = 0; s < p; ++s) {
        const int64_t b = (int64_t)q * p + s;
        const int64_t f0 = a.bfirst[b], f1 = a.bend[b];
        if (f1 <= f0) continue;
        g = (q + s) % p;
        prev_same_block = false;  // a new block never carries items
        open_chunk(f0, kFirstOfBlock);
        for (int64_t e = f0; e < f1; ++e) {
            const int32_t i = a.srow[e], j = a.scol[e];
            int32_t v = a.rowmap[i];
            bool row_in = v >= 0 && (int64_t)(v >> 8) == c;
            bool tok_new = nt == 0 || j != cur_tok;
            if (nrat == kMaxRatingsPerChunk || (tok_new && nt == a.tmax) || (!row_in && nr == a.rmax)) {
                close_chunk(false);
                open_chunk(e, 0u);
                row_in = false;
                tok_new = true;
            }
            int32_t ts;
            if (tok_new) {
                ts = nt++;
                tid[ts] = j;
                tcar[ts] = 0;
                tphys[ts] = -1;
                tv[ts] = kFill ? (int32_t)a.vord[a.vid[e] + a.is_start[e] - 1u] : 0;
                if (prev_same_block && nrat == 0 && j == prev_last_tok) {
                    tcar[ts] = 1;
                    tphys[ts] = prev_last_tok_phys;
                    if (kFill) a.slots[prev_slot_base + prev_nr + prev_last_tok_slot].flags |= kSlotKeep;
                }
                cur_tok = j;
            } else {
                ts = nt - 1;
            }
            int32_t rs;
            if (!row_in) {
                rs = nr++;
                rid[rs] = i;
                rcar[rs] = 0;
                rphys[rs] = -1;
                if (v >= 0 && c > 0 && (int64_t)(v >> 8) == c - 1) {
                    rcar[rs] = 1;
                    rphys[rs] = prev_rphys[v & 255];
                    if (kFill) a.slots[prev_slot_base + (v & 255)].flags |= kSlotKeep;
                }
                a.rowmap[i] = (int32_t)((c << 8) | rs);
            } else {
                rs = v & 255;
            }
            lrs[nrat] = (uint8_t)rs;
            lts[nrat] = (uint8_t)ts;
            ++nrat;
        }
        close_chunk(true);
    }
    if (!kFill) {
        a.ck_count[q] = c;
        a.sl_count[q] = nslots_local;
    }
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

int bits_for(uint64_t maxval) {
    int b = 1;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b;
}

template <typename T>
hipError_t dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void **)p, count * sizeof(T));
}

}  // namespace

void free_plan(Plan *pl) {
    (void)hipFree(pl->row_start);
    (void)hipFree(pl->wck);
    (void)hipFree(pl->chunks);
    (void)hipFree(pl->slots);
    (void)hipFree(pl->ratings);
    (void)hipFree(pl->nvis);
    *pl = Plan();
}

#define CK(x)                                   \
    do {                                        \
        hipError_t _e = (x);                    \
        if (_e != hipSuccess) { rc = _e; goto done; } \
    } while (0)

hipError_t build_plan(Plan *pl, int64_t m, int64_t n, int64_t nnz, const int32_t *d_row,
                      const int32_t *d_col, const float *d_val, int32_t p, int32_t kp, int32_t rmax,
                      int32_t tmax, uint64_t seed, hipStream_t st, int *err_code, char *msg,
                      size_t msg_len) {
    hipError_t rc = hipSuccess;
    *err_code = 0;
    *pl = Plan();
    pl->m = m; pl->n = n; pl->nnz = nnz; pl->p = p; pl->kp = kp; pl->rmax = rmax; pl->tmax = tmax;

    unsigned long long *deg = nullptr;
    int64_t *rowptr = nullptr, *bfirst = nullptr, *bend = nullptr;
    int64_t *ck_count = nullptr, *sl_count = nullptr, *ck_off = nullptr, *sl_off = nullptr;
    int32_t *err = nullptr, *rowmap = nullptr;
    uint32_t *is_start = nullptr, *vid = nullptr, *vidx = nullptr, *vidx_s = nullptr, *nvis = nullptr,
             *seg = nullptr, *vord = nullptr;
    uint64_t *vkey = nullptr, *vkey_s = nullptr;
    int64_t nvisits = 0;
    uint64_t *key1 = nullptr, *key1s = nullptr;
    uint32_t *idx1 = nullptr, *idx1s = nullptr, *key2 = nullptr, *key2s = nullptr;
    int32_t *srow = nullptr, *scol = nullptr;
    float *sval = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    int32_t h_err = 0;
    const int64_t nb2 = (int64_t)p * p;
    ChunkerArgs ca{};
    int64_t h_tot[2] = {0, 0};

    CK(dalloc(&pl->row_start, p + 1));
    CK(dalloc(&pl->wck, p + 1));
    CK(dalloc(&err, 1));
    CK(hipMemsetAsync(err, 0, sizeof(int32_t), st));
    CK(dalloc(&deg, m + 1));
    CK(dalloc(&rowptr, m + 1));
    CK(hipMemsetAsync(deg, 0, sizeof(unsigned long long) * (m + 1), st));

    // 1-3: degrees, scan, partition
    if (nnz > 0)
        hipLaunchKernelGGL(k_check_degree, dim3(grid_for(nnz)), dim3(kThreads), 0, st, d_row, d_col, nnz,
                           m, n, deg, err);
    CK(hipGetLastError());
    {
        size_t need = 0;
        CK(hipcub::DeviceScan::ExclusiveSum(nullptr, need, (const int64_t *)deg, rowptr, m + 1, st));
        if (need > tmp_bytes) { (void)hipFree(tmp); tmp = nullptr; CK(hipMalloc(&tmp, need)); tmp_bytes = need; }
        CK(hipcub::DeviceScan::ExclusiveSum(tmp, need, (const int64_t *)deg, rowptr, m + 1, st));
    }
    hipLaunchKernelGGL(k_partition, dim3((p + 1 + 63) / 64), dim3(64), 0, st, rowptr, m, nnz, p,
                       pl->row_start);
    CK(hipGetLastError());
    CK(hipMemcpyAsync(&h_err, err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (h_err & 1) {
        *err_code = 1;
        snprintf(msg, msg_len, "rating index out of range (row must be in [0,%lld), column in [0,%lld))",
                 (long long)m, (long long)n);
        goto done;
    }

    // 4: order by (j, i), reject duplicates, then stable order by (q, s)
    CK(dalloc(&key1, nnz)); CK(dalloc(&key1s, nnz));
    CK(dalloc(&idx1, nnz)); CK(dalloc(&idx1s, nnz));
    if (nnz > 0) {
        hipLaunchKernelGGL(k_key_ji, dim3(grid_for(nnz)), dim3(kThreads), 0, st, d_row, d_col, nnz, m,
                           key1, idx1);
        CK(hipGetLastError());
        int eb = bits_for((uint64_t)n * (uint64_t)m);
        size_t need = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, need, key1, key1s, idx1, idx1s, nnz, 0, eb, st));
        if (need > tmp_bytes) { (void)hipFree(tmp); tmp = nullptr; CK(hipMalloc(&tmp, need)); tmp_bytes = need; }
        CK(hipcub::DeviceRadixSort::SortPairs(tmp, need, key1, key1s, idx1, idx1s, nnz, 0, eb, st));
        hipLaunchKernelGGL(k_check_dup, dim3(grid_for(nnz)), dim3(kThreads), 0, st, key1s, nnz, err);
        CK(hipGetLastError());
        CK(hipMemcpyAsync(&h_err, err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        if (h_err & 2) {
            *err_code = 1;
            snprintf(msg, msg_len, "repeated (row, column) pair in the ratings: Omega must be a set");
            goto done;
        }
    }
    (void)hipFree(key1); key1 = nullptr;
    (void)hipFree(key1s); key1s = nullptr;
    (void)hipFree(idx1); idx1 = nullptr;
    CK(dalloc(&key2, nnz)); CK(dalloc(&key2s, nnz));
    if (nnz > 0) {
        hipLaunchKernelGGL(k_key_qs, dim3(grid_for(nnz)), dim3(kThreads), 0, st, idx1s, d_row, d_col, nnz,
                           pl->row_start, p, seed, key2);
        CK(hipGetLastError());
        CK(dalloc(&idx1, nnz));  // reuse as output indices
        int eb = bits_for((uint64_t)nb2 - 1);
        size_t need = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, need, key2, key2s, idx1s, idx1, nnz, 0, eb, st));
        if (need > tmp_bytes) { (void)hipFree(tmp); tmp = nullptr; CK(hipMalloc(&tmp, need)); tmp_bytes = need; }
        CK(hipcub::DeviceRadixSort::SortPairs(tmp, need, key2, key2s, idx1s, idx1, nnz, 0, eb, st));
    }
    (void)hipFree(key2); key2 = nullptr;
    CK(dalloc(&srow, nnz)); CK(dalloc(&scol, nnz)); CK(dalloc(&sval, nnz));
    if (nnz > 0) {
        hipLaunchKernelGGL(k_gather, dim3(grid_for(nnz)), dim3(kThreads), 0, st, idx1, d_row, d_col, d_val,
                           nnz, srow, scol, sval);
        CK(hipGetLastError());
    }
    (void)hipFree(idx1); idx1 = nullptr;
    (void)hipFree(idx1s); idx1s = nullptr;

    // 5: blocks; visits of every item numbered in ring order
    CK(dalloc(&bfirst, nb2)); CK(dalloc(&bend, nb2));
    CK(hipMemsetAsync(bfirst, 0, sizeof(int64_t) * nb2, st));
    CK(hipMemsetAsync(bend, 0, sizeof(int64_t) * nb2, st));
    CK(dalloc(&nvis, n + 1));
    CK(dalloc(&seg, n + 1));
    CK(hipMemsetAsync(nvis, 0, sizeof(uint32_t) * (n + 1), st));
    CK(dalloc(&is_start, nnz)); CK(dalloc(&vid, nnz));
    if (nnz > 0) {
        hipLaunchKernelGGL(k_block_bounds, dim3(grid_for(nnz)), dim3(kThreads), 0, st, key2s, nnz, bfirst,
                           bend);
        CK(hipGetLastError());
        hipLaunchKernelGGL(k_visit_start, dim3(grid_for(nnz)), dim3(kThreads), 0, st, key2s, scol, nnz, is_start);
        CK(hipGetLastError());
        size_t need = 0;
        CK(hipcub::DeviceScan::ExclusiveSum(nullptr, need, is_start, vid, nnz, st));
        if (need > tmp_bytes) { (void)hipFree(tmp); tmp = nullptr; CK(hipMalloc(&tmp, need)); tmp_bytes = need; }
        CK(hipcub::DeviceScan::ExclusiveSum(tmp, need, is_start, vid, nnz, st));
        uint32_t h_last[2] = {0, 0};
        CK(hipMemcpyAsync(&h_last[0], vid + nnz - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        CK(hipMemcpyAsync(&h_last[1], is_start + nnz - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        nvisits = (int64_t)h_last[0] + h_last[1];
    }
    CK(dalloc(&vkey, nvisits)); CK(dalloc(&vkey_s, nvisits));
    CK(dalloc(&vidx, nvisits)); CK(dalloc(&vidx_s, nvisits)); CK(dalloc(&vord, nvisits));
    if (nnz > 0) {
        hipLaunchKernelGGL(k_visit_keys, dim3(grid_for(nnz)), dim3(kThreads), 0, st, is_start, vid, key2s, scol, nnz,
                           p, vkey, vidx, nvis);
        CK(hipGetLastError());
        int eb = bits_for((uint64_t)n * (uint64_t)p);
        size_t need = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, need, vkey, vkey_s, vidx, vidx_s, nvisits, 0, eb, st));
        if (need > tmp_bytes) { (void)hipFree(tmp); tmp = nullptr; CK(hipMalloc(&tmp, need)); tmp_bytes = need; }
        CK(hipcub::DeviceRadixSort::SortPairs(tmp, need, vkey, vkey_s, vidx, vidx_s, nvisits, 0, eb, st));
        need = 0;
        CK(hipcub::DeviceScan::ExclusiveSum(nullptr, need, nvis, seg, n + 1, st));
        if (need > tmp_bytes) { (void)hipFree(tmp); tmp = nullptr; CK(hipMalloc(&tmp, need)); tmp_bytes = need; }
        CK(hipcub::DeviceScan::ExclusiveSum(tmp, need, nvis, seg, n + 1, st));
        hipLaunchKernelGGL(k_visit_ordinal, dim3(grid_for(nvisits)), dim3(kThreads), 0, st, vkey_s, vidx_s, seg,
                           nvisits, p, vord);
        CK(hipGetLastError());
    }
    pl->nvisits = nvisits;
    CK(dalloc(&pl->nvis, n));
    CK(hipMemcpyAsync(pl->nvis, nvis, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st));

    // 6: chunks, two passes
    CK(dalloc(&rowmap, m));
    CK(dalloc(&ck_count, p + 1)); CK(dalloc(&sl_count, p + 1));
    CK(dalloc(&ck_off, p + 1)); CK(dalloc(&sl_off, p + 1));
    CK(hipMemsetAsync(ck_count, 0, sizeof(int64_t) * (p + 1), st));
    CK(hipMemsetAsync(sl_count, 0, sizeof(int64_t) * (p + 1), st));
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(m)), dim3(kThreads), 0, st, rowmap, m, -1);
    ca.srow = srow; ca.scol = scol; ca.sval = sval;
    ca.bfirst = bfirst; ca.bend = bend; ca.vid = vid; ca.is_start = is_start; ca.vord = vord; ca.nvis = nvis;
    ca.p = p; ca.rmax = rmax; ca.tmax = tmax; ca.rowmap = rowmap;
    ca.ck_count = ck_count; ca.sl_count = sl_count;
    hipLaunchKernelGGL(k_chunker<false>, dim3((p + 63) / 64), dim3(64), 0, st, ca);
    CK(hipGetLastError());
    {
        size_t need = 0;
        CK(hipcub::DeviceScan::ExclusiveSum(nullptr, need, ck_count, ck_off, p + 1, st));
        if (need > tmp_bytes) { (void)hipFree(tmp); tmp = nullptr; CK(hipMalloc(&tmp, need)); tmp_bytes = need; }
        CK(hipcub::DeviceScan::ExclusiveSum(tmp, need, ck_count, ck_off, p + 1, st));
        CK(hipcub::DeviceScan::ExclusiveSum(tmp, need, sl_count, sl_off, p + 1, st));
    }
    CK(hipMemcpyAsync(&h_tot[0], ck_off + p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&h_tot[1], sl_off + p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    pl->nchunks = h_tot[0];
    pl->nslots = h_tot[1];
    CK(dalloc(&pl->chunks, pl->nchunks));
    CK(dalloc(&pl->slots, pl->nslots));
    CK(dalloc(&pl->ratings, nnz));
    CK(hipMemcpyAsync(pl->wck, ck_off, sizeof(int64_t) * (p + 1), hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(m)), dim3(kThreads), 0, st, rowmap, m, -1);
    ca.ck_off = ck_off; ca.sl_off = sl_off;
    ca.chunks = pl->chunks; ca.slots = pl->slots; ca.ratings = pl->ratings;
    hipLaunchKernelGGL(k_chunker<true>, dim3((p + 63) / 64), dim3(64), 0, st, ca);
    CK(hipGetLastError());
    CK(hipStreamSynchronize(st));

done:
    (void)hipFree(deg); (void)hipFree(rowptr); (void)hipFree(bfirst); (void)hipFree(bend);
    (void)hipFree(is_start); (void)hipFree(vid); (void)hipFree(vidx); (void)hipFree(vidx_s); (void)hipFree(nvis);
    (void)hipFree(seg); (void)hipFree(vord); (void)hipFree(vkey); (void)hipFree(vkey_s);
    (void)hipFree(ck_count); (void)hipFree(sl_count); (void)hipFree(ck_off); (void)hipFree(sl_off);
    (void)hipFree(err); (void)hipFree(rowmap); (void)hipFree(key1); (void)hipFree(key1s); (void)hipFree(idx1); (void)hipFree(idx1s);
    (void)hipFree(key2); (void)hipFree(key2s); (void)hipFree(srow); (void)hipFree(scol); (void)hipFree(sval); (void)hipFree(tmp);
    if (rc != hipSuccess || *err_code != 0) free_plan(pl);
    return rc;
}

}  // namespace nomad
