// Layout of a problem for the NOMAD workers (runs once inside nomad_init).
//
//   1. check indices, count ratings per row;
//   2. exclusive scan -> rowptr;
//   3. row partition: row_start[q] = min{ i : rowptr[i] >= ceil(q * nnz / p) } (the
//      "same number of ratings" split of section 3.1, footnote), then the same rule
//      inside each worker's block for its compute waves;
//   4. order the ratings by (worker q, ring sub-step s = (g(j) - q) mod p, item j, row i)
//      with two stable radix sorts (first by (j, i), then by (q, s)); a repeated (i, j)
//      is rejected (Omega is a set);
//   5. visits (maximal runs of one (worker, item)) numbered in ring order per item, and
//      per worker in processing order;
//   6. per rating: the visit information its wave needs (visit index, first / last rating
//      of the wave in the visit, the wave before it in the visit); per visit: item,
//      ordinal, visits of the item per epoch, last wave;
//   7. the ratings of each wave gathered into one stream, in processing order (a stable
//      sort by (worker, wave));
//   8. in each wave's stream, the ratings whose row is used again within the next D
//      ratings (the rows a wave keeps in flight): those rows are handed on on chip.
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

#define GRID_LOOP(e, n) \
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (n); e += (int64_t)gridDim.x * blockDim.x)

__global__ void k_check_degree(const int32_t *row, const int32_t *col, int64_t nnz, int64_t m,
                               int64_t n, unsigned long long *deg, int32_t *err) {
    GRID_LOOP(e, nnz) {
        int32_t i = row[e], j = col[e];
        if (i < 0 || i >= m || j < 0 || j >= n) {
            atomicOr(err, 1);
            continue;
        }
        atomicAdd(&deg[i], 1ull);
    }
}

// Smallest i in [lo, hi] with rowptr[i] >= target (rowptr is non-decreasing).
__device__ inline int64_t lower_row(const int64_t *rowptr, int64_t lo, int64_t hi, int64_t target) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (rowptr[mid] >= target) hi = mid; else lo = mid + 1;
    }
    return lo;
}

__global__ void k_partition(const int64_t *rowptr, int64_t m, int64_t nnz, int32_t p,
                            int64_t *row_start) {
    int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q > p) return;
    if (q == 0) { row_start[0] = 0; return; }
    if (q == p) { row_start[p] = m; return; }
    const int64_t target = ((int64_t)q * nnz + p - 1) / p;
    row_start[q] = lower_row(rowptr, 0, m, target);
}

// Wave w of worker q starts at the smallest row i of the block with
// #ratings in [row_start[q], i) >= ceil(w * nnz_q / nw).
__global__ void k_wave_partition(const int64_t *rowptr, const int64_t *row_start, int64_t m, int32_t p,
                                 int32_t nw, int64_t *wave_start) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t > (int64_t)p * nw) return;
    if (t == (int64_t)p * nw) { wave_start[t] = m; return; }
    const int32_t q = (int32_t)(t / nw), w = (int32_t)(t % nw);
    const int64_t r0 = row_start[q], r1 = row_start[q + 1];
    const int64_t base = rowptr[r0], nq = rowptr[r1] - base;
    const int64_t target = base + ((int64_t)w * nq + nw - 1) / nw;
    wave_start[t] = lower_row(rowptr, r0, r1, target);
}

// Largest index t in [0, cnt) with bounds[t] <= i.
__device__ inline int32_t find_block(const int64_t *bounds, int32_t cnt, int64_t i) {
    int32_t lo = 0, hi = cnt - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (bounds[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void k_key_ji(const int32_t *row, const int32_t *col, int64_t nnz, int64_t m,
                         uint64_t *key, uint32_t *idx) {
    GRID_LOOP(e, nnz) {
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
    GRID_LOOP(e, nnz) {
        uint32_t x = idx[e];
        int32_t q = find_block(row_start, p, row[x]);
        int32_t g = item_group(seed, col[x], p);
        int32_t s = (g - q + p) % p;
        key[e] = (uint32_t)q * (uint32_t)p + (uint32_t)s;
    }
}

__global__ void k_gather(const uint32_t *idx, const int32_t *row, const int32_t *col,
                         const float *val, int64_t nnz, int32_t *srow, int32_t *scol, float *sval) {
    GRID_LOOP(e, nnz) {
        uint32_t x = idx[e];
        srow[e] = row[x];
        scol[e] = col[x];
        sval[e] = val[x];
    }
}

// Visits: maximal runs of one (worker, item) in the (q, s, j, i) order.
__global__ void k_visit_start(const uint32_t *key2, const int32_t *scol, int64_t nnz, uint32_t *is_start) {
    GRID_LOOP(e, nnz)
        is_start[e] = (e == 0 || key2[e] != key2[e - 1] || scol[e] != scol[e - 1]) ? 1u : 0u;
}

// For each visit (at its first rating e): sort key (item, sub-step) and the visit id.
__global__ void k_visit_keys(const uint32_t *is_start, const uint32_t *vid, const uint32_t *key2,
                             const int32_t *scol, int64_t nnz, int32_t p, uint64_t *vkey, uint32_t *vidx,
                             uint32_t *nvis) {
    GRID_LOOP(e, nnz) {
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
    GRID_LOOP(t, nv) {
        const uint64_t j = vkey_sorted[t] / (uint64_t)p;
        vord[vidx_sorted[t]] = (uint32_t)(t - seg[j]);
    }
}

// First visit of each worker: the visit of its first rating in the sorted order (the
// next worker's first visit if it has no ratings).
__global__ void k_visit_base(const int64_t *rowptr, const int64_t *row_start, const uint32_t *vid, int64_t nnz,
                             int64_t nvisits, int32_t p, int64_t *vbase) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q > p) return;
    const int64_t e = rowptr[row_start[q]];
    vbase[q] = (q < p && e < nnz) ? (int64_t)vid[e] : nvisits;
}

// Rating records and visit records.
__global__ void k_records(const int32_t *srow, const int32_t *scol, const float *sval, const uint32_t *key2,
                          const uint32_t *is_start, const uint32_t *vid, const uint32_t *vord, const uint32_t *nvis,
                          const int64_t *vbase, const int64_t *wave_start, int64_t nnz, int32_t p, int32_t nw,
                          RatingRec *rec, VisitRec *visits, uint32_t *key3) {
    GRID_LOOP(e, nnz) {
        const int32_t q = (int32_t)(key2[e] / (uint32_t)p);
        const int64_t *ws = wave_start + (int64_t)q * nw;
        const int32_t w = find_block(ws, nw, srow[e]);
        const uint32_t v = vid[e] + is_start[e] - 1u;  // global visit id
        const bool next_start = e + 1 == nnz || is_start[e + 1];
        const bool first = is_start[e] || find_block(ws, nw, srow[e - 1]) != w;
        const bool last = next_start || find_block(ws, nw, srow[e + 1]) != w;
        const uint32_t prev = (first && !is_start[e]) ? (uint32_t)find_block(ws, nw, srow[e - 1]) + 1u : 0u;
        const uint32_t x = (uint32_t)((int64_t)v - vbase[q]);
        RatingRec r;
        r.row = srow[e];
        r.r = sval[e];
        r.info = x | (first ? kInfoFirst : 0u) | (last ? kInfoLast : 0u) | (prev << kInfoPrevShift);
        r.fwd = 0;
        rec[e] = r;
        key3[e] = (uint32_t)q * (uint32_t)nw + (uint32_t)w;
        if (is_start[e]) {
            visits[v].j = scol[e];
            visits[v].v = vord[v];
            visits[v].nvis = nvis[scol[e]];
        }
        if (next_start) visits[v].lastw = w;
    }
}

// Rows used again inside the window: for every rating of a wave's stream (taken
// cyclically, as the stream repeats every epoch) the distance back to the previous rating
// of the same row if it is below D, and the matching forward distance at that earlier
// rating.  One thread per wave; the rows of a wave are its own, so `last` (m entries, -1 on
// entry) is shared without conflicts.
__global__ void k_forward(RatingRec *recs, const int64_t *rbase, int64_t nwt, int32_t D, int64_t *last) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nwt) return;
    RatingRec *r = recs + rbase[t];
    const int64_t cnt = rbase[t + 1] - rbase[t];
    for (int64_t p = 0; p < 2 * cnt; ++p) {
        const int64_t pos = p < cnt ? p : p - cnt;
        const int32_t row = r[pos].row;
        if (p >= cnt) {
            const int64_t prev = last[row];
            const int64_t d = p - prev;
            if (prev >= 0 && d < D) {
                r[pos].fwd |= (uint32_t)d << 8;
                const int64_t src = pos - d >= 0 ? pos - d : pos - d + cnt;
                r[src].fwd |= (uint32_t)d;
            }
        }
        last[row] = p;
    }
    for (int64_t p = 0; p < cnt; ++p) last[r[p].row] = -1;
}

__global__ void k_count_keys(const uint32_t *key, int64_t nnz, unsigned long long *cnt) {
    GRID_LOOP(e, nnz) atomicAdd(&cnt[key[e]], 1ull);
}

__global__ void k_permute_recs(const uint32_t *idx, const RatingRec *in, int64_t nnz, RatingRec *out) {
    GRID_LOOP(e, nnz) out[e] = in[idx[e]];
}

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v) {
    GRID_LOOP(e, n) p[e] = v;
}

__global__ void k_iota(uint32_t *p, int64_t n) {
    GRID_LOOP(e, n) p[e] = (uint32_t)e;
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

// Temporary storage of the hipCUB calls, grown on demand.
struct Tmp {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t need(size_t b) {
        if (b <= bytes) return hipSuccess;
        (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, b);
        if (e == hipSuccess) bytes = b;
        return e;
    }
    ~Tmp() { (void)hipFree(p); }
};

// Worker of each visit, and the visit's item as a sort key.
__global__ void k_visit_owner(const int64_t *vbase, int32_t p, const VisitRec *visits, int64_t nv, int32_t *vq,
                              uint32_t *vj, uint32_t *vidx) {
    GRID_LOOP(v, nv) {
        vq[v] = find_block(vbase, p, v);
        vj[v] = (uint32_t)visits[v].j;
        vidx[v] = (uint32_t)v;
    }
}

// Ratings of each visit (worker q's local item x = visit vbase[q] + x).
__global__ void k_visit_ratings(const RatingRec *recs, int64_t nnz, const int64_t *rbase, int64_t nwt, int32_t nw,
                                const int64_t *vbase, unsigned int *vcnt) {
    GRID_LOOP(e, nnz) {
        const int32_t t = find_block(rbase, (int32_t)nwt, e);
        const int32_t q = t / nw;
        atomicAdd(&vcnt[vbase[q] + (int64_t)(recs[e].info & kInfoXMask)], 1u);
    }
}

// Holder entries in (item, worker) order, and the number of holders of each item.
__global__ void k_holders(const uint32_t *vidx_sorted, const int32_t *vq, const int64_t *vbase, const VisitRec *visits,
                          const unsigned int *vcnt, int64_t nv, int32_t *hold, int32_t *hx, int32_t *hitem,
                          int32_t *hcnt, unsigned long long *cnt) {
    GRID_LOOP(i, nv) {
        const int64_t v = vidx_sorted[i];
        const int32_t q = vq[v];
        hold[i] = q;
        hx[i] = (int32_t)(v - vbase[q]);
        hitem[i] = visits[v].j;
        hcnt[i] = (int32_t)vcnt[v];
        atomicAdd(&cnt[visits[v].j], 1ull);
    }
}

__global__ void k_count_active(const int64_t *hoff, int64_t n, unsigned long long *active) {
    GRID_LOOP(j, n) {
        if (hoff[j + 1] > hoff[j]) atomicAdd(active, 1ull);
    }
}

// xoff at the first record of each (visit, wave): every record that starts its wave's part
// of a visit.
__global__ void k_xoff_first(const RatingRec *recs, int64_t nnz, const int64_t *rbase, int64_t nwt, int32_t nw,
                             const int64_t *vbase, int32_t *xoff) {
    GRID_LOOP(e, nnz) {
        const uint32_t info = recs[e].info;
        if (!(info & kInfoFirst)) continue;
        const int32_t t = find_block(rbase, (int32_t)nwt, e);
        const int32_t q = t / nw, w = t - q * nw;
        const int64_t v = vbase[q] + (int64_t)(info & kInfoXMask);
        xoff[v * nw + w] = (int32_t)(e - rbase[t]);
    }
}

// Visits without records in a wave start where the wave's next visit does (one thread per
// wave, backwards over its worker's visits).
__global__ void k_xoff_fill(const int64_t *rbase, int64_t nwt, int32_t nw, const int64_t *vbase, int32_t *xoff) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nwt) return;
    const int32_t q = (int32_t)(t / nw), w = (int32_t)(t - (int64_t)q * nw);
    int32_t next = (int32_t)(rbase[t + 1] - rbase[t]);
    for (int64_t v = vbase[q + 1] - 1; v >= vbase[q]; --v) {
        int32_t &o = xoff[v * nw + w];
        if (o < 0) o = next;
        else next = o;
    }
}

// Sort key of each visit in the ring order of an epoch: sub-step s = (g(j) - q) mod p, then
// worker q (a worker's visits are already in (s, j) order, which a stable sort keeps).
__global__ void k_visit_ring_key(const int64_t *vbase, int32_t p, const VisitRec *visits, int64_t nv, uint64_t seed,
                                 uint32_t *key, uint32_t *vidx) {
    GRID_LOOP(v, nv) {
        const int32_t q = find_block(vbase, p, v);
        const int32_t g = item_group(seed, visits[v].j, p);
        const int32_t sub = g >= q ? g - q : g - q + p;
        key[v] = (uint32_t)sub * (uint32_t)p + (uint32_t)q;
        vidx[v] = (uint32_t)v;
    }
}

__global__ void k_gather_counts(const uint32_t *vidx_sorted, const unsigned int *vcnt, int64_t nv, int64_t *out) {
    GRID_LOOP(i, nv) out[i] = (int64_t)vcnt[vidx_sorted[i]];
}

__global__ void k_scatter_starts(const uint32_t *vidx_sorted, const int64_t *pos, int64_t nv, int64_t *vstart) {
    GRID_LOOP(i, nv) vstart[vidx_sorted[i]] = pos[i];
}

// Holder map of uniform routing: hmap[q * n + j] = the holder entry of (q, j).
__global__ void k_holder_map(const int32_t *hold, const int32_t *hitem, int64_t nv, int64_t n, int32_t *hmap) {
    GRID_LOOP(g, nv) hmap[(int64_t)hold[g] * n + hitem[g]] = (int32_t)g;
}

}  // namespace

void free_plan(Plan *pl) {
    (void)hipFree(pl->vstart);
    (void)hipFree(pl->hmap);
    (void)hipFree(pl->row_start);
    (void)hipFree(pl->wave_start);
    (void)hipFree(pl->rbase);
    (void)hipFree(pl->recs);
    (void)hipFree(pl->vbase);
    (void)hipFree(pl->visits);
    (void)hipFree(pl->hold);
    (void)hipFree(pl->hx);
    (void)hipFree(pl->hitem);
    (void)hipFree(pl->hcnt);
    (void)hipFree(pl->hoff);
    (void)hipFree(pl->xoff);
    *pl = Plan();
}

#define CK(x)                                   \
    do {                                        \
        hipError_t _e = (x);                    \
        if (_e != hipSuccess) { rc = _e; goto done; } \
    } while (0)

hipError_t build_async_tables(Plan *pl, hipStream_t st) {
    hipError_t rc = hipSuccess;
    const int64_t nv = pl->nvisits, n = pl->n, nwt = (int64_t)pl->p * pl->nw;
    int32_t *vq = nullptr;
    uint32_t *vj = nullptr, *vj_s = nullptr, *vidx = nullptr, *vidx_s = nullptr;
    unsigned long long *cnt = nullptr, *act = nullptr;
    unsigned int *vcnt = nullptr;
    Tmp tmp;
    CK(dalloc(&pl->hold, nv > 0 ? nv : 1));
    CK(dalloc(&pl->hx, nv > 0 ? nv : 1));
    CK(dalloc(&pl->hitem, nv > 0 ? nv : 1));
    CK(dalloc(&pl->hcnt, nv > 0 ? nv : 1));
    CK(dalloc(&pl->hoff, n + 1));
    CK(dalloc(&pl->xoff, nv * pl->nw > 0 ? nv * pl->nw : 1));
    CK(dalloc(&cnt, n + 1));
    CK(dalloc(&act, 1));
    CK(hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * (n + 1), st));
    CK(hipMemsetAsync(act, 0, sizeof(unsigned long long), st));
    if (nv > 0) {
        CK(dalloc(&vq, nv)); CK(dalloc(&vj, nv)); CK(dalloc(&vj_s, nv)); CK(dalloc(&vidx, nv)); CK(dalloc(&vidx_s, nv));
        CK(dalloc(&vcnt, nv));
        CK(hipMemsetAsync(vcnt, 0, sizeof(unsigned int) * nv, st));
        if (pl->nnz > 0) {
            hipLaunchKernelGGL(k_visit_ratings, dim3(grid_for(pl->nnz)), dim3(kThreads), 0, st, pl->recs, pl->nnz,
                               pl->rbase, nwt, pl->nw, pl->vbase, vcnt);
            CK(hipGetLastError());
        }
        hipLaunchKernelGGL(k_visit_owner, dim3(grid_for(nv)), dim3(kThreads), 0, st, pl->vbase, pl->p, pl->visits,
                           nv, vq, vj, vidx);
        CK(hipGetLastError());
        const int eb = bits_for((uint64_t)(n > 1 ? n - 1 : 1));
        size_t need = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, need, vj, vj_s, vidx, vidx_s, nv, 0, eb, st));
        CK(tmp.need(need));
        CK(hipcub::DeviceRadixSort::SortPairs(tmp.p, need, vj, vj_s, vidx, vidx_s, nv, 0, eb, st));
        hipLaunchKernelGGL(k_holders, dim3(grid_for(nv)), dim3(kThreads), 0, st, vidx_s, vq, pl->vbase, pl->visits,
                           vcnt, nv, pl->hold, pl->hx, pl->hitem, pl->hcnt, cnt);
        CK(hipGetLastError());
    }
    {
        size_t need = 0;
        CK(hipcub::DeviceScan::ExclusiveSum(nullptr, need, (const int64_t *)cnt, pl->hoff, n + 1, st));
        CK(tmp.need(need));
        CK(hipcub::DeviceScan::ExclusiveSum(tmp.p, need, (const int64_t *)cnt, pl->hoff, n + 1, st));
    }
    hipLaunchKernelGGL(k_count_active, dim3(grid_for(n)), dim3(kThreads), 0, st, pl->hoff, n, act);
    CK(hipGetLastError());
    if (nv > 0) {
        CK(hipMemsetAsync(pl->xoff, 0xFF, sizeof(int32_t) * nv * pl->nw, st));
        if (pl->nnz > 0) {
            hipLaunchKernelGGL(k_xoff_first, dim3(grid_for(pl->nnz)), dim3(kThreads), 0, st, pl->recs, pl->nnz,
                               pl->rbase, nwt, pl->nw, pl->vbase, pl->xoff);
            CK(hipGetLastError());
        }
        hipLaunchKernelGGL(k_xoff_fill, dim3(grid_for(nwt, 64)), dim3(64), 0, st, pl->rbase, nwt, pl->nw, pl->vbase,
                           pl->xoff);
        CK(hipGetLastError());
    }
    {
        unsigned long long a = 0;
        CK(hipMemcpyAsync(&a, act, sizeof(a), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        pl->active = (int64_t)a;
    }
done:
    (void)hipFree(vq); (void)hipFree(vj); (void)hipFree(vj_s); (void)hipFree(vidx); (void)hipFree(vidx_s);
    (void)hipFree(cnt); (void)hipFree(act); (void)hipFree(vcnt);
    return rc;
}

hipError_t build_visit_starts(Plan *pl, uint64_t seed, hipStream_t st) {
    hipError_t rc = hipSuccess;
    const int64_t nv = pl->nvisits, nwt = (int64_t)pl->p * pl->nw;
    unsigned int *vcnt = nullptr;
    uint32_t *key = nullptr, *key_s = nullptr, *vidx = nullptr, *vidx_s = nullptr;
    int64_t *cnt = nullptr, *pos = nullptr;
    Tmp tmp;
    CK(dalloc(&pl->vstart, nv));
    if (nv > 0) {
        CK(dalloc(&vcnt, nv)); CK(dalloc(&key, nv)); CK(dalloc(&key_s, nv)); CK(dalloc(&vidx, nv));
        CK(dalloc(&vidx_s, nv)); CK(dalloc(&cnt, nv)); CK(dalloc(&pos, nv));
        CK(hipMemsetAsync(vcnt, 0, sizeof(unsigned int) * nv, st));
        if (pl->nnz > 0) {
            hipLaunchKernelGGL(k_visit_ratings, dim3(grid_for(pl->nnz)), dim3(kThreads), 0, st, pl->recs, pl->nnz,
                               pl->rbase, nwt, pl->nw, pl->vbase, vcnt);
            CK(hipGetLastError());
        }
        hipLaunchKernelGGL(k_visit_ring_key, dim3(grid_for(nv)), dim3(kThreads), 0, st, pl->vbase, pl->p, pl->visits,
                           nv, seed, key, vidx);
        CK(hipGetLastError());
        const int kb = bits_for((uint64_t)pl->p * (uint64_t)pl->p);
        size_t need = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, need, key, key_s, vidx, vidx_s, nv, 0, kb, st));
        CK(tmp.need(need));
        CK(hipcub::DeviceRadixSort::SortPairs(tmp.p, need, key, key_s, vidx, vidx_s, nv, 0, kb, st));
        hipLaunchKernelGGL(k_gather_counts, dim3(grid_for(nv)), dim3(kThreads), 0, st, vidx_s, vcnt, nv, cnt);
        CK(hipGetLastError());
        need = 0;
        CK(hipcub::DeviceScan::ExclusiveSum(nullptr, need, (const int64_t *)cnt, pos, nv, st));
        CK(tmp.need(need));
        CK(hipcub::DeviceScan::ExclusiveSum(tmp.p, need, (const int64_t *)cnt, pos, nv, st));
        hipLaunchKernelGGL(k_scatter_starts, dim3(grid_for(nv)), dim3(kThreads), 0, st, vidx_s, pos, nv, pl->vstart);
        CK(hipGetLastError());
        CK(hipStreamSynchronize(st));
    }
done:
    (void)hipFree(vcnt); (void)hipFree(key); (void)hipFree(key_s); (void)hipFree(vidx); (void)hipFree(vidx_s);
    (void)hipFree(cnt); (void)hipFree(pos);
    return rc;
}

hipError_t build_holder_map(Plan *pl, hipStream_t st) {
    hipError_t rc = hipSuccess;
    const size_t cells = (size_t)pl->p * (size_t)pl->n;
    CK(dalloc(&pl->hmap, cells));
    CK(hipMemsetAsync(pl->hmap, 0xFF, sizeof(int32_t) * cells, st));
    if (pl->nvisits > 0) {
        hipLaunchKernelGGL(k_holder_map, dim3(grid_for(pl->nvisits)), dim3(kThreads), 0, st, pl->hold, pl->hitem,
                           pl->nvisits, pl->n, pl->hmap);
        CK(hipGetLastError());
    }
done:
    return rc;
}

// Ratings per row (rows outside [0, m) are skipped here; the layout reports them).
__global__ void k_row_count(const int32_t *row, int64_t nnz, int64_t m, uint32_t *cnt) {
    GRID_LOOP(e, nnz) {
        const int32_t i = row[e];
        if (i >= 0 && i < m) atomicAdd(&cnt[i], 1u);
    }
}

hipError_t max_row_degree(const int32_t *d_row, int64_t nnz, int64_t m, hipStream_t st, int64_t *out) {
    *out = 0;
    if (m <= 0 || nnz <= 0) return hipSuccess;
    uint32_t *cnt = nullptr;
    void *tmp = nullptr;
    size_t need = 0;
    uint32_t h_max = 0;
    hipError_t e = hipMalloc(&cnt, sizeof(uint32_t) * (size_t)m);
    if (e == hipSuccess) e = hipMemsetAsync(cnt, 0, sizeof(uint32_t) * (size_t)m, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_row_count, dim3(grid_for(nnz)), dim3(kThreads), 0, st, d_row, nnz, m, cnt);
        e = hipGetLastError();
    }
    uint32_t *none = nullptr;
    if (e == hipSuccess) e = hipcub::DeviceReduce::Max(nullptr, need, cnt, none, m, st);
    const size_t off = (need + 255) & ~(size_t)255;
    if (e == hipSuccess) e = hipMalloc(&tmp, off + sizeof(uint32_t));
    if (e == hipSuccess) e = hipcub::DeviceReduce::Max(tmp, need, cnt, (uint32_t *)((char *)tmp + off), m, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&h_max, (char *)tmp + off, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(tmp);
    (void)hipFree(cnt);
    if (e == hipSuccess) *out = (int64_t)h_max;
    return e;
}

hipError_t build_plan(Plan *pl, int64_t m, int64_t n, int64_t nnz, const int32_t *d_row, const int32_t *d_col,
                      const float *d_val, int32_t p, int32_t nw, int32_t window, uint64_t seed, hipStream_t st,
                      int *err_code, char *msg, size_t msg_len) {
    hipError_t rc = hipSuccess;
    *err_code = 0;
    *pl = Plan();
    pl->m = m; pl->n = n; pl->nnz = nnz; pl->p = p; pl->nw = nw;

    Tmp tmp;
    unsigned long long *deg = nullptr, *kcount = nullptr;
    int64_t *rowptr = nullptr;
    int32_t *err = nullptr;
    uint32_t *is_start = nullptr, *vid = nullptr, *vidx = nullptr, *vidx_s = nullptr, *nvis = nullptr,
             *seg = nullptr, *vord = nullptr;
    uint64_t *vkey = nullptr, *vkey_s = nullptr;
    int64_t nvisits = 0;
    uint64_t *key1 = nullptr, *key1s = nullptr;
    uint32_t *idx1 = nullptr, *idx1s = nullptr, *key2 = nullptr, *key2s = nullptr, *key3 = nullptr,
             *key3s = nullptr, *idx3 = nullptr, *idx3s = nullptr;
    int32_t *srow = nullptr, *scol = nullptr;
    float *sval = nullptr;
    RatingRec *rec0 = nullptr;
    int32_t h_err = 0;
    const int64_t nb2 = (int64_t)p * p;
    const int64_t nwt = (int64_t)p * nw;

    CK(dalloc(&pl->row_start, p + 1));
    CK(dalloc(&pl->wave_start, nwt + 1));
    CK(dalloc(&pl->rbase, nwt + 1));
    CK(dalloc(&pl->vbase, p + 1));
    CK(dalloc(&err, 1));
    CK(hipMemsetAsync(err, 0, sizeof(int32_t), st));
    CK(dalloc(&deg, m + 1));
    CK(dalloc(&rowptr, m + 1));
    CK(hipMemsetAsync(deg, 0, sizeof(unsigned long long) * (m + 1), st));

    // 1-3: degrees, scan, partitions
    if (nnz > 0)
        hipLaunchKernelGGL(k_check_degree, dim3(grid_for(nnz)), dim3(kThreads), 0, st, d_row, d_col, nnz,
                           m, n, deg, err);
    CK(hipGetLastError());
    {
        size_t need = 0;
        CK(hipcub::DeviceScan::ExclusiveSum(nullptr, need, (const int64_t *)deg, rowptr, m + 1, st));
        CK(tmp.need(need));
        CK(hipcub::DeviceScan::ExclusiveSum(tmp.p, need, (const int64_t *)deg, rowptr, m + 1, st));
    }
    if (m > 0) {
        // the largest row degree (read when the asynchronous kernel's variant is chosen)
        size_t need = 0;
        unsigned long long *none = nullptr;
        CK(hipcub::DeviceReduce::Max(nullptr, need, deg, none, m, st));
        const size_t off = (need + 255) & ~(size_t)255;
        CK(tmp.need(off + sizeof(unsigned long long)));
        unsigned long long *d_max = (unsigned long long *)((char *)tmp.p + off);
        CK(hipcub::DeviceReduce::Max(tmp.p, need, deg, d_max, m, st));
        unsigned long long h_max = 0;
        CK(hipMemcpyAsync(&h_max, d_max, sizeof(h_max), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        pl->max_row_degree = (int64_t)h_max;
    }
    hipLaunchKernelGGL(k_partition, dim3((p + 1 + 63) / 64), dim3(64), 0, st, rowptr, m, nnz, p, pl->row_start);
    CK(hipGetLastError());
    hipLaunchKernelGGL(k_wave_partition, dim3(grid_for(nwt + 1)), dim3(kThreads), 0, st, rowptr, pl->row_start, m,
                       p, nw, pl->wave_start);
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
        hipLaunchKernelGGL(k_key_ji, dim3(grid_for(nnz)), dim3(kThreads), 0, st, d_row, d_col, nnz, m, key1, idx1);
        CK(hipGetLastError());
        const int eb = bits_for((uint64_t)n * (uint64_t)m);
        size_t need = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, need, key1, key1s, idx1, idx1s, nnz, 0, eb, st));
        CK(tmp.need(need));
        CK(hipcub::DeviceRadixSort::SortPairs(tmp.p, need, key1, key1s, idx1, idx1s, nnz, 0, eb, st));
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
        CK(dalloc(&idx1, nnz));  // output indices
        const int eb = bits_for((uint64_t)nb2 - 1);
        size_t need = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, need, key2, key2s, idx1s, idx1, nnz, 0, eb, st));
        CK(tmp.need(need));
        CK(hipcub::DeviceRadixSort::SortPairs(tmp.p, need, key2, key2s, idx1s, idx1, nnz, 0, eb, st));
    }
    (void)hipFree(key2); key2 = nullptr;
    CK(dalloc(&srow, nnz)); CK(dalloc(&scol, nnz)); CK(dalloc(&sval, nnz));
    if (nnz > 0) {
        hipLaunchKernelGGL(k_gather, dim3(grid_for(nnz)), dim3(kThreads), 0, st, idx1, d_row, d_col, d_val, nnz,
                           srow, scol, sval);
        CK(hipGetLastError());
    }
    (void)hipFree(idx1); idx1 = nullptr;
    (void)hipFree(idx1s); idx1s = nullptr;

    // 5: visits of every item numbered in ring order
    CK(dalloc(&nvis, n + 1));
    CK(dalloc(&seg, n + 1));
    CK(hipMemsetAsync(nvis, 0, sizeof(uint32_t) * (n + 1), st));
    CK(dalloc(&is_start, nnz)); CK(dalloc(&vid, nnz));
    if (nnz > 0) {
        hipLaunchKernelGGL(k_visit_start, dim3(grid_for(nnz)), dim3(kThreads), 0, st, key2s, scol, nnz, is_start);
        CK(hipGetLastError());
        size_t need = 0;
        CK(hipcub::DeviceScan::ExclusiveSum(nullptr, need, is_start, vid, nnz, st));
        CK(tmp.need(need));
        CK(hipcub::DeviceScan::ExclusiveSum(tmp.p, need, is_start, vid, nnz, st));
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
        const int eb = bits_for((uint64_t)n * (uint64_t)p);
        size_t need = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, need, vkey, vkey_s, vidx, vidx_s, nvisits, 0, eb, st));
        CK(tmp.need(need));
        CK(hipcub::DeviceRadixSort::SortPairs(tmp.p, need, vkey, vkey_s, vidx, vidx_s, nvisits, 0, eb, st));
        need = 0;
        CK(hipcub::DeviceScan::ExclusiveSum(nullptr, need, nvis, seg, n + 1, st));
        CK(tmp.need(need));
        CK(hipcub::DeviceScan::ExclusiveSum(tmp.p, need, nvis, seg, n + 1, st));
        hipLaunchKernelGGL(k_visit_ordinal, dim3(grid_for(nvisits)), dim3(kThreads), 0, st, vkey_s, vidx_s, seg,
                           nvisits, p, vord);
        CK(hipGetLastError());
    }
    (void)hipFree(vkey); vkey = nullptr;
    (void)hipFree(vkey_s); vkey_s = nullptr;
    (void)hipFree(vidx); vidx = nullptr;
    (void)hipFree(vidx_s); vidx_s = nullptr;
    pl->nvisits = nvisits;
    hipLaunchKernelGGL(k_visit_base, dim3((p + 1 + 63) / 64), dim3(64), 0, st, rowptr, pl->row_start, vid, nnz,
                       nvisits, p, pl->vbase);
    CK(hipGetLastError());

    // 6: records
    CK(dalloc(&pl->visits, nvisits));
    CK(dalloc(&rec0, nnz));
    CK(dalloc(&key3, nnz));
    if (nnz > 0) {
        hipLaunchKernelGGL(k_records, dim3(grid_for(nnz)), dim3(kThreads), 0, st, srow, scol, sval, key2s, is_start,
                           vid, vord, nvis, pl->vbase, pl->wave_start, nnz, p, nw, rec0, pl->visits, key3);
        CK(hipGetLastError());
    }
    (void)hipFree(srow); srow = nullptr;
    (void)hipFree(scol); scol = nullptr;
    (void)hipFree(sval); sval = nullptr;
    (void)hipFree(key2s); key2s = nullptr;
    (void)hipFree(is_start); is_start = nullptr;
    (void)hipFree(vid); vid = nullptr;

    // 7: one stream per wave
    CK(dalloc(&kcount, nwt + 1));
    CK(hipMemsetAsync(kcount, 0, sizeof(unsigned long long) * (nwt + 1), st));
    CK(dalloc(&pl->recs, nnz));
    if (nnz > 0) {
        hipLaunchKernelGGL(k_count_keys, dim3(grid_for(nnz)), dim3(kThreads), 0, st, key3, nnz, kcount);
        CK(hipGetLastError());
        CK(dalloc(&key3s, nnz)); CK(dalloc(&idx3, nnz)); CK(dalloc(&idx3s, nnz));
        hipLaunchKernelGGL(k_iota, dim3(grid_for(nnz)), dim3(kThreads), 0, st, idx3, nnz);
        CK(hipGetLastError());
        const int eb = bits_for((uint64_t)(nwt > 1 ? nwt - 1 : 1));
        size_t need = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, need, key3, key3s, idx3, idx3s, nnz, 0, eb, st));
        CK(tmp.need(need));
        CK(hipcub::DeviceRadixSort::SortPairs(tmp.p, need, key3, key3s, idx3, idx3s, nnz, 0, eb, st));
        hipLaunchKernelGGL(k_permute_recs, dim3(grid_for(nnz)), dim3(kThreads), 0, st, idx3s, rec0, nnz, pl->recs);
        CK(hipGetLastError());
    }
    {
        size_t need = 0;
        CK(hipcub::DeviceScan::ExclusiveSum(nullptr, need, (const int64_t *)kcount, pl->rbase, nwt + 1, st));
        CK(tmp.need(need));
        CK(hipcub::DeviceScan::ExclusiveSum(tmp.p, need, (const int64_t *)kcount, pl->rbase, nwt + 1, st));
    }
    if (nnz > 0) {
        int64_t *last = nullptr;
        CK(dalloc(&last, m));
        hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(m)), dim3(kThreads), 0, st, last, m, (int64_t)-1);
        hipLaunchKernelGGL(k_forward, dim3(grid_for(nwt, 64)), dim3(64), 0, st, pl->recs, pl->rbase, nwt, window,
                           last);
        hipError_t fe = hipGetLastError();
        if (fe == hipSuccess) fe = hipStreamSynchronize(st);
        (void)hipFree(last);
        CK(fe);
    }
    {
        std::vector<int64_t> vb(p + 1);
        CK(hipMemcpyAsync(vb.data(), pl->vbase, sizeof(int64_t) * (p + 1), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        int64_t mx = 0;
        for (int32_t q = 0; q < p; ++q) mx = vb[q + 1] - vb[q] > mx ? vb[q + 1] - vb[q] : mx;
        pl->max_worker_visits = mx;
        if (mx > (int64_t)kInfoXMask) {
            *err_code = 5;
            snprintf(msg, msg_len, "a worker has %lld visits per epoch; at most %u are supported", (long long)mx,
                     kInfoXMask);
            goto done;
        }
    }

done:
    (void)hipFree(deg); (void)hipFree(kcount); (void)hipFree(rowptr); (void)hipFree(err);
    (void)hipFree(is_start); (void)hipFree(vid); (void)hipFree(vidx); (void)hipFree(vidx_s); (void)hipFree(nvis);
    (void)hipFree(seg); (void)hipFree(vord); (void)hipFree(vkey); (void)hipFree(vkey_s);
    (void)hipFree(key1); (void)hipFree(key1s); (void)hipFree(idx1); (void)hipFree(idx1s);
    (void)hipFree(key2); (void)hipFree(key2s); (void)hipFree(key3); (void)hipFree(key3s); (void)hipFree(idx3);
    (void)hipFree(idx3s); (void)hipFree(srow); (void)hipFree(scol); (void)hipFree(sval); (void)hipFree(rec0);
    if (rc != hipSuccess || *err_code != 0) free_plan(pl);
    return rc;
}

}  // namespace nomad
