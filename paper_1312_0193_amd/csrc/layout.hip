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
//   6. plan each worker's chunks and LDS slots (planner.h) in two passes: count, then
//      fill.
#include <hipcub/hipcub.hpp>

#include <cstdio>
#include <cstring>
#include <vector>

#include "nomad_internal.h"
#include "planner.h"

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

// Per-rating visit information for the planner: v | nvis << 16 (the visit's ordinal
// among the item's visits in one epoch of the ring order, and the item's visits per epoch).
__global__ void k_vinfo(const uint32_t *vid, const uint32_t *is_start, const uint32_t *vord, const uint32_t *nvis,
                        const int32_t *scol, int64_t nnz, uint32_t *vinfo) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        vinfo[e] = vord[vid[e] + is_start[e] - 1u] | (nvis[scol[e]] << 16);
}

// First rating of each worker in the (q, s, j, i) order: rowptr at its first row.
__global__ void k_worker_first(const int64_t *rowptr, const int64_t *row_start, int32_t p, int64_t *wfirst) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q <= p) wfirst[q] = rowptr[row_start[q]];
}

// One thread per worker runs the planner (planner.h): count pass, then fill pass.
template <bool kFill>
__global__ void k_planner(PlanIn in, const int64_t *wfirst, PlanOut base, const int64_t *ck_off,
                          const int64_t *ev_off, int64_t *ck_count, int64_t *ev_count, int64_t *ld_count,
                          int32_t *err, int32_t p) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= p) return;
    PlanOut o = base;
    if (kFill) {
        o.ck0 = ck_off[q];
        o.ev0 = ev_off[q];
    }
    const PlanCount r = plan_worker<kFill>(in, wfirst[q], wfirst[q + 1], o);
    if (r.status) atomicOr(err, 4);
    if (!kFill) {
        ck_count[q] = r.chunks;
        ev_count[q] = r.events;
        ld_count[q] = r.loads;
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
    (void)hipFree(pl->events);
    (void)hipFree(pl->ratings);
    *pl = Plan();
}

#define CK(x)                                   \
    do {                                        \
        hipError_t _e = (x);                    \
        if (_e != hipSuccess) { rc = _e; goto done; } \
    } while (0)

hipError_t build_plan(Plan *pl, int64_t m, int64_t n, int64_t nnz, const int32_t *d_row,
                      const int32_t *d_col, const float *d_val, int32_t p, int32_t kp, int32_t slots,
                      int32_t loads, uint64_t seed, hipStream_t st, int *err_code, char *msg,
                      size_t msg_len) {
    hipError_t rc = hipSuccess;
    *err_code = 0;
    *pl = Plan();
    pl->m = m; pl->n = n; pl->nnz = nnz; pl->p = p; pl->kp = kp; pl->slots = slots; pl->loads = loads;

    unsigned long long *deg = nullptr;
    int64_t *rowptr = nullptr;
    int64_t *ck_count = nullptr, *ev_count = nullptr, *ld_count = nullptr, *ck_off = nullptr, *ev_off = nullptr;
    int64_t *wfirst = nullptr;
    int32_t *err = nullptr, *rowmap = nullptr, *nxt = nullptr;
    uint32_t *vinfo = nullptr;
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
    PlanIn pin{};
    PlanOut pout{};
    int64_t h_tot[3] = {0, 0, 0};

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

    // 6: per-worker plans, two passes
    CK(dalloc(&vinfo, nnz));
    CK(dalloc(&nxt, nnz));
    CK(dalloc(&rowmap, m));
    CK(dalloc(&wfirst, p + 1));
    CK(dalloc(&ck_count, p + 1)); CK(dalloc(&ev_count, p + 1)); CK(dalloc(&ld_count, p + 1));
    CK(dalloc(&ck_off, p + 1)); CK(dalloc(&ev_off, p + 1));
    CK(hipMemsetAsync(ck_count, 0, sizeof(int64_t) * (p + 1), st));
    CK(hipMemsetAsync(ev_count, 0, sizeof(int64_t) * (p + 1), st));
    CK(hipMemsetAsync(ld_count, 0, sizeof(int64_t) * (p + 1), st));
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(m)), dim3(kThreads), 0, st, rowmap, m, -1);
    hipLaunchKernelGGL(k_worker_first, dim3((p + 1 + 63) / 64), dim3(64), 0, st, rowptr, pl->row_start, p, wfirst);
    CK(hipGetLastError());
    if (nnz > 0) {
        hipLaunchKernelGGL(k_vinfo, dim3(grid_for(nnz)), dim3(kThreads), 0, st, vid, is_start, vord, nvis, scol, nnz,
                           vinfo);
        CK(hipGetLastError());
    }
    pin.srow = srow; pin.scol = scol; pin.sval = sval; pin.blk = key2s; pin.vinfo = vinfo;
    pin.slots = slots; pin.cap = loads; pin.look = kLookahead; pin.nxt = nxt; pin.rowmap = rowmap;
    hipLaunchKernelGGL(k_planner<false>, dim3((p + 63) / 64), dim3(64), 0, st, pin, wfirst, pout, ck_off, ev_off,
                       ck_count, ev_count, ld_count, err, p);
    CK(hipGetLastError());
    {
        size_t need = 0;
        CK(hipcub::DeviceScan::ExclusiveSum(nullptr, need, ck_count, ck_off, p + 1, st));
        if (need > tmp_bytes) { (void)hipFree(tmp); tmp = nullptr; CK(hipMalloc(&tmp, need)); tmp_bytes = need; }
        CK(hipcub::DeviceScan::ExclusiveSum(tmp, need, ck_count, ck_off, p + 1, st));
        CK(hipcub::DeviceScan::ExclusiveSum(tmp, need, ev_count, ev_off, p + 1, st));
    }
    CK(hipMemcpyAsync(&h_tot[0], ck_off + p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&h_tot[1], ev_off + p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(&h_err, err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (h_err & 4) {
        *err_code = 1;
        snprintf(msg, msg_len, "%d LDS slots per worker are too few", slots);
        goto done;
    }
    {
        std::vector<int64_t> lc(p + 1);
        CK(hipMemcpy(lc.data(), ld_count, sizeof(int64_t) * (p + 1), hipMemcpyDeviceToHost));
        int64_t t = 0;
        for (int32_t q = 0; q < p; ++q) t += lc[q];
        pl->nloads = t;
    }
    pl->nchunks = h_tot[0];
    pl->nevents = h_tot[1];
    CK(dalloc(&pl->chunks, pl->nchunks));
    CK(dalloc(&pl->events, pl->nevents));
    CK(dalloc(&pl->ratings, nnz));
    CK(hipMemcpyAsync(pl->wck, ck_off, sizeof(int64_t) * (p + 1), hipMemcpyDeviceToDevice, st));
    pout.chunks = pl->chunks; pout.events = pl->events; pout.ratings = pl->ratings;
    hipLaunchKernelGGL(k_planner<true>, dim3((p + 63) / 64), dim3(64), 0, st, pin, wfirst, pout, ck_off, ev_off,
                       ck_count, ev_count, ld_count, err, p);
    CK(hipGetLastError());
    CK(hipStreamSynchronize(st));

done:
    (void)hipFree(deg); (void)hipFree(rowptr);
    (void)hipFree(is_start); (void)hipFree(vid); (void)hipFree(vidx); (void)hipFree(vidx_s); (void)hipFree(nvis);
    (void)hipFree(seg); (void)hipFree(vord); (void)hipFree(vkey); (void)hipFree(vkey_s);
    (void)hipFree(ck_count); (void)hipFree(ev_count); (void)hipFree(ld_count); (void)hipFree(ck_off);
    (void)hipFree(ev_off); (void)hipFree(wfirst); (void)hipFree(vinfo); (void)hipFree(nxt);
    (void)hipFree(err); (void)hipFree(rowmap); (void)hipFree(key1); (void)hipFree(key1s); (void)hipFree(idx1); (void)hipFree(idx1s);
    (void)hipFree(key2); (void)hipFree(key2s); (void)hipFree(srow); (void)hipFree(scol); (void)hipFree(sval); (void)hipFree(tmp);
    if (rc != hipSuccess || *err_code != 0) free_plan(pl);
    return rc;
}

}  // namespace nomad
