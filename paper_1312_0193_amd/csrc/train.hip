// NOMAD worker kernel: one wavefront = one worker (Algorithm 1), persistent for a whole
// nomad_train_epochs call.
//
// Worker q walks its chunks in plan order, epoch after epoch.  Before a chunk uses an
// item h_j that it does not carry over from the previous chunk, it waits until item j
// has finished every earlier visit in the ring order (a per-item counter of finished
// visits reaches this visit's ticket), which makes worker q the sole owner of h_j
// (owner-computes rule, section 3.1).  The chunk's rows w_i and items h_j are staged in
// LDS, the SGD updates of section 2.3 run over the chunk's ratings in plan order on LDS,
// and an item leaving LDS is written back and passed on by advancing its counter.
//
// Software pipeline (per iteration x, one chunk; one LDS staging area per worker):
//   top    wait for the memory traffic issued in iteration x-1; pass on the items chunk
//          x-1 finished with (written back right after its updates); write back chunk
//          x-1's rows that chunk x does not keep in their LDS slots; write chunk x's
//          prefetched vectors (registers) into their LDS slots.  If some of chunk x was
//          not prefetched (an item not yet free when polled, or the first chunk of an
//          epoch), wait for its items and load what is missing;
//   issue  prefetch chunk x+1 into registers (rows; its new items too when they were
//          seen free), records of chunk x+3, ratings of chunk x+2, and poll the counters
//          of the items chunk x+2 takes over;
//   sgd    the updates of chunk x on LDS, no global memory access; then the items the
//          next chunk does not keep are written back (device-coherent) so that the next
//          top can pass them on.
// A worker that blocks has already passed on every item it finished with, which keeps
// the ring order free of waiting cycles.
//
// Memory ordering of a hand-off: item vectors are written with device-coherent stores
// (agent scope, sc1) and the counter is advanced with a device-coherent store only after
// "s_waitcnt vmcnt(0)" has seen those stores complete; the next owner polls the counter
// with device-coherent loads and reads the item with device-coherent loads.  Rows w_i
// are private to their worker (always the same wavefront, hence the same CU and XCD) and
// use ordinary cached loads and stores; a wavefront's own accesses to one address are
// performed in program order.
#include <cmath>
#include <utility>

#include "nomad_internal.h"

namespace nomad {
namespace {

#define DPP_F(x, ctrl, rm, bc) \
    __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, (x)), (ctrl), (rm), 0xF, (bc)))

__device__ __forceinline__ int rl_i(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ float rl_f(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// Sum over the wavefront of x; lanes beyond the active 16-lane rows must hold 0.
// Row-wise butterfly with DPP, then row broadcasts toward lane 63 (or 31 / 15).
template <int NR16>
__device__ __forceinline__ float wave_sum(float x) {
    x += DPP_F(x, 0xB1, 0xF, true);   // quad_perm [1,0,3,2]
    x += DPP_F(x, 0x4E, 0xF, true);   // quad_perm [2,3,0,1]
    x += DPP_F(x, 0x124, 0xF, true);  // row_ror 4
    x += DPP_F(x, 0x128, 0xF, true);  // row_ror 8
    if constexpr (NR16 == 1) return rl_f(x, 15);
    x += DPP_F(x, 0x142, 0xA, false); // row_bcast 15 into rows 1 and 3
    if constexpr (NR16 == 2) return rl_f(x, 31);
    x += DPP_F(x, 0x143, 0xC, false); // row_bcast 31 into rows 2 and 3
    return rl_f(x, 63);
}

template <int VEC>
__device__ __forceinline__ void lds_read(const float *p, float (&v)[VEC]) {
    if constexpr (VEC == 1) { v[0] = p[0]; }
    if constexpr (VEC == 2) { float2 t = *(const float2 *)p; v[0] = t.x; v[1] = t.y; }
    if constexpr (VEC == 4) { float4 t = *(const float4 *)p; v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w; }
}
template <int VEC>
__device__ __forceinline__ void lds_write(float *p, const float (&v)[VEC]) {
    if constexpr (VEC == 1) { p[0] = v[0]; }
    if constexpr (VEC == 2) { *(float2 *)p = make_float2(v[0], v[1]); }
    if constexpr (VEC == 4) { *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]); }
}



// Seconds-scale bound on any single wait, so that a broken schedule ends the kernel
// instead of hanging the device (100 MHz constant clock).
constexpr uint64_t kWaitLimitTicks = 20ull * 100000000ull;

// Slot records of one chunk, one per lane (rows first, then items): global id,
// phys | flags << 16, and for items the visit ordinal and visits per epoch.
struct Recs {
    int id, pf, v, nvis;
};
__device__ __forceinline__ int rec_phys(int pf) { return (int)(int16_t)(pf & 0xffff); }
__device__ __forceinline__ bool rec_new(int pf) { return ((pf >> 16) & kSlotNew) != 0; }
__device__ __forceinline__ bool rec_keep(int pf) { return ((pf >> 16) & kSlotKeep) != 0; }

__device__ __forceinline__ Recs load_recs(const SlotRec *g, int count, int lane) {
    Recs r{0, 0, 0, 0};
    if (lane < count) {
        const int4 v = *(const int4 *)(g + lane);
        r.id = v.x;
        r.pf = v.y;
        r.v = v.z;
        r.nvis = v.w;
    }
    return r;
}

// Staging geometry: a vector of kp floats is lpr = kp / 4 lanes of 16 bytes; one step
// moves rpi = 64 / lpr vectors, lane l handling piece l % lpr of vector l / lpr.
struct Geo {
    int kp, lpr, rpi, vb, piece;
    bool act;
};
__device__ __forceinline__ Geo make_geo(int kp, int lane) {
    Geo g;
    g.kp = kp;
    g.lpr = kp >> 2;
    g.rpi = 64 / g.lpr;
    g.vb = lane / g.lpr;
    g.piece = lane - g.vb * g.lpr;
    g.act = g.vb < g.rpi;
    return g;
}

// This lane's value of a per-slot record field for vector vb of the step at `base`.
__device__ __forceinline__ int slot_val(int field, int base, const Geo &g) {
    if (g.rpi <= 4) {
        int out = __builtin_amdgcn_readlane(field, base);
        for (int b = 1; b < g.rpi; ++b) {
            const int v = __builtin_amdgcn_readlane(field, base + b);
            out = g.vb == b ? v : out;
        }
        return out;
    }
    return __shfl(field, (base + g.vb) & 63);
}

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint64_t u64x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4_t coherent_load4(const float *p) {
    u64x2_t v;
    v.x = __hip_atomic_load((const uint64_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    v.y = __hip_atomic_load((const uint64_t *)p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(f32x4_t, v);
}
__device__ __forceinline__ void coherent_store4(float *p, f32x4_t v) {
    const u64x2_t u = __builtin_bit_cast(u64x2_t, v);
    __hip_atomic_store((uint64_t *)p, u.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store((uint64_t *)p + 1, u.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void wait_all() { asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory"); }

// Register staging of one chunk: step i of the rows holds vectors [rpi i, rpi i + rpi).
struct Staging {
    f32x4_t row[kRowPiecesPerLane];
    f32x4_t item[kItemPiecesPerLane];
};

struct ChunkMeta {
    int64_t rat, slot;
    int nrat, nr, nt;
    int group;
    int epoch;
    bool epoch_start;
};

// Position of a chunk in the worker's cyclic walk: chunk index and epoch.
struct Cursor {
    int64_t c;
    int epoch;
};
__device__ __forceinline__ Cursor advance(Cursor u, int64_t nck) {
    if (++u.c == nck) {
        u.c = 0;
        ++u.epoch;
    }
    return u;
}
__device__ __forceinline__ ChunkMeta chunk_meta(const TrainArgs &a, int64_t c0, Cursor u) {
    const ChunkRec r = a.chunks[c0 + u.c];
    ChunkMeta m;
    m.rat = r.rat;
    m.slot = r.slot;
    m.nrat = r.info & 255;
    m.nr = (r.info >> 8) & 255;
    m.nt = (r.info >> 16) & 255;
    m.group = r.group;
    m.epoch = u.epoch;
    m.epoch_start = u.c == 0;
    return m;
}

__device__ __forceinline__ int item_lane_field(int field, int nr, int lane) { return __shfl(field, (lane + nr) & 63); }

// Counter value at which this chunk's visit of an item may start.
__device__ __forceinline__ uint32_t item_ticket(const ChunkMeta &m, int v, int nvis) {
    return (uint32_t)((int64_t)m.epoch * nvis + v);
}

// Plan validation: a malformed plan (ids or slots out of range) ends the kernel instead
// of letting a load or a store touch memory outside the factors or the staging area.
__device__ __forceinline__ bool recs_ok(const TrainArgs &a, const ChunkMeta &m, const Recs &r, int lane) {
    bool bad = m.nr > a.rmax || m.nt > a.tmax || m.nrat > kMaxRatingsPerChunk || m.nrat < 1;
    if (lane < m.nr + m.nt) {
        const bool is_row = lane < m.nr;
        const int ph = rec_phys(r.pf);
        bad |= r.id < 0 || r.id >= (is_row ? a.m : a.n) || ph < 0 || ph >= (is_row ? a.rmax : a.tmax);
    }
    return __builtin_amdgcn_ballot_w64(bad) == 0;
}
__device__ __forceinline__ bool ratings_ok(const TrainArgs &a, const ChunkMeta &m, const RatingRec &rr, int lane) {
    bool bad = false;
    if (lane < m.nrat) bad = (int)(rr.slots & 255) >= a.rmax || (int)(rr.slots >> 8) >= a.tmax;
    return __builtin_amdgcn_ballot_w64(bad) == 0;
}

// Load into registers the new rows / items of chunk m (rows with plain loads, items with
// device-coherent loads).  Steps use literal indices so the staging stays in registers.
template <int I>
__device__ __forceinline__ void prefetch_row_step(const TrainArgs &a, const ChunkMeta &m, const Recs &r,
                                                  Staging &st, const Geo &g) {
    const int base = g.rpi * I;
    if (base < m.nr) {
        const int id = slot_val(r.id, base, g), pf = slot_val(r.pf, base, g);
        if (g.act && base + g.vb < m.nr && rec_new(pf))
            st.row[I] = *(const f32x4_t *)(a.W + (int64_t)id * g.kp + g.piece * 4);
    }
}
template <int I>
__device__ __forceinline__ void prefetch_item_step(const TrainArgs &a, const ChunkMeta &m, const Recs &r,
                                                   Staging &st, const Geo &g) {
    const int base = g.rpi * I;
    if (base < m.nt) {
        const int id = slot_val(r.id, m.nr + base, g), pf = slot_val(r.pf, m.nr + base, g);
        if (g.act && base + g.vb < m.nt && rec_new(pf))
            st.item[I] = coherent_load4(a.H + (int64_t)id * g.kp + g.piece * 4);
    }
}
template <int... I, int... J>
__device__ __forceinline__ void prefetch_steps(const TrainArgs &a, const ChunkMeta &m, const Recs &r, Staging &st,
                                               const Geo &g, bool rows, bool items,
                                               std::integer_sequence<int, I...>, std::integer_sequence<int, J...>) {
    if (rows) (prefetch_row_step<I>(a, m, r, st, g), ...);
    if (items) (prefetch_item_step<J>(a, m, r, st, g), ...);
}
__device__ __forceinline__ void prefetch(const TrainArgs &a, const ChunkMeta &m, const Recs &r, Staging &st,
                                         const Geo &g, bool rows, bool items) {
    prefetch_steps(a, m, r, st, g, rows, items, std::make_integer_sequence<int, kRowPiecesPerLane>(),
                   std::make_integer_sequence<int, kItemPiecesPerLane>());
}

// Write staged vectors into their LDS slots (same predicate as prefetch).
template <int I>
__device__ __forceinline__ void commit_row_step(const ChunkMeta &m, const Recs &r, const Staging &st, float *lds,
                                                const Geo &g) {
    const int base = g.rpi * I;
    if (base < m.nr) {
        const int pf = slot_val(r.pf, base, g);
        if (g.act && base + g.vb < m.nr && rec_new(pf))
            *(f32x4_t *)(lds + rec_phys(pf) * g.kp + g.piece * 4) = st.row[I];
    }
}
template <int I>
__device__ __forceinline__ void commit_item_step(const ChunkMeta &m, const Recs &r, const Staging &st, float *lds,
                                                 int rmax, const Geo &g) {
    const int base = g.rpi * I;
    if (base < m.nt) {
        const int pf = slot_val(r.pf, m.nr + base, g);
        if (g.act && base + g.vb < m.nt && rec_new(pf))
            *(f32x4_t *)(lds + (rmax + rec_phys(pf)) * g.kp + g.piece * 4) = st.item[I];
    }
}
template <int... I, int... J>
__device__ __forceinline__ void commit_steps(const ChunkMeta &m, const Recs &r, const Staging &st, float *lds, int rmax,
                                             const Geo &g, bool rows, bool items, std::integer_sequence<int, I...>,
                                             std::integer_sequence<int, J...>) {
    if (rows) (commit_row_step<I>(m, r, st, lds, g), ...);
    if (items) (commit_item_step<J>(m, r, st, lds, rmax, g), ...);
}
__device__ __forceinline__ void commit(const ChunkMeta &m, const Recs &r, const Staging &st, float *lds, int rmax,
                                       const Geo &g, bool rows, bool items) {
    commit_steps(m, r, st, lds, rmax, g, rows, items, std::make_integer_sequence<int, kRowPiecesPerLane>(),
                 std::make_integer_sequence<int, kItemPiecesPerLane>());
}

// Store chunk m's rows that the next chunk does not keep (or all of them).
__device__ __forceinline__ void write_back_rows(const TrainArgs &a, const ChunkMeta &m, const Recs &r,
                                                const float *lds, const Geo &g, bool all) {
    for (int base = 0; base < m.nr; base += g.rpi) {
        const int id = slot_val(r.id, base, g), pf = slot_val(r.pf, base, g);
        if (g.act && base + g.vb < m.nr && (all || !rec_keep(pf)))
            *(f32x4_t *)(a.W + (int64_t)id * g.kp + g.piece * 4) =
                *(const f32x4_t *)(lds + rec_phys(pf) * g.kp + g.piece * 4);
    }
}

// Store chunk m's items that the next chunk does not keep (or all), device-coherent.
__device__ __forceinline__ void write_back_items(const TrainArgs &a, const ChunkMeta &m, const Recs &r,
                                                 const float *lds, const Geo &g, bool all) {
    for (int base = 0; base < m.nt; base += g.rpi) {
        const int id = slot_val(r.id, m.nr + base, g), pf = slot_val(r.pf, m.nr + base, g);
        if (g.act && base + g.vb < m.nt && (all || !rec_keep(pf)))
            coherent_store4(a.H + (int64_t)id * g.kp + g.piece * 4,
                            *(const f32x4_t *)(lds + (a.rmax + rec_phys(pf)) * g.kp + g.piece * 4));
    }
}

// Items of chunk m passed on after its write back (lane t = item slot t): id in those
// lanes, -1 elsewhere; *tk = the counter value to publish.
__device__ __forceinline__ int leaving_items(const ChunkMeta &m, const Recs &r, bool all, int lane, uint32_t *tk) {
    const int id = item_lane_field(r.id, m.nr, lane), pf = item_lane_field(r.pf, m.nr, lane);
    const int v = item_lane_field(r.v, m.nr, lane), nv = item_lane_field(r.nvis, m.nr, lane);
    *tk = item_ticket(m, v, nv) + 1u;
    return (lane < m.nt && (all || !rec_keep(pf))) ? id : -1;
}

// Items chunk m takes over (not kept by its predecessor): id in those lanes, -1 elsewhere;
// *tk = the counter value to wait for.
__device__ __forceinline__ int new_items(const ChunkMeta &m, const Recs &r, int lane, uint32_t *tk) {
    const int id = item_lane_field(r.id, m.nr, lane), pf = item_lane_field(r.pf, m.nr, lane);
    const int v = item_lane_field(r.v, m.nr, lane), nv = item_lane_field(r.nvis, m.nr, lane);
    *tk = item_ticket(m, v, nv);
    return (lane < m.nt && rec_new(pf)) ? id : -1;
}

__device__ __forceinline__ void publish(uint32_t *tok, int id, uint32_t tk) {
    if (id >= 0) __hip_atomic_store(tok + id, tk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t poll_items(const uint32_t *tok, int id) {
    return id >= 0 ? __hip_atomic_load(tok + id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
}

// Block until every lane's item counter equals its ticket; false if the kernel must end.
__device__ __forceinline__ bool acquire_items(uint32_t *tok, int id, uint32_t tk, uint32_t *abort_flag) {
    bool pending = id >= 0 && __hip_atomic_load(tok + id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != tk;
    if (__builtin_amdgcn_ballot_w64(pending) == 0) return true;
    const uint64_t t0 = wall_clock64();
    while (true) {
        __builtin_amdgcn_s_sleep(2);
        if (pending) pending = __hip_atomic_load(tok + id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != tk;
        if (__builtin_amdgcn_ballot_w64(pending) == 0) return true;
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (wall_clock64() - t0 > kWaitLimitTicks) {
            __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
}

// SGD over the chunk's ratings in plan order, on LDS.  The next rating's row (and item,
// when it changes) is read ahead; a read-ahead row equal to the current one takes the
// freshly updated value.  Lanes beyond the vector width compute on zeros and write to a
// scratch line of LDS.
template <int VEC, int NR16>
__device__ __forceinline__ void sgd_chunk(float *buf, float *dump, int kp, int rmax, const RatingRec &rr, int nrat,
                                          float s, float shrink, int lane) {
    const bool on = lane * VEC < kp;
    const int roff = on ? lane * VEC : 0;
    float *const wbase = on ? buf + lane * VEC : dump + lane * VEC;  // write address base
    const int r_sl = (int)rr.slots;
    const float r_val = rr.r;
    int sl = rl_i(r_sl, 0);
    float r = rl_f(r_val, 0);
    int rs = sl & 255, ts = sl >> 8;
    float w[VEC], h[VEC];
    lds_read<VEC>(buf + rs * kp + roff, w);
    lds_read<VEC>(buf + (rmax + ts) * kp + roff, h);
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        w[v] = on ? w[v] : 0.0f;
        h[v] = on ? h[v] : 0.0f;
    }
    for (int x = 0; x < nrat; ++x) {
        const int xn = x + 1 < nrat ? x + 1 : x;
        const int sln = rl_i(r_sl, xn);
        const float rn = rl_f(r_val, xn);
        const int rsn = sln & 255, tsn = sln >> 8;
        const bool switch_item = tsn != ts;
        float wn[VEC], hn[VEC];
        lds_read<VEC>(buf + rsn * kp + roff, wn);
        if (switch_item) lds_read<VEC>(buf + (rmax + tsn) * kp + roff, hn);
        float d = 0.0f;
#pragma unroll
        for (int v = 0; v < VEC; ++v) d = fmaf(w[v], h[v], d);
        d = wave_sum<NR16>(d);
        const float se = s * (r - d);
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const float wv = w[v], hv = h[v];
            w[v] = fmaf(se, hv, shrink * wv);
            h[v] = fmaf(se, wv, shrink * hv);
        }
        lds_write<VEC>(wbase + rs * kp, w);
        if (x + 1 == nrat) {
            lds_write<VEC>(wbase + (rmax + ts) * kp, h);
            break;
        }
        if (switch_item) {
            lds_write<VEC>(wbase + (rmax + ts) * kp, h);
#pragma unroll
            for (int v = 0; v < VEC; ++v) h[v] = on ? hn[v] : 0.0f;
        }
        if (rsn != rs) {
#pragma unroll
            for (int v = 0; v < VEC; ++v) w[v] = on ? wn[v] : 0.0f;
        }
        rs = rsn;
        ts = tsn;
        r = rn;
    }
}

__device__ __forceinline__ void raise_abort(uint32_t *abort_flag, uint32_t code, int lane) {
    wait_all();
    if (lane == 0) __hip_atomic_store(abort_flag, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void record_visits(const TrainArgs &a, int q, const ChunkMeta &m, int id, uint32_t tk) {
    if (id < 0) return;
    const int64_t slot = (int64_t)atomicAdd((unsigned long long *)a.trace_len, 1ull);
    if (slot < a.trace_cap) {
        a.trace[4 * slot + 0] = q;
        a.trace[4 * slot + 1] = id;
        a.trace[4 * slot + 2] = m.epoch;
        a.trace[4 * slot + 3] = (int32_t)tk;
    }
}

// Clock read only when per-worker counters are requested.
__device__ __forceinline__ uint64_t tick(bool on) { return on ? wall_clock64() : 0; }

template <int VEC, int NR16>
__global__ __launch_bounds__(64) void k_train(TrainArgs a, uint32_t *abort_flag) {
    extern __shared__ float4 lds4[];
    const int q = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t c0 = a.wck[q], c1 = a.wck[q + 1];
    const int64_t nck = c1 - c0;
    if (nck <= 0 || a.epochs <= 0) return;
    const int kp = a.kp, rmax = a.rmax;
    const Geo geo = make_geo(kp, lane);
    float *const lds = reinterpret_cast<float *>(lds4);
    float *const dump = lds + (a.rmax + a.tmax) * kp;
    const int64_t total = nck * (int64_t)a.epochs;
    const bool prof = a.wstats != nullptr;
    const uint64_t t_start = tick(prof);
    uint64_t t_acq = 0, t_mem = 0, t_sgd = 0, t_issue = 0, t_stage = 0, n_rat = 0;
    uint32_t *const tok = a.tok_done;

    // Prologue: metadata of chunks 0..3, records of chunks 0..2, ratings of chunks 0, 1.
    Cursor u0{0, a.epoch0};
    const Cursor u1 = advance(u0, nck), u2 = advance(u1, nck), u3 = advance(u2, nck);
    ChunkMeta m0 = chunk_meta(a, c0, u0);
    ChunkMeta m1 = chunk_meta(a, c0, u1);
    ChunkMeta m2 = chunk_meta(a, c0, u2);
    ChunkMeta m3 = chunk_meta(a, c0, u3);
    Cursor u4 = advance(u3, nck);
    Recs r0 = load_recs(a.slots + m0.slot, m0.nr + m0.nt, lane);
    Recs r1 = load_recs(a.slots + m1.slot, m1.nr + m1.nt, lane);
    Recs r2 = load_recs(a.slots + m2.slot, m2.nr + m2.nt, lane);
    RatingRec rr0{0, 0.0f}, rr1{0, 0.0f};
    if (lane < m0.nrat) rr0 = a.ratings[m0.rat + lane];
    if (lane < m1.nrat) rr1 = a.ratings[m1.rat + lane];
    wait_all();
    if (!recs_ok(a, m0, r0, lane) || !ratings_ok(a, m0, rr0, lane) || !recs_ok(a, m1, r1, lane) ||
        !recs_ok(a, m2, r2, lane)) {
        raise_abort(abort_flag, 2u, lane);
        return;
    }
    Staging st;
    bool staged_rows = false, staged_items = false;  // chunk m0's new vectors are in `st`
    uint32_t poll = 0;                                // lane t: counter of chunk m1's new item t
    bool polled = false;
    {
        uint32_t tk;
        const int id = new_items(m1, r1, lane, &tk);
        poll = poll_items(tok, id);
        polled = true;
    }
    int pend_id = -1;  // items written back in the previous iteration, to be passed on
    uint32_t pend_tk = 0;
    ChunkMeta mp = m0;  // chunk it-1
    Recs rp = r0;
    int s_epoch = -1;
    float s_step = 0.0f, s_shrink = 1.0f;

    for (int64_t it = 0; it < total; ++it) {
        const bool has_next = it + 1 < total, has_next2 = it + 2 < total, has_next3 = it + 3 < total;
        const ChunkMeta m4 = chunk_meta(a, c0, u4);  // used from the next iteration on

        // ---- top
        const uint64_t t_top = tick(prof);
        wait_all();
        const uint64_t t_s0 = tick(prof);
        t_mem += t_s0 - t_top;
        publish(tok, pend_id, pend_tk);
        pend_id = -1;
        if (it > 0 && (!ratings_ok(a, m0, rr0, lane) || (has_next2 && !recs_ok(a, m2, r2, lane)))) {
            raise_abort(abort_flag, 2u, lane);
            return;
        }
        if (it > 0) write_back_rows(a, mp, rp, lds, geo, false);
        if (!staged_rows || !staged_items) {
            // Everything this worker could pass on was passed on above; wait for the
            // items and load what was not prefetched.
            uint32_t tk;
            const int id = new_items(m0, r0, lane, &tk);
            const uint64_t t_a = tick(prof);
            if (!staged_items && !acquire_items(tok, id, tk, abort_flag)) {
                wait_all();
                return;
            }
            prefetch(a, m0, r0, st, geo, !staged_rows, !staged_items);
            wait_all();
            t_acq += tick(prof) - t_a;
            if (a.trace && !staged_items) record_visits(a, q, m0, id, tk);
        }
        commit(m0, r0, st, lds, rmax, geo, true, true);
        if (a.trace && staged_items) {
            uint32_t tk;
            const int id = new_items(m0, r0, lane, &tk);
            record_visits(a, q, m0, id, tk);
        }
        const uint64_t t_i0 = tick(prof);
        t_stage += t_i0 - t_s0;

        // ---- issue: prefetch chunk it+1 (not across an epoch boundary), records it+3,
        //      ratings it+2, poll the counters of chunk it+2's new items
        bool staged_rows1 = false, staged_items1 = false;
        if (has_next && !m1.epoch_start) {
            uint32_t tk;
            const int id = new_items(m1, r1, lane, &tk);
            staged_rows1 = true;
            staged_items1 = __builtin_amdgcn_ballot_w64(id >= 0 && !(polled && poll == tk)) == 0;
            prefetch(a, m1, r1, st, geo, true, staged_items1);
        }
        Recs r3 = r2;
        if (has_next3) r3 = load_recs(a.slots + m3.slot, m3.nr + m3.nt, lane);
        RatingRec rr2 = rr1;
        if (has_next2 && lane < m2.nrat) rr2 = a.ratings[m2.rat + lane];
        bool polled2 = false;
        uint32_t poll2 = 0;
        if (has_next2) {
            uint32_t tk;
            const int id = new_items(m2, r2, lane, &tk);
            poll2 = poll_items(tok, id);
            polled2 = true;
        }

        // ---- sgd on chunk it
        const uint64_t t_g0 = tick(prof);
        t_issue += t_g0 - t_i0;
        if (m0.epoch != s_epoch) {
            s_epoch = m0.epoch;
            s_step = (float)(a.alpha / (1.0 + a.beta * pow((double)s_epoch, a.gamma)));
            s_shrink = 1.0f - s_step * a.lambda;
        }
        sgd_chunk<VEC, NR16>(lds, dump, kp, rmax, rr0, m0.nrat, s_step, s_shrink, lane);
        t_sgd += tick(prof) - t_g0;
        n_rat += m0.nrat;
        // Items chunk it is done with leave now; they are passed on at the next top.
        write_back_items(a, m0, r0, lds, geo, !has_next);
        pend_id = leaving_items(m0, r0, !has_next, lane, &pend_tk);

        mp = m0;
        rp = r0;
        m0 = m1;
        r0 = r1;
        rr0 = rr1;
        m1 = m2;
        r1 = r2;
        rr1 = rr2;
        m2 = m3;
        r2 = r3;
        m3 = m4;
        u4 = advance(u4, nck);
        poll = poll2;
        polled = polled2;
        staged_rows = staged_rows1;
        staged_items = staged_items1;
    }
    // The last chunk (now mp): everything back to global memory, then pass on its items
    // and those written back in the last iteration.
    write_back_rows(a, mp, rp, lds, geo, true);
    wait_all();
    publish(tok, pend_id, pend_tk);
    if (lane == 0 && prof) {
        int64_t *w = a.wstats + (int64_t)q * kWStatCount;
        w[kWStatTotal] = (int64_t)(wall_clock64() - t_start);
        w[kWStatAcquire] = (int64_t)t_acq;
        w[kWStatMemWait] = (int64_t)t_mem;
        w[kWStatChunks] = total;
        w[kWStatSgd] = (int64_t)t_sgd;
        w[kWStatIssue] = (int64_t)t_issue;
        w[kWStatRatings] = (int64_t)n_rat;
        w[kWStatStage] = (int64_t)t_stage;
    }
}

template <int VEC, int NR16>
hipError_t launch_t(const TrainArgs &a, int32_t p, size_t lds, uint32_t *abort_flag, hipStream_t st) {
    hipLaunchKernelGGL((k_train<VEC, NR16>), dim3(p), dim3(64), lds, st, a, abort_flag);
    return hipGetLastError();
}

template <int VEC, int NR16>
const void *kernel_ptr() { return (const void *)&k_train<VEC, NR16>; }

const void *pick_kernel(int kp) {
    if (kp <= 16) return kernel_ptr<1, 1>();
    if (kp <= 32) return kernel_ptr<1, 2>();
    if (kp <= 64) return kernel_ptr<1, 4>();
    if (kp <= 128) return kernel_ptr<2, 4>();
    return kernel_ptr<4, 4>();
}

}  // namespace

size_t train_lds_bytes(int32_t kp, int32_t rmax, int32_t tmax) {
    // one staging area and one scratch line for lanes beyond the vector width
    return (size_t)(rmax + tmax) * (size_t)kp * sizeof(float) + 64 * 4 * sizeof(float);
}

bool train_chunk_fits(int32_t kp, int32_t rmax, int32_t tmax) {
    const int lpr = kp / 4, rpi = 64 / lpr;
    return rmax <= rpi * kRowPiecesPerLane && tmax <= rpi * kItemPiecesPerLane && rmax + tmax <= kMaxSlots;
}

hipError_t train_max_workers(int32_t kp, int32_t rmax, int32_t tmax, int32_t *max_workers) {
    int dev = 0, cus = 0, nb = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const size_t lds = train_lds_bytes(kp, rmax, tmax);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pick_kernel(kp), 64, lds);
    if (e != hipSuccess) return e;
    *max_workers = nb * cus;
    return hipSuccess;
}

hipError_t launch_train(const TrainArgs &a, int32_t p, uint32_t *abort_flag, hipStream_t st) {
    const size_t lds = train_lds_bytes(a.kp, a.rmax, a.tmax);
    if (a.kp <= 16) return launch_t<1, 1>(a, p, lds, abort_flag, st);
    if (a.kp <= 32) return launch_t<1, 2>(a, p, lds, abort_flag, st);
    if (a.kp <= 64) return launch_t<1, 4>(a, p, lds, abort_flag, st);
    if (a.kp <= 128) return launch_t<2, 4>(a, p, lds, abort_flag, st);
    return launch_t<4, 4>(a, p, lds, abort_flag, st);
}

}  // namespace nomad
