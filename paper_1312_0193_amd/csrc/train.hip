// NOMAD worker kernel: one workgroup = one worker (Algorithm 1), persistent for a whole
// nomad_train_epochs call.  The workgroup has two wavefronts:
//
//   compute wave   runs the SGD updates of section 2.3 over each chunk's ratings in plan
//                  order, on vectors held in LDS, and counts finished chunks ("done");
//   memory wave    stages chunks ahead of it ("staged"): once the compute wave has freed a
//                  chunk's slots it writes back the rows the chunk evicts and loads rows
//                  w_i and items h_j straight into their LDS slots (LDS-DMA loads), copies
//                  the chunk's rating records into a small LDS ring, and after the compute
//                  wave has finished a chunk passes on the items whose visit ended there.
//
// Owner-computes rule (section 3.1): before the memory wave loads an item for a visit it
// waits until the item has finished every earlier visit in the ring order (a per-item
// counter of finished visits reaches the visit's ticket), so worker q is the sole owner
// of h_j while the visit lasts.  When the visit ends the item is written back and the
// counter advanced.  Rows w_i are owned by the worker for good.
//
// Memory-wave pipeline, iteration x (chunk x):
//   wait for the loads and stores of iteration x-1; pass on items whose write-back
//   completed; load what was not loaded ahead (items that were not yet free when polled,
//   or the first chunk of an epoch); publish chunk x to the compute wave; retire the
//   chunks the compute wave has finished; wait until the compute wave has finished every
//   chunk that used the slots chunk x+1 overwrites, write back the rows chunk x+1 evicts
//   and issue its loads; poll the items of chunk x+2, read the events of chunk x+3 and
//   the record of chunk x+4.
// Every wait of the memory wave keeps passing on finished items, so a worker never holds
// an item that another worker waits for while it waits itself (no cycles in the ring
// order), and every wait is bounded in time.
//
// Memory ordering of a hand-off: item vectors are written with device-coherent stores
// (agent scope) and the counter is advanced with a device-coherent store only after
// "s_waitcnt vmcnt(0)" has seen those stores complete; the next owner polls the counter
// with device-coherent loads and reads the item with device-coherent loads.  Rows use
// ordinary loads and stores from the same wavefront, whose accesses to one address are
// performed in program order.  The two wavefronts of a worker synchronise through LDS
// words written after "s_waitcnt lgkmcnt(0)".
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

// Cross-row steps of a wavefront sum, on gfx950's lane swaps.  With the same value in
// both operands, v_permlane16_swap leaves rows (0,0,2,2) in one register and (1,1,3,3)
// in the other; v_permlane32_swap leaves the lower half in both halves of one register
// and the upper half in the other.  Written as asm: the compiler's own form of these
// swaps returns the first result in place of the second.  The s_nop pairs cover the
// VALU-to-swap and swap-to-VALU hazards.
__device__ __forceinline__ float swap_add16(float x) {
    float y = x;
    asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1\n\ts_nop 1" : "+v"(x), "+v"(y));
    return x + y;
}
__device__ __forceinline__ float swap_add32(float x) {
    float y = x;
    asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1\n\ts_nop 1" : "+v"(x), "+v"(y));
    return x + y;
}

// Sum over the first NR16 16-lane rows of x, returned in every lane (lanes beyond the
// active rows must hold 0): butterfly within each row with DPP, then the row swaps.
template <int NR16>
__device__ __forceinline__ float wave_sum(float x) {
    x += DPP_F(x, 0xB1, 0xF, true);   // quad_perm [1,0,3,2]
    x += DPP_F(x, 0x4E, 0xF, true);   // quad_perm [2,3,0,1]
    x += DPP_F(x, 0x124, 0xF, true);  // row_ror 4
    x += DPP_F(x, 0x128, 0xF, true);  // row_ror 8
    if constexpr (NR16 >= 2) x = swap_add16(x);
    if constexpr (NR16 >= 4) x = swap_add32(x);
    return x;
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

__device__ __forceinline__ void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void wait_lgkm() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

// Clock read only when per-worker counters are requested.
__device__ __forceinline__ uint64_t tick(bool on) { return on ? wall_clock64() : 0; }

// ---------------------------------------------------------------------------------------
// LDS of one worker: S vector slots, a ring of kRing staged chunks (rating records and
// the items each chunk releases), and the synchronisation words.
enum SyncWord { kStaged = 0, kDone = 1, kStop = 2 };

struct Lds {
    float *vec;         // S x kp
    RatingRec *rat;     // kRing x 64
    int32_t *rel_id;    // kRing x 64
    uint32_t *rel_tk;   // kRing x 64
    int32_t *rel_slot;  // kRing x 64
    int32_t *cnt;       // kRing x 2: ratings, releases
    int32_t *sync;      // staged, done, stop, unused
    float *zero;        // 64 x 4 zeros: read and written by lanes beyond the vector width
};

constexpr size_t kRingBytes = (size_t)kRing * 64 * (sizeof(RatingRec) + 3 * sizeof(int32_t)) + kRing * 2 * 4 + 4 * 4;

// LDS of one worker (a multiple of 16 bytes): slots, ring, synchronisation, zero line.
__host__ __device__ inline size_t worker_lds_bytes(int kp, int slots) {
    return (size_t)slots * (size_t)kp * sizeof(float) + kRingBytes + 64 * 4 * sizeof(float);
}

__device__ __forceinline__ Lds lds_layout(void *base, int S, int kp) {
    char *p = (char *)base;
    Lds L;
    L.vec = (float *)p;
    p += (size_t)S * kp * sizeof(float);
    L.rat = (RatingRec *)p;
    p += kRing * 64 * sizeof(RatingRec);
    L.rel_id = (int32_t *)p;
    p += kRing * 64 * 4;
    L.rel_tk = (uint32_t *)p;
    p += kRing * 64 * 4;
    L.rel_slot = (int32_t *)p;
    p += kRing * 64 * 4;
    L.cnt = (int32_t *)p;
    p += kRing * 2 * 4;
    L.sync = (int32_t *)p;
    p += 4 * 4;
    L.zero = (float *)p;
    return L;
}

__device__ __forceinline__ int sync_load(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void sync_store(int32_t *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---------------------------------------------------------------------------------------
// Compute wave.

// SGD over one chunk's ratings in plan order, on LDS.
//
// Lane l holds elements [VEC l, VEC l + VEC) of a vector; lanes beyond the vector width
// read and write a line of zeros (their terms add nothing to the dot products).  Every
// rating issues the same LDS operations: write its row and item, then read the row and
// item of the rating two ahead into one of two alternating register sets.  A read-ahead
// row is stale only if it is the row of the rating just before it, which then takes the
// freshly updated registers instead; likewise for an item continuing its run (an item
// has a single run of ratings per chunk, so the first read of a run is never stale).
template <int VEC>
struct SgdLane {
    float *base;  // this lane's elements of slot 0 (or the zero line)
    int stride;   // floats per slot (kp), 0 for lanes beyond the vector width
};

template <int VEC>
__device__ __forceinline__ void read_vec(const SgdLane<VEC> &ln, int slot, float (&v)[VEC]) {
    lds_read<VEC>(ln.base + __umul24(slot, ln.stride), v);
}
template <int VEC>
__device__ __forceinline__ void write_vec(const SgdLane<VEC> &ln, int slot, const float (&v)[VEC]) {
    lds_write<VEC>(ln.base + __umul24(slot, ln.stride), v);
}

template <int VEC>
struct SgdState {
    float w[VEC], h[VEC];  // rating x-1's updated row and item
    int rs_p, ts_p;        // their slots (-1: none yet)
};

template <int VEC, int NR16>
__device__ __forceinline__ void sgd_step(const SgdLane<VEC> &ln, SgdState<VEC> &S, float (&wb)[VEC],
                                         float (&hb)[VEC], int r_sl, float r_val, int x, int nrat, float s,
                                         float shrink) {
    const int sl = rl_i(r_sl, x);
    const int rs = sl & 255, ts = (sl >> 8) & 255;
    const float r = rl_f(r_val, x);
    const bool same_row = rs == S.rs_p, same_item = ts == S.ts_p;
    float w[VEC], h[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        w[v] = same_row ? S.w[v] : wb[v];
        h[v] = same_item ? S.h[v] : hb[v];
    }
    float d = 0.0f;
#pragma unroll
    for (int v = 0; v < VEC; ++v) d = fmaf(w[v], h[v], d);
    d = wave_sum<NR16>(d);
    const float se = s * (r - d);
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        S.w[v] = fmaf(se, h[v], shrink * w[v]);
        S.h[v] = fmaf(se, w[v], shrink * h[v]);
    }
    write_vec<VEC>(ln, rs, S.w);
    write_vec<VEC>(ln, ts, S.h);
    S.rs_p = rs;
    S.ts_p = ts;
    const int x2 = x + 2 < nrat ? x + 2 : nrat - 1;
    const int sl2 = rl_i(r_sl, x2);
    read_vec<VEC>(ln, sl2 & 255, wb);
    read_vec<VEC>(ln, (sl2 >> 8) & 255, hb);
}

template <int VEC, int NR16>
__device__ __forceinline__ void sgd_chunk(const SgdLane<VEC> &ln, const RatingRec &rr, int nrat, float s,
                                          float shrink) {
    if (nrat <= 0) return;
    const int r_sl = (int)rr.slots;
    const float r_val = rr.r;
    float wb0[VEC], hb0[VEC], wb1[VEC], hb1[VEC];
    const int sl0 = rl_i(r_sl, 0), sl1 = rl_i(r_sl, nrat > 1 ? 1 : 0);
    read_vec<VEC>(ln, sl0 & 255, wb0);
    read_vec<VEC>(ln, (sl0 >> 8) & 255, hb0);
    read_vec<VEC>(ln, sl1 & 255, wb1);
    read_vec<VEC>(ln, (sl1 >> 8) & 255, hb1);
    SgdState<VEC> S;
    S.rs_p = -1;
    S.ts_p = -1;
#pragma unroll
    for (int v = 0; v < VEC; ++v) S.w[v] = S.h[v] = 0.0f;
    int x = 0;
    for (; x + 1 < nrat; x += 2) {
        sgd_step<VEC, NR16>(ln, S, wb0, hb0, r_sl, r_val, x, nrat, s, shrink);
        sgd_step<VEC, NR16>(ln, S, wb1, hb1, r_sl, r_val, x + 1, nrat, s, shrink);
    }
    if (x < nrat) sgd_step<VEC, NR16>(ln, S, wb0, hb0, r_sl, r_val, x, nrat, s, shrink);
}

template <int VEC, int NR16>
__device__ __forceinline__ void compute_wave(const TrainArgs &a, const Lds &L, int64_t nck, int q, int lane) {
    const bool prof = a.timing;
    const uint64_t t_start = tick(prof);
    uint64_t t_sgd = 0, t_starve = 0;
    int64_t n_rat = 0;
    const int64_t total = nck * a.epochs;
    int epoch = -1, ex = a.epoch0;
    int64_t lx = 0;
    float s_step = 0.0f, s_shrink = 1.0f;
    const bool on = lane * VEC < a.kp;
    SgdLane<VEC> ln;
    ln.base = on ? L.vec + lane * VEC : L.zero + lane * VEC;
    ln.stride = on ? a.kp : 0;
    for (int64_t x = 0; x < total; ++x) {
        if (sync_load(&L.sync[kStaged]) <= x) {
            const uint64_t t0 = tick(prof);
            while (sync_load(&L.sync[kStaged]) <= x) {
                if (sync_load(&L.sync[kStop])) return;
                __builtin_amdgcn_s_sleep(1);
            }
            t_starve += tick(prof) - t0;
        }
        compiler_fence();
        const int ent = (int)(x & (kRing - 1));
        const int nrat = L.cnt[2 * ent];
        RatingRec rr{0u, 0.0f};
        if (lane < nrat) rr = L.rat[ent * 64 + lane];
        if (ex != epoch) {
            // s_t = alpha / (1 + beta t^gamma), t = epochs done (every rating is updated
            // once per epoch), eq. (stepsize_method).
            epoch = ex;
            const double t = (double)ex;
            const double sd = a.alpha / (1.0 + a.beta * (t > 0.0 ? pow(t, a.gamma) : 0.0));
            s_step = (float)sd;
            s_shrink = 1.0f - s_step * a.lambda;
        }
        const uint64_t t0 = tick(prof);
        sgd_chunk<VEC, NR16>(ln, rr, nrat, s_step, s_shrink);
        wait_lgkm();
        t_sgd += tick(prof) - t0;
        n_rat += nrat;
        if (lane == 0) sync_store(&L.sync[kDone], (int)(x + 1));
        if (++lx == nck) {
            lx = 0;
            ++ex;
        }
    }
    if (a.wstats && lane == 0) {
        int64_t *w = a.wstats + (int64_t)q * kWStatCount;
        w[kWStatTotal] = (int64_t)(tick(prof) - t_start);
        w[kWStatChunks] = total;
        w[kWStatSgd] = (int64_t)t_sgd;
        w[kWStatRatings] = n_rat;
        w[kWStatStarve] = (int64_t)t_starve;
    }
}

// ---------------------------------------------------------------------------------------
// Memory wave.

struct Meta {
    int64_t rat, ev;
    int nrat, nload, nrel, nflush, need;
};

// Record of the chunk at local index lc of the worker's plan (chunk x = lc + epoch * nck
// of the call); an empty record when x is past the end of the call.
__device__ __forceinline__ Meta load_meta(const TrainArgs &a, int64_t c0, int64_t lc, bool valid) {
    Meta m{0, 0, 0, 0, 0, 0, 0};
    if (!valid) return m;
    const ChunkRec r = a.chunks[c0 + lc];
    m.rat = r.rat;
    m.ev = r.ev;
    m.nrat = r.nrat;
    m.nload = r.nload;
    m.nrel = r.nrel;
    m.nflush = r.nflush;
    m.need = r.need_done;
    return m;
}

// Event records of one chunk, one per lane (loads, then releases).
struct Ev {
    int id;
    int sk;
    int evict;
    int vis;
};
__device__ __forceinline__ Ev load_ev(const EvRec *g, int count, int lane) {
    Ev e{0, 0, -1, 0};
    if (lane < count) {
        const int4 v = *(const int4 *)(g + lane);
        e.id = v.x;
        e.sk = v.y;
        e.evict = v.z;
        e.vis = v.w;
    }
    return e;
}
__device__ __forceinline__ int ev_slot(int sk) { return sk & 255; }
__device__ __forceinline__ int ev_kind(int sk) { return (sk >> 8) & 255; }
// Counter value at which the visit may start in epoch `epoch`.
__device__ __forceinline__ uint32_t ev_ticket(int vis, int epoch) {
    return (uint32_t)((int64_t)epoch * (int64_t)((uint32_t)vis >> 16) + (int64_t)(vis & 0xffff));
}

typedef __attribute__((address_space(3))) void lds_void_t;

__device__ __forceinline__ uint32_t lds_addr(const float *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) float *)p;
}

// LDS reads of the memory wave, waited for inside the asm block.  Written as asm so that
// the compiler does not put "s_waitcnt vmcnt(0)" in front of them (it cannot tell these
// slots from those the wave's LDS-DMA loads write, and would make every read wait for
// all outstanding stores).  The slots read here are never the target of a load in
// flight: a slot is read before any load into it is issued.
__device__ __forceinline__ void lds_read4x4_now(uint32_t p0, uint32_t p1, uint32_t p2, uint32_t p3, f32x4_t &v0,
                                                f32x4_t &v1, f32x4_t &v2, f32x4_t &v3) {
    asm volatile(
        "ds_read_b128 %0, %4\n\t"
        "ds_read_b128 %1, %5\n\t"
        "ds_read_b128 %2, %6\n\t"
        "ds_read_b128 %3, %7\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(v0), "=&v"(v1), "=&v"(v2), "=&v"(v3)
        : "v"(p0), "v"(p1), "v"(p2), "v"(p3)
        : "memory");
}

struct MemoryWave {
    const TrainArgs &a;
    const Lds &L;
    const int64_t c0, nck, total;
    const int q, lane, kp;
    uint32_t *const abort_flag;
    const bool prof;
    int64_t retired = 0;  // chunks whose releases have been issued
    int64_t retired_lc = 0;  // its local index in the plan
    int pub_id = -1;      // items written back, counter value to publish (one per lane)
    uint32_t pub_tk = 0;
    int pub_n = 0;
    uint64_t t_acq = 0, t_mem = 0, t_slot = 0, t_commit = 0, t_retire = 0, t_issue = 0, t_evict = 0, t_poll = 0;
    int64_t n_loads = 0, n_late = 0;

    __device__ MemoryWave(const TrainArgs &a_, const Lds &L_, int64_t c0_, int64_t nck_, int q_, int lane_,
                          uint32_t *abort_)
        : a(a_), L(L_), c0(c0_), nck(nck_), total(nck_ * a_.epochs), q(q_), lane(lane_), kp(a_.kp),
          abort_flag(abort_), prof(a_.timing) {}

    __device__ __forceinline__ void publish() {
        if (lane < pub_n) __hip_atomic_store(a.tok_done + pub_id, pub_tk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        pub_n = 0;
    }

    // Copy `count` vectors from LDS slots to global memory (W, or H with device-coherent
    // stores): lane t < count of `id` / `sk` gives the vector's id (< 0: skip) and slot.
    // A vector is kp / 4 lanes of 16 bytes, so one instruction moves rpi = 64 / (kp / 4)
    // vectors.  All reads of a batch of 8 instructions land in distinct registers before
    // the first store, so no read of a batch waits for a store of the same batch.
    __device__ __forceinline__ void slots_to_global(float *dst, bool coherent, int id, int sk, int count) {
        constexpr int kRounds = 8;
        const int lpr = kp >> 2, rpi = 64 / lpr, vb = lane / lpr, piece = lane - vb * lpr;
        const bool act = vb < rpi;
        const uint32_t base = lds_addr(L.vec) + (uint32_t)piece * 16u;
        for (int b0 = 0; b0 < count; b0 += kRounds * rpi) {
            int gid[kRounds];
            uint32_t src[kRounds];
#pragma unroll
            for (int r = 0; r < kRounds; ++r) {
                gid[r] = -1;
                src[r] = base;
                if (b0 + r * rpi < count) {
                    const int t = b0 + r * rpi + vb;
                    const int g = __shfl(id, t & 63), s = ev_slot(__shfl(sk, t & 63));
                    gid[r] = (act && t < count) ? g : -1;
                    src[r] = base + (uint32_t)((gid[r] >= 0 ? s : 0) * kp) * 4u;
                }
            }
            f32x4_t v[kRounds];
#pragma unroll
            for (int r = 0; r < kRounds; r += 4)
                if (b0 + r * rpi < count)
                    lds_read4x4_now(src[r], src[r + 1], src[r + 2], src[r + 3], v[r], v[r + 1], v[r + 2], v[r + 3]);
#pragma unroll
            for (int r = 0; r < kRounds; ++r) {
                if (b0 + r * rpi >= count || gid[r] < 0) continue;
                float *p = dst + (int64_t)gid[r] * kp + piece * 4;
                if (coherent)
                    coherent_store4(p, v[r]);
                else
                    *(f32x4_t *)p = v[r];
            }
        }
    }

    // Write back the rows left in LDS at the end of an epoch (after its last chunk y).
    __device__ __forceinline__ void flush() {
        const Meta m = load_meta(a, c0, nck - 1, true);
        const int64_t f0 = m.ev + m.nload + m.nrel;
        for (int b0 = 0; b0 < m.nflush; b0 += 64) {
            const int cnt = m.nflush - b0 < 64 ? m.nflush - b0 : 64;
            const Ev f = load_ev(a.events + f0 + b0, cnt, lane);
            wait_vm();
            const bool ok = lane >= cnt || (f.id >= 0 && f.id < a.m && ev_slot(f.sk) < a.slots);
            if (__builtin_amdgcn_ballot_w64(!ok) != 0) continue;  // malformed: skip (validated elsewhere)
            slots_to_global(a.W, false, f.id, f.sk, cnt);
        }
    }

    // Pass on the items of every chunk the compute wave has finished: device-coherent
    // write-back now, counter published once the stores have completed.
    __device__ __forceinline__ void retire() {
        const int64_t d = sync_load(&L.sync[kDone]);
        compiler_fence();
        while (retired < d) {
            const int64_t y = retired;
            const int ent = (int)(y & (kRing - 1));
            const int nrel = L.cnt[2 * ent + 1];
            if (nrel > 0) {
                if (pub_n + nrel > 64) {
                    wait_vm();
                    publish();
                }
                const int rid = lane < nrel ? L.rel_id[ent * 64 + lane] : -1;
                const int rsl = lane < nrel ? L.rel_slot[ent * 64 + lane] : 0;
                slots_to_global(a.H, true, rid, rsl, nrel);
                const int r = lane - pub_n;
                if (r >= 0 && r < nrel) {
                    pub_id = L.rel_id[ent * 64 + r];
                    pub_tk = L.rel_tk[ent * 64 + r];
                }
                pub_n += nrel;
            }
            if (retired_lc == nck - 1) {
                flush();
                retired_lc = 0;
            } else {
                ++retired_lc;
            }
            ++retired;
        }
    }

    // Retire and publish while waiting.
    __device__ __forceinline__ void service() {
        retire();
        if (pub_n > 0) {
            wait_vm();
            publish();
        }
    }

    __device__ __forceinline__ bool give_up(uint64_t t0) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return true;
        if (wall_clock64() - t0 > kWaitLimitTicks) {
            if (lane == 0) __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return true;
        }
        return false;
    }

    // End the worker early: tell the compute wave, and record `code` (if non-zero).
    __device__ __forceinline__ void stop(uint32_t code) {
        wait_vm();
        if (code && lane == 0) __hip_atomic_store(abort_flag, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (lane == 0) sync_store(&L.sync[kStop], 1);
    }

    // Wait until the compute wave has finished `need` chunks.
    __device__ __forceinline__ bool wait_done(int64_t need) {
        if (sync_load(&L.sync[kDone]) >= need) return true;
        const uint64_t t0 = wall_clock64();
        while (sync_load(&L.sync[kDone]) < need) {
            service();
            if (give_up(t0)) return false;
            __builtin_amdgcn_s_sleep(1);
        }
        if (prof) t_slot += wall_clock64() - t0;
        return true;
    }

    // Wait until every item event of `e` flagged in `mask` may start (epoch `epoch`).
    __device__ __forceinline__ bool acquire(const Ev &e, uint64_t mask, int epoch) {
        const bool mine = ((mask >> lane) & 1ull) != 0;
        const uint32_t tk = ev_ticket(e.vis, epoch);
        bool pending = mine && __hip_atomic_load(a.tok_done + e.id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != tk;
        if (__builtin_amdgcn_ballot_w64(pending) == 0) return true;
        const uint64_t t0 = wall_clock64();
        while (true) {
            service();
            __builtin_amdgcn_s_sleep(2);
            if (pending)
                pending = __hip_atomic_load(a.tok_done + e.id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != tk;
            if (__builtin_amdgcn_ballot_w64(pending) == 0) break;
            if (give_up(t0)) return false;
        }
        if (prof) t_acq += wall_clock64() - t0;
        return true;
    }

    // Plan validation: a malformed plan (ids or slots out of range) ends the kernel
    // instead of letting a load or a store touch memory outside its arrays.
    __device__ __forceinline__ bool events_ok(const Meta &m, const Ev &e) {
        bool bad = m.nrat > kMaxRatingsPerChunk || m.nload + m.nrel > kMaxEventsPerChunk || m.nrat < 0;
        if (lane < m.nload) {
            const int k = ev_kind(e.sk);
            bad |= ev_slot(e.sk) >= a.slots || (k != kEvLoadRow && k != kEvLoadItem) || e.id < 0 ||
                   e.id >= (k == kEvLoadRow ? a.m : a.n) || e.evict >= a.m;
        } else if (lane < m.nload + m.nrel) {
            bad |= ev_kind(e.sk) != kEvRelease || ev_slot(e.sk) >= a.slots || e.id < 0 || e.id >= a.n;
        }
        return __builtin_amdgcn_ballot_w64(bad) == 0;
    }
    __device__ __forceinline__ bool ratings_ok(const Meta &m, const RatingRec &rr) {
        bool bad = false;
        if (lane < m.nrat) bad = (int)(rr.slots & 255) >= a.slots || (int)((rr.slots >> 8) & 255) >= a.slots;
        return __builtin_amdgcn_ballot_w64(bad) == 0;
    }

    __device__ __forceinline__ uint64_t kind_mask(const Ev &e, int nload, int kind) {
        return __builtin_amdgcn_ballot_w64(lane < nload && ev_kind(e.sk) == kind);
    }

    // Write back the rows a chunk's loads evict (their slots must be free).
    __device__ __forceinline__ void evict(const Ev &e, int nload) {
        slots_to_global(a.W, false, e.evict, e.sk, nload);
    }

    // Load the vectors of the events flagged in `mask` into their slots: each event lane
    // computes its source address and LDS slot address once, then one LDS-DMA
    // instruction per vector (rows plain, items device-coherent).
    __device__ __forceinline__ void load_vectors(const Ev &e, int nload, uint64_t mask) {
        const bool item = ev_kind(e.sk) == kEvLoadItem;
        const uint64_t src = (uint64_t)(uintptr_t)((item ? a.H : a.W) + (int64_t)e.id * kp);
        const uint32_t s_lo = (uint32_t)src, s_hi = (uint32_t)(src >> 32);
        const int dst = ev_slot(e.sk) * kp;
        const uint64_t items = mask & kind_mask(e, nload, kEvLoadItem), rows = mask & ~items;
        const bool on = lane < (kp >> 2);
        for (uint64_t mk = rows; mk; mk &= mk - 1) {
            const int t = __builtin_ctzll(mk);
            const uint64_t p = (uint64_t)(uint32_t)__builtin_amdgcn_readlane(s_lo, t) |
                               ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(s_hi, t) << 32);
            float *d = L.vec + __builtin_amdgcn_readlane(dst, t);
            if (on)
                __builtin_amdgcn_global_load_lds((const void *)((const float *)(uintptr_t)p + lane * 4),
                                                 (lds_void_t *)d, 16, 0, 0);
        }
        for (uint64_t mk = items; mk; mk &= mk - 1) {
            const int t = __builtin_ctzll(mk);
            const uint64_t p = (uint64_t)(uint32_t)__builtin_amdgcn_readlane(s_lo, t) |
                               ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(s_hi, t) << 32);
            float *d = L.vec + __builtin_amdgcn_readlane(dst, t);
            if (on)
                __builtin_amdgcn_global_load_lds((const void *)((const float *)(uintptr_t)p + lane * 4),
                                                 (lds_void_t *)d, 16, 0, 16);
        }
    }

    __device__ __forceinline__ void run() {
        if (total <= 0) return;
        // Local plan index of chunk x+4 (advanced with wrap-around, no division).
        int64_t lc4 = 0;
        auto next_lc = [&](int64_t lc) { return lc + 1 == nck ? 0 : lc + 1; };
        Meta m0 = load_meta(a, c0, lc4, 0 < total);
        lc4 = next_lc(lc4);
        Meta m1 = load_meta(a, c0, lc4, 1 < total);
        lc4 = next_lc(lc4);
        Meta m2 = load_meta(a, c0, lc4, 2 < total);
        lc4 = next_lc(lc4);
        Meta m3 = load_meta(a, c0, lc4, 3 < total);
        lc4 = next_lc(lc4);
        Ev e0 = load_ev(a.events + m0.ev, m0.nload + m0.nrel, lane);
        Ev e1 = load_ev(a.events + m1.ev, m1.nload + m1.nrel, lane);
        Ev e2 = load_ev(a.events + m2.ev, m2.nload + m2.nrel, lane);
        RatingRec rr0{0u, 0.0f}, rr1{0u, 0.0f};
        if (lane < m0.nrat) rr0 = a.ratings[m0.rat + lane];
        wait_vm();
        if (!events_ok(m0, e0) || !events_ok(m1, e1) || !events_ok(m2, e2)) {
            stop(2u);
            return;
        }
        uint32_t pr1 = 0, pr2 = 0;
        if (lane < m1.nload && ev_kind(e1.sk) == kEvLoadItem)
            pr1 = __hip_atomic_load(a.tok_done + e1.id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint64_t fm0 = 0, fm1 = 0;  // loads of chunk x / x+1 already issued
        int64_t lx = 0;
        int ex = a.epoch0;
        for (int64_t x = 0; x < total; ++x) {
            // Loads of this chunk issued in iteration x-1 and write-backs are complete.
            uint64_t t0 = tick(prof);
            wait_vm();
            t_mem += tick(prof) - t0;
            if (pub_n > 0) publish();
            if (!events_ok(m2, e2)) {
                stop(2u);
                return;
            }
            const int64_t xbase = x - lx;  // first chunk of this epoch
            // A new epoch starts once the previous one has been written back entirely.
            if (x > 0 && lx == 0) {
                if (!wait_done(x)) { stop(0u); return; }
                retire();
            }
            if (!ratings_ok(m0, rr0)) {
                stop(2u);
                return;
            }
            const uint64_t loads = m0.nload >= 64 ? ~0ull : ((1ull << m0.nload) - 1ull);
            const uint64_t rem = loads & ~fm0;
            n_loads += m0.nload;
            if (rem) {
                // Not prefetched: the first chunk of an epoch, or items that were not free
                // when polled.
                n_late += __builtin_popcountll(rem);
                if (fm0 == 0) {
                    int64_t need = xbase + m0.need;
                    if (x - kRing + 1 > need) need = x - kRing + 1;
                    if (!wait_done(need)) { stop(0u); return; }
                    retire();
                    evict(e0, m0.nload);
                }
                const uint64_t items = kind_mask(e0, m0.nload, kEvLoadItem) & rem;
                if (items && !acquire(e0, items, ex)) { stop(0u); return; }
                load_vectors(e0, m0.nload, rem);
                t0 = tick(prof);
                wait_vm();
                t_mem += tick(prof) - t0;
            }
            uint64_t tc = tick(prof);
            // Ring entry for the compute wave: ratings, and the items released after it.
            const int ent = (int)(x & (kRing - 1));
            if (lane < m0.nrat) L.rat[ent * 64 + lane] = rr0;
            {
                const int src = (m0.nload + lane) & 63;
                const int rid = __shfl(e0.id, src), rsk = __shfl(e0.sk, src), rvis = __shfl(e0.vis, src);
                if (lane < m0.nrel) {
                    L.rel_id[ent * 64 + lane] = rid;
                    L.rel_slot[ent * 64 + lane] = ev_slot(rsk);
                    L.rel_tk[ent * 64 + lane] = ev_ticket(rvis, ex) + 1u;
                }
            }
            if (lane == 0) {
                L.cnt[2 * ent] = m0.nrat;
                L.cnt[2 * ent + 1] = m0.nrel;
            }
            wait_lgkm();
            if (lane == 0) sync_store(&L.sync[kStaged], (int)(x + 1));
            t_commit += tick(prof) - tc;
            if (a.trace) {
                // One record per item taken over, in event order (the order of the visits).
                const uint64_t im = kind_mask(e0, m0.nload, kEvLoadItem);
                int64_t base = 0;
                if (lane == 0 && im) base = (int64_t)atomicAdd((unsigned long long *)a.trace_len,
                                                               (unsigned long long)__builtin_popcountll(im));
                base = __shfl(base, 0);
                const int64_t slot = base + __builtin_popcountll(im & ((1ull << lane) - 1ull));
                if (((im >> lane) & 1ull) && slot < a.trace_cap) {
                    a.trace[4 * slot + 0] = q;
                    a.trace[4 * slot + 1] = e0.id;
                    a.trace[4 * slot + 2] = ex;
                    a.trace[4 * slot + 3] = (int32_t)ev_ticket(e0.vis, ex);
                }
            }
            tc = tick(prof);
            retire();
            t_retire += tick(prof) - tc;

            // Chunk x+1 (not across an epoch boundary: the epoch's rows are written back
            // first): once its slots are free, write back the rows it evicts and load its
            // rows and the items seen free.  Then poll chunk x+2, read events x+3 and the
            // record of x+4.
            const int64_t lx1 = lx + 1 == nck ? 0 : lx + 1;
            const int ex1 = lx + 1 == nck ? ex + 1 : ex;
            fm1 = 0;
            if (x + 1 < total) {
                if (lane < m1.nrat) rr1 = a.ratings[m1.rat + lane];
                if (lx1 != 0) {
                    int64_t need = xbase + m1.need;
                    if (x + 1 - kRing + 1 > need) need = x + 1 - kRing + 1;
                    if (!wait_done(need)) { stop(0u); return; }
                    tc = tick(prof);
                    retire();
                    t_retire += tick(prof) - tc;
                    tc = tick(prof);
                    evict(e1, m1.nload);
                    t_evict += tick(prof) - tc;
                    tc = tick(prof);
                    const uint64_t rows = kind_mask(e1, m1.nload, kEvLoadRow);
                    const bool ready =
                        lane < m1.nload && ev_kind(e1.sk) == kEvLoadItem && pr1 == ev_ticket(e1.vis, ex1);
                    fm1 = rows | __builtin_amdgcn_ballot_w64(ready);
                    load_vectors(e1, m1.nload, fm1);
                    t_issue += tick(prof) - tc;
                }
            }
            tc = tick(prof);
            pr2 = 0;
            if (x + 2 < total && lane < m2.nload && ev_kind(e2.sk) == kEvLoadItem)
                pr2 = __hip_atomic_load(a.tok_done + e2.id, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const Ev e3 = load_ev(a.events + m3.ev, m3.nload + m3.nrel, lane);
            const Meta m4 = load_meta(a, c0, lc4, x + 4 < total);
            lc4 = next_lc(lc4);
            t_poll += tick(prof) - tc;

            m0 = m1;
            m1 = m2;
            m2 = m3;
            m3 = m4;
            e0 = e1;
            e1 = e2;
            e2 = e3;
            pr1 = pr2;
            rr0 = rr1;
            fm0 = fm1;
            lx = lx1;
            ex = ex1;
        }
        // Everything computed: pass on the last items, write back the last rows.
        if (!wait_done(total)) { stop(0u); return; }
        retire();
        wait_vm();
        publish();
    }
};

// A workgroup holds `group` workers: waves [0, group) are their compute waves and waves
// [group, 2 group) their memory waves, each worker with its own part of the LDS.  With
// waves dealt to the SIMDs in turn, a SIMD then runs one compute and one memory wave
// instead of two compute waves.
template <int VEC, int NR16>
__global__ __launch_bounds__(512) void k_worker(TrainArgs a, uint32_t *abort_flag) {
    extern __shared__ float4 lds4[];
    const int G = a.group;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sub = wave % G;
    const bool compute = wave < G;
    const int q = blockIdx.x * G + sub;
    const Lds L = lds_layout((char *)lds4 + (size_t)sub * worker_lds_bytes(a.kp, a.slots), a.slots, a.kp);
    if (compute) {
        if (lane < 4) L.sync[lane] = 0;
        for (int i = lane; i < 64 * 4; i += 64) L.zero[i] = 0.0f;
    }
    __syncthreads();
    if (q >= a.p) return;
    const int64_t c0 = a.wck[q], nck = a.wck[q + 1] - c0;
    if (nck <= 0 || a.epochs <= 0) return;
    if (compute) {
        compute_wave<VEC, NR16>(a, L, nck, q, lane);
    } else {
        const uint64_t t_start = tick(a.timing);
        MemoryWave mw(a, L, c0, nck, q, lane, abort_flag);
        mw.run();
        if (a.wstats && lane == 0) {
            int64_t *w = a.wstats + (int64_t)q * kWStatCount;
            w[kWStatAcquire] = (int64_t)mw.t_acq;
            w[kWStatMemWait] = (int64_t)mw.t_mem;
            w[kWStatSlotWait] = (int64_t)mw.t_slot;
            w[kWStatMemTotal] = (int64_t)(tick(a.timing) - t_start);
            w[kWStatCommit] = (int64_t)mw.t_commit;
            w[kWStatRetire] = (int64_t)mw.t_retire;
            w[kWStatIssue] = (int64_t)mw.t_issue;
            w[kWStatLoads] = mw.n_loads;
            w[kWStatLate] = mw.n_late;
            w[14] = (int64_t)mw.t_evict;
            w[15] = (int64_t)mw.t_poll;
        }
    }
}

template <int VEC, int NR16>
hipError_t launch_t(const TrainArgs &a, int32_t blocks, size_t lds, uint32_t *abort_flag, hipStream_t st) {
    hipLaunchKernelGGL((k_worker<VEC, NR16>), dim3(blocks), dim3(128 * a.group), lds, st, a, abort_flag);
    return hipGetLastError();
}

template <int VEC, int NR16>
const void *kernel_ptr() { return (const void *)&k_worker<VEC, NR16>; }

const void *pick_kernel(int kp) {
    if (kp <= 16) return kernel_ptr<1, 1>();
    if (kp <= 32) return kernel_ptr<1, 2>();
    if (kp <= 64) return kernel_ptr<1, 4>();
    if (kp <= 128) return kernel_ptr<2, 4>();
    return kernel_ptr<4, 4>();
}

}  // namespace

size_t train_lds_bytes(int32_t kp, int32_t slots) { return worker_lds_bytes(kp, slots); }

int32_t train_group(int32_t kp, int32_t slots, size_t max_lds_per_block) {
    const size_t per = worker_lds_bytes(kp, slots);
    for (int32_t g = 4; g > 1; g >>= 1)
        if ((size_t)g * per <= max_lds_per_block) return g;
    return 1;
}

hipError_t train_max_workers(int32_t kp, int32_t slots, int32_t group, int32_t *max_workers) {
    int dev = 0, cus = 0, nb = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)group * worker_lds_bytes(kp, slots);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pick_kernel(kp), 128 * group, lds);
    if (e != hipSuccess) return e;
    *max_workers = nb * cus * group;
    return hipSuccess;
}

hipError_t launch_train(const TrainArgs &a, int32_t p, uint32_t *abort_flag, hipStream_t st) {
    const size_t lds = (size_t)a.group * worker_lds_bytes(a.kp, a.slots);
    const int32_t blocks = (p + a.group - 1) / a.group;
    if (a.kp <= 16) return launch_t<1, 1>(a, blocks, lds, abort_flag, st);
    if (a.kp <= 32) return launch_t<1, 2>(a, blocks, lds, abort_flag, st);
    if (a.kp <= 64) return launch_t<1, 4>(a, blocks, lds, abort_flag, st);
    if (a.kp <= 128) return launch_t<2, 4>(a, blocks, lds, abort_flag, st);
    return launch_t<4, 4>(a, blocks, lds, abort_flag, st);
}

}  // namespace nomad
