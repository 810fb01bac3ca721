// NOMAD worker kernel (Algorithm 1, in the hybrid form of section 3.4): one workgroup is
// one worker and stays resident for a whole nomad_train_epochs call.  A workgroup has
// nw compute wavefronts and one memory wavefront.
//
//   compute wave w   owns a contiguous sub-block of the worker's rows.  It reads its
//                    ratings as one stream in processing order and runs the SGD updates
//                    of section 2.3 on them.  Rows w_i stream through registers: the row
//                    of the rating D places ahead is loaded while the current one is
//                    updated, and a row used again inside that window is handed on
//                    through LDS instead of being re-read.  The item h_j of a visit comes
//                    from an LDS slot and goes back there at the end of the wave's part
//                    of the visit; the waves of the worker take the item in ascending
//                    order (rows ascending).
//   memory wave      takes items over (a visit may start once the item's counter of
//                    finished visits equals the visit's ticket), loads them into LDS
//                    slots, and passes each item on once the last wave holding ratings of
//                    it is done: device-coherent write-back of h_j, then the counter
//                    advanced.
//
// The serial order this realises is the fixed ring order: worker q, sub-step s, items of
// group (q + s) mod p ascending, rows ascending.  Every row and every item sees its
// updates in that order, so the result does not depend on timing, on nw or on the number
// of item slots.
//
// Memory ordering of a hand-off between workers: the item is written with
// device-coherent stores, "s_waitcnt vmcnt(0)" sees them complete, and only then is the
// counter advanced with a device-coherent store; the next owner polls the counter with
// device-coherent loads and loads the item with device-coherent LDS-DMA loads.  Rows use
// ordinary loads and stores of the one wavefront that owns them, whose accesses to one
// address are performed in program order.  Waves of a worker synchronise through LDS
// words written after "s_waitcnt lgkmcnt(0)".
#include <cmath>
#include <utility>

#include <hipcub/hipcub.hpp>

#include "nomad_internal.h"

namespace nomad {
namespace {

#define DPP_F(x, ctrl, rm, bc) \
    __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, (x)), (ctrl), (rm), 0xF, (bc)))

__device__ __forceinline__ int rl_i(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ float rl_f(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// The residual e = -d loss(r, d) / d d of one rating at prediction d (section 2: the method
// takes any separable loss; the updates of section 2.3 read e in place of r - d).  LOSS 0:
// the square loss, e = r - d.  LOSS 1: the logistic loss log(1 + exp(-r d)) of labels +-1,
// e = r / (1 + exp(r d)) (exp overflowing to infinity gives e = 0, its limit).
template <int LOSS>
__device__ __forceinline__ float residual(float r, float d) {
    if constexpr (LOSS == 1) return r / (1.0f + __expf(r * d));
    else return r - d;
}

// Sum of x over the wavefront, valid in lane 63 only: a butterfly within each 16-lane row
// with DPP (every lane of row r then holds its row sum S_r), then the row broadcasts add
// lane 15 into row 1 and lane 47 into row 3, and lane 31 into row 3, so that lane 63 holds
// (S_2 + S_3) + (S_0 + S_1); the other lanes hold partial or undefined values.  The sum
// ends in one lane instead of all of them, which takes fewer dependent steps than lane
// swaps that leave it everywhere; the additions pair the same terms.  The caller finishes
// its scalar arithmetic in lane 63 and reads the result from there.
__device__ __forceinline__ float wave_sum_last(float x) {
    x += DPP_F(x, 0xB1, 0xF, true);   // quad_perm [1,0,3,2]
    x += DPP_F(x, 0x4E, 0xF, true);   // quad_perm [2,3,0,1]
    x += DPP_F(x, 0x124, 0xF, true);  // row_ror 4
    x += DPP_F(x, 0x128, 0xF, true);  // row_ror 8
    // The row broadcasts as one DPP addition each, written out: the compiler emits a DPP move
    // and an addition for them.  The rows outside the row mask keep their value (the operand
    // is tied to the result); the two wait states before each are those a DPP read needs
    // after a vector write of its operand.  Each addition takes the same two terms as before,
    // in the other order, which gives the same sum.
    asm("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf" : "+v"(x));
    asm("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf" : "+v"(x));
    return x;
}

typedef __attribute__((address_space(3))) float lds_float;
typedef __attribute__((address_space(3))) uint32_t lds_u32;

// VEC consecutive floats of global memory or LDS.
template <int VEC>
__device__ __forceinline__ void vload(const float *p, float (&v)[VEC]) {
    if constexpr (VEC == 1) { v[0] = p[0]; }
    if constexpr (VEC == 2) { const float2 t = *(const float2 *)p; v[0] = t.x; v[1] = t.y; }
    if constexpr (VEC == 4) { const float4 t = *(const float4 *)p; v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w; }
}
template <int VEC>
__device__ __forceinline__ void vstore(float *p, const float (&v)[VEC]) {
    if constexpr (VEC == 1) { p[0] = v[0]; }
    if constexpr (VEC == 2) { *(float2 *)p = make_float2(v[0], v[1]); }
    if constexpr (VEC == 4) { *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]); }
}
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) f32x2v lds_f32x2;
typedef __attribute__((address_space(3))) f32x4v lds_f32x4;

template <int VEC>
__device__ __forceinline__ void lload(const lds_float *p, float (&v)[VEC]) {
    if constexpr (VEC == 1) { v[0] = p[0]; }
    if constexpr (VEC == 2) { const f32x2v t = *(const lds_f32x2 *)p; v[0] = t.x; v[1] = t.y; }
    if constexpr (VEC == 4) { const f32x4v t = *(const lds_f32x4 *)p; v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w; }
}
template <int VEC>
__device__ __forceinline__ void lstore(lds_float *p, const float (&v)[VEC]) {
    if constexpr (VEC == 1) { p[0] = v[0]; }
    if constexpr (VEC == 2) { *(lds_f32x2 *)p = f32x2v{v[0], v[1]}; }
    if constexpr (VEC == 4) { *(lds_f32x4 *)p = f32x4v{v[0], v[1], v[2], v[3]}; }
}

// Seconds-scale bound on any single wait, so that a broken schedule ends the kernel
// instead of hanging the device (100 MHz constant clock).
constexpr uint64_t kWaitLimitTicks = 20ull * 100000000ull;

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint64_t u64x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void coherent_store4(float *p, f32x4_t v) {
    const u64x2_t u = __builtin_bit_cast(u64x2_t, v);
    __hip_atomic_store((uint64_t *)p, u.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store((uint64_t *)p + 1, u.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Number of consecutive set bits of m from bit 0 (64 when all are set; the count-trailing-
// zeros instruction gives -1 for a zero input).
__device__ __forceinline__ int leading_run(uint64_t m) { return ~m == 0 ? 64 : (int)__builtin_ctzll(~m); }

__device__ __forceinline__ void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void wait_lgkm() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

// Clock read only when phase timing is requested.
__device__ __forceinline__ uint64_t tick(bool on) { return on ? wall_clock64() : 0; }

__device__ __forceinline__ int sync_load(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void sync_store(int32_t *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}



// ---------------------------------------------------------------------------------------
// LDS of a worker: item slots, the row slots and record ring of every compute wave, and
// the words the waves synchronise on.
constexpr int kRecBatch = 64;   // records a compute wave stages with one load
constexpr int kRecRing = 3;     // batches a compute wave holds

struct Lds {
    float *items;     // slots x kp
    char *rows;       // nw x (D + 1) x kp elements of W's storage type: row slots of every compute wave
    RatingRec *recs;  // nw x kRecRing x kRecBatch: staged records of every compute wave
    int32_t *item;    // kMaxItemSlots: the item in each slot
    int32_t *sx;      // kMaxItemSlots: asynchronous schedules: the item's local index at the worker
    int32_t *se;      // kMaxItemSlots: asynchronous schedules: the visit's step counter t
    float *ss, *sc;   // kMaxItemSlots: asynchronous schedules: the visit's step size s_t and s_t lambda
    int32_t *flag;    // nw: 1 + the last visit each compute wave finished
    int32_t *ctl;     // [0] visits loaded, [1] stop
};

__host__ __device__ inline size_t lds_bytes(int kp, int nw, int slots, int window, int wbytes) {
    return (size_t)slots * kp * sizeof(float) + (size_t)nw * (window + 1) * kp * wbytes +
           (size_t)nw * kRecRing * kRecBatch * sizeof(RatingRec) + (5 * kMaxItemSlots + kMaxWaves + 1 + 4) * 4;
}

__device__ __forceinline__ Lds lds_layout(void *base, int kp, int nw, int slots, int window, int wbytes) {
    char *p = (char *)base;
    Lds L;
    L.items = (float *)p;
    p += (size_t)slots * kp * sizeof(float);
    L.rows = p;
    p += (size_t)nw * (window + 1) * kp * wbytes;
    L.recs = (RatingRec *)p;
    p += (size_t)nw * kRecRing * kRecBatch * sizeof(RatingRec);
    L.item = (int32_t *)p;
    p += kMaxItemSlots * 4;
    L.sx = (int32_t *)p;
    p += kMaxItemSlots * 4;
    L.se = (int32_t *)p;
    p += kMaxItemSlots * 4;
    L.ss = (float *)p;
    p += kMaxItemSlots * 4;
    L.sc = (float *)p;
    p += kMaxItemSlots * 4;
    L.flag = (int32_t *)p;
    p += (kMaxWaves + 1) * 4;
    L.ctl = (int32_t *)p;
    return L;
}

__device__ __forceinline__ lds_float *to_lds(float *p) { return (lds_float *)(p); }

// Record the end of the worker: every wave stops waiting.
__device__ __forceinline__ void raise_abort(uint32_t *abort_flag, const Lds &L, uint32_t code) {
    __hip_atomic_store(abort_flag, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sync_store(&L.ctl[1], 1);
}

// First wait that ran out of time: diag[0] = 1 + worker, then wave (-1: memory wave) and
// what it waited for.
__device__ __forceinline__ void note_timeout(int32_t *diag, int q, int w, int a0, int a1, int a2, int a3) {
    if (atomicCAS(diag, 0, q + 1) == 0) {
        diag[1] = w;
        diag[2] = a0;
        diag[3] = a1;
        diag[4] = a2;
        diag[5] = a3;
    }
}

// Wait until the LDS word *p exceeds x.  False if the worker is stopping.
__device__ __forceinline__ bool wait_above(const int32_t *p, int x, const Lds &L, uint32_t *abort_flag,
                                           int lane, int32_t *diag, int q, int w, int which) {
    if (sync_load(p) > x) return true;
    const uint64_t t0 = wall_clock64();
    while (sync_load(p) <= x) {
        if (sync_load(&L.ctl[1])) return false;
        if (wall_clock64() - t0 > kWaitLimitTicks) {
            if (lane == 0) {
                note_timeout(diag, q, w, x, sync_load(p), which, sync_load(&L.ctl[0]));
                raise_abort(abort_flag, L, 1u);
            }
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// ---------------------------------------------------------------------------------------
// LDS-DMA loads, written as asm so that the compiler neither sees them as LDS writes (it
// would then wait for every outstanding memory operation before each LDS read) nor counts
// them; the waits for them are explicit.  m0 holds the LDS address of lane 0's data; lane
// l writes at m0 + l * (bytes per lane).  Lanes outside `mask` do nothing.  m0 and exec
// are restored; the exec mask is set with an instruction that writes SCC, so SCC is
// declared clobbered (the compiler keeps carries of 64-bit scalar arithmetic in SCC).

__device__ __forceinline__ uint32_t lds_off(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char *)p;
}

#define NOMAD_DMA16(cpol)                                   \
    uint64_t saved;                                         \
    uint32_t m0s;                                           \
    asm volatile(                                           \
        "s_mov_b32 %1, m0\n\t"                              \
        "s_mov_b64 %0, exec\n\t"                            \
        "s_and_b64 exec, exec, %4\n\t"                      \
        "s_mov_b32 m0, %3\n\t"                              \
        "s_nop 0\n\t"                                       \
        "global_load_lds_dwordx4 %2, off" cpol "\n\t"        \
        "s_mov_b64 exec, %0\n\t"                            \
        "s_mov_b32 m0, %1"                                  \
        : "=&s"(saved), "=&s"(m0s)                          \
        : "v"(src), "s"(lds), "s"(mask)                     \
        : "memory", "scc")

// Scalar operands go through readfirstlane: the compiler may otherwise hand a value it
// cannot prove uniform to an "s" operand in a vector register.
__device__ __forceinline__ uint32_t sgpr32(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ uint64_t sgpr64(uint64_t x) {
    return (uint64_t)sgpr32((uint32_t)x) | ((uint64_t)sgpr32((uint32_t)(x >> 32)) << 32);
}

__device__ __forceinline__ void dma16(const void *src, uint32_t lds_, uint64_t mask_) {
    const uint32_t lds = sgpr32(lds_);
    const uint64_t mask = sgpr64(mask_);
    NOMAD_DMA16("");
}
// Scalar base address plus a 32-bit lane offset.
__device__ __forceinline__ void dma16s(const void *base_, uint32_t voff, uint32_t lds_, uint64_t mask_) {
    const void *base = (const void *)sgpr64((uint64_t)(uintptr_t)base_);
    const uint32_t lds = sgpr32(lds_);
    const uint64_t mask = sgpr64(mask_);
    uint64_t saved;
    uint32_t m0s;
    asm volatile(
        "s_mov_b32 %1, m0\n\t"
        "s_mov_b64 %0, exec\n\t"
        "s_and_b64 exec, exec, %5\n\t"
        "s_mov_b32 m0, %4\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dwordx4 %2, %3\n\t"
        "s_mov_b64 exec, %0\n\t"
        "s_mov_b32 m0, %1"
        : "=&s"(saved), "=&s"(m0s)
        : "v"(voff), "s"(base), "s"(lds), "s"(mask)
        : "memory", "scc");
}
// Device-coherent form (sc1), for items handed over by other workers.
__device__ __forceinline__ void dma16_coherent(const void *src, uint32_t lds_, uint64_t mask_) {
    const uint32_t lds = sgpr32(lds_);
    const uint64_t mask = sgpr64(mask_);
    NOMAD_DMA16(" sc1");
}

__device__ __forceinline__ void dma4(const void *src, uint32_t lds_) {
    const uint32_t lds = sgpr32(lds_);
    uint32_t m0s;
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %2\n\t"
        "s_nop 0\n\t"
        "global_load_lds_dword %1, off\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(m0s)
        : "v"(src), "s"(lds)
        : "memory");
}

// ---------------------------------------------------------------------------------------
// Compute wave.
//
// Rows: the rows of the next D ratings are in flight into D LDS slots: step y updates
// rating y (slot y mod D) and then starts loading the row of rating y + D into that slot.
// Every step issues exactly one row load and one store, so at the end of step y
// 2(D-2) memory operations have been issued after the load of rating y + 2's row, and
// "s_waitcnt vmcnt(2D-4)" sees that load complete; step y + 1 reads that row from LDS at
// its start, before its own update, so the read overlaps the update.  A row used again
// within the window is not re-read: the layout marks, in each record, the distance to the
// next use of its row and back to the previous one; the earlier update writes its result
// into the later rating's slot (or, for the very next rating, hands it on in registers),
// and the later rating's load goes to a spare slot.  (The earlier update is still
// stored, so a window reaching past the end of the launch loses nothing.)
//
// Records: staged in LDS 64 at a time by one LDS-DMA load, two batches ahead, in a ring of
// three batches; a record is read with one broadcast LDS read.  (Records read through the
// scalar cache would put the scalar-memory latency into every step: scalar loads and LDS
// reads share one counter and scalar loads complete out of order.)
//
// Vectors are padded to 64 * VEC floats, so every lane holds VEC elements.

typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) u32x4v lds_u32x4;
typedef uint32_t u32x2v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) u32x2v lds_u32x2;
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef __attribute__((address_space(3))) char lds_char;
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// Integer hash "lowbias32" (C. Wellons, hash-prospector): the counter-based generator of
// the stochastic rounding bits.
__device__ __forceinline__ uint32_t lowbias32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// Step size of eq. (stepsize_method), s_t = alpha / (1 + beta t^gamma), in double rounded
// to float, and s_t lambda rounded from double.
__device__ __forceinline__ void step_size(const TrainArgs &a, double t, float &s, float &c) {
    s = (float)(a.alpha / (1.0 + a.beta * (t > 0.0 ? pow(t, a.gamma) : 0.0)));
    c = (float)((double)s * (double)a.lambda);
}

// VEC elements of a row in W's storage type (FP32, or bfloat16 = the upper half of an
// FP32) to and from FP32 registers, in LDS and in global memory.  The bfloat16 values
// stored are exactly the registers' values (rounded before).
template <int VEC, bool BF>
__device__ __forceinline__ void row_lload(const lds_char *p, float (&v)[VEC]) {
    if constexpr (!BF) {
        lload<VEC>((const lds_float *)p, v);
    } else if constexpr (VEC == 1) {
        v[0] = __uint_as_float((uint32_t)*(const lds_u16 *)p << 16);
    } else if constexpr (VEC == 2) {
        const uint32_t t = *(const lds_u32 *)p;
        v[0] = __uint_as_float(t << 16);
        v[1] = __uint_as_float(t & 0xFFFF0000u);
    } else {
        const u32x2v t = *(const lds_u32x2 *)p;
        v[0] = __uint_as_float(t.x << 16);
        v[1] = __uint_as_float(t.x & 0xFFFF0000u);
        v[2] = __uint_as_float(t.y << 16);
        v[3] = __uint_as_float(t.y & 0xFFFF0000u);
    }
}
template <int VEC>
__device__ __forceinline__ uint32_t bf_pair(const float (&v)[VEC], int i) {
    return (__float_as_uint(v[i]) >> 16) | (__float_as_uint(v[i + 1]) & 0xFFFF0000u);
}
template <int VEC, bool BF>
__device__ __forceinline__ void row_lstore(lds_char *p, const float (&v)[VEC]) {
    if constexpr (!BF) {
        lstore<VEC>((lds_float *)p, v);
    } else if constexpr (VEC == 1) {
        *(lds_u16 *)p = (uint16_t)(__float_as_uint(v[0]) >> 16);
    } else if constexpr (VEC == 2) {
        *(lds_u32 *)p = bf_pair<VEC>(v, 0);
    } else {
        *(lds_u32x2 *)p = u32x2v{bf_pair<VEC>(v, 0), bf_pair<VEC>(v, 2)};
    }
}
template <int VEC, bool BF>
__device__ __forceinline__ void row_gstore(char *p, const float (&v)[VEC]) {
    if constexpr (!BF) {
        vstore<VEC>((float *)p, v);
    } else if constexpr (VEC == 1) {
        *(uint16_t *)p = (uint16_t)(__float_as_uint(v[0]) >> 16);
    } else if constexpr (VEC == 2) {
        *(uint32_t *)p = bf_pair<VEC>(v, 0);
    } else {
        *(uint2 *)p = make_uint2(bf_pair<VEC>(v, 0), bf_pair<VEC>(v, 2));
    }
}

// The stored form of an updated row: bfloat16 rounding of the FP32 result, nearest-even
// (the hardware conversion, two elements per instruction) or stochastic: the low 16 bits
// plus random bits, truncated; the bits of element l come from the half (l mod 2) of a
// hash of (key of the rating, l / 2), the key hashing (seed, row, item, epoch).
// RND: the rounding rule when known at compile time (0 nearest-even, 1 stochastic), or -1
// to read it from the arguments (a branch per update: it splits an unrolled loop into one
// scheduling region per update).
template <int VEC, bool BF, int RND = -1>
__device__ __forceinline__ void round_stored(const TrainArgs &a, int loff, float (&v)[VEC], int row, int item,
                                         int t) {
    if constexpr (BF) {
        if (RND == 0 || (RND < 0 && a.rounding == 0)) {
            if constexpr (VEC == 1) {
                v[0] = (float)(__bf16)v[0];
            } else {
#pragma unroll
                for (int i = 0; i < VEC; i += 2) {
                    const uint32_t pk = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2v{v[i], v[i + 1]}, bf16x2v));
                    v[i] = __uint_as_float(pk << 16);
                    v[i + 1] = __uint_as_float(pk & 0xFFFF0000u);
                }
            }
        } else {
            const uint32_t key = a.sr_seed ^ ((uint32_t)row * 0x9E3779B1u) ^ ((uint32_t)item * 0x85EBCA77u) ^
                                 ((uint32_t)t * 0xC2B2AE3Du);
            const uint32_t c = lowbias32(key);
            uint32_t word = 0;  // the hash word of the current pair of elements
#pragma unroll
            for (int i = 0; i < VEC; ++i) {
                const int l = loff + i;
                if (VEC == 1 || (i & 1) == 0) word = lowbias32(c + (uint32_t)(l >> 1));
                const uint32_t bits = (l & 1) ? (word >> 16) : (word & 0xFFFFu);
                v[i] = __uint_as_float((__float_as_uint(v[i]) + bits) & 0xFFFF0000u);
            }
        }
    }
}

template <int VEC, int D, bool BF, int LOSS, int RND>
struct ComputeWave {
    static_assert(2 * (D - 2) <= 63 && D >= 4, "vmcnt range");
    static constexpr int ES = BF ? 2 : 4;  // bytes per stored element of W
    const TrainArgs &a;
    const Lds &L;
    const int q, w, lane, kp;
    const int loff;           // first element of the lane
    const int rb;             // bytes of a stored row
    const RatingRec *rs;      // the wave's stream
    const int64_t cnt;        // ratings per epoch
    const int64_t total;      // ratings of the launch
    lds_char *const rows;     // D + 1 row slots (the last one takes loads that are not used), at the lane's elements
    const uint32_t rows_lds;
    const uint32_t recs_lds;  // record ring: kRecRing x kRecBatch records
    lds_float *const items;
    const uint64_t row_mask;  // lanes that load a row (16 bytes each)
    char *const wlane;        // W at the lane's elements of row 0
    int64_t bpos = 0;         // stream position of the next record batch
    int bent = 0;             // ring entry of the next record batch
    uint64_t forwarded = 0, t_wait = 0;
    uint32_t viol = 0;  // ownership checks: ratings of rows the wave does not own

    __device__ ComputeWave(const TrainArgs &a_, const Lds &L_, int q_, int w_, int lane_, int64_t r0, int64_t cnt_)
        : a(a_), L(L_), q(q_), w(w_), lane(lane_), kp(a_.kp), loff(lane_ * VEC), rb(a_.kp * ES),
          rs(a_.recs + r0), cnt(cnt_), total(cnt_ * a_.epochs),
          rows((lds_char *)L_.rows + (size_t)w_ * (D + 1) * a_.kp * ES + lane_ * VEC * ES),
          rows_lds(lds_off(L_.rows) + (uint32_t)(w_ * (D + 1) * a_.kp * ES)),
          recs_lds(lds_off(L_.recs) + (uint32_t)(w_ * kRecRing * kRecBatch * (int)sizeof(RatingRec))),
          items(to_lds(L_.items) + lane_ * VEC),
          row_mask((a_.kp * ES / 16) >= 64 ? ~0ull : ((1ull << (a_.kp * ES / 16)) - 1ull)),
          wlane((char *)a_.W + lane_ * VEC * ES) {}

    __device__ __forceinline__ void load_row(int row, int slot) {
        dma16s((const char *)a.W + (int64_t)row * rb, (uint32_t)(lane & 63) * 16u, rows_lds + (uint32_t)(slot * rb),
               row_mask);
    }
    __device__ __forceinline__ void round_row(float (&v)[VEC], int row, int item, int t) const {
        round_stored<VEC, BF, RND>(a, loff, v, row, item, t);
    }
    __device__ __forceinline__ void placeholder_store() {
        if (lane == 0) a.dummy[(int64_t)q * kMaxWaves + w] = 0.0f;
    }
    // Stage the next kRecBatch records of the stream (taken cyclically): lane l loads one.
    __device__ __forceinline__ void load_batch() {
        int64_t pos = bpos + lane;
        while (pos >= cnt) pos -= cnt;
        dma16(rs + pos, recs_lds + (uint32_t)(bent * kRecBatch * (int)sizeof(RatingRec)), ~0ull);
        bpos += kRecBatch;
        while (bpos >= cnt) bpos -= cnt;
        bent = bent == kRecRing - 1 ? 0 : bent + 1;
    }
    // LDS address of the record after the one at `ad`, in ring order.
    __device__ __forceinline__ uint32_t rec_next(uint32_t ad) const {
        ad += (uint32_t)sizeof(RatingRec);
        return ad == recs_lds + (uint32_t)(kRecRing * kRecBatch * sizeof(RatingRec)) ? recs_lds : ad;
    }
    // A staged record: one LDS read that every lane makes at the same address, then the
    // fields as scalars (done where they are needed, so that the read overlaps the work in
    // between).
    __device__ __forceinline__ u32x4v rec_read(uint32_t ad) const { return *(const lds_u32x4 *)(uintptr_t)ad; }
    __device__ __forceinline__ static RatingRec rec_of(const u32x4v v) {
        RatingRec r;
        r.row = __builtin_amdgcn_readfirstlane((int)v.x);
        r.r = __int_as_float(__builtin_amdgcn_readfirstlane((int)v.y));
        r.info = (uint32_t)__builtin_amdgcn_readfirstlane((int)v.z);
        r.fwd = (uint32_t)__builtin_amdgcn_readfirstlane((int)v.w);
        return r;
    }
    __device__ __forceinline__ RatingRec rec_at(uint32_t ad) const { return rec_of(rec_read(ad)); }
    // Only the row and the forwarding distances of a staged record (all that a row load
    // needs; reading dwords that are not used would let the compiler give their registers
    // to other values while the read is in flight, and wait for it there).
    __device__ __forceinline__ u32x2v rec_read_rf(uint32_t ad) const {
        const lds_u32 *p = (const lds_u32 *)(uintptr_t)ad;
        return u32x2v{p[0], p[3]};
    }

    __device__ void run() {
        if (total <= 0) return;
        const uint64_t t_start = tick(a.timing);
        if (a.owner) {
            // Ownership (section 3.1), checked once for the launch and outside the update
            // loop: every rating of the wave's stream, which is the sequence of ratings it
            // updates (each once per epoch), must be of a row the wave owns.
            const int64_t lo = a.wave_start[(int64_t)q * a.nw + w], hi = a.wave_start[(int64_t)q * a.nw + w + 1];
            uint32_t bad = 0;
            for (int64_t p0 = 0; p0 < cnt; p0 += 64) {
                const int64_t pos = p0 + lane;
                bool b = false;
                if (pos < cnt) {
                    const int64_t r = rs[pos].row;
                    b = r < lo || r >= hi;
                }
                bad += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(b));
            }
            viol = bad * (uint32_t)a.epochs;
        }
        load_batch();
        load_batch();
        wait_vm();
        // Prologue: the rows of ratings 0..D-1, each load followed by a placeholder store
        // (as every later step issues one load and one store).
        uint32_t ai = recs_lds;  // record of the next rating to issue
        int64_t ip = 0;          // next rating to issue
        for (; ip < D; ++ip) {
            if (ip < total) {
                const RatingRec ir = rec_at(ai);
                const int prv = (int)((ir.fwd >> 8) & 255u);
                load_row(ir.row, (prv && prv <= ip) ? D : (int)ip);
            } else {
                load_row(0, D);
            }
            placeholder_store();
            ai = rec_next(ai);
        }
        // State at the top of step y: rc = record of rating y (scalars), vn = record of
        // y + 1 and vi = record of y + D (LDS reads issued in the step before), wn = the row
        // of rating y as read from its slot, and (f1, nwp) = whether rating y - 1 hands
        // its row on to rating y in registers, and that row.
        RatingRec rc = rec_at(recs_lds);
        u32x4v vn = rec_read(recs_lds + (uint32_t)sizeof(RatingRec));
        u32x2v vi = rec_read_rf(ai);
        ai = rec_next(ai);                                            // record of y + D + 1
        uint32_t an = recs_lds + 2u * (uint32_t)sizeof(RatingRec);   // record of y + 2
        float h[VEC], wn[VEC], nwp[VEC];
        bool f1 = false;
#pragma unroll
        for (int v = 0; v < VEC; ++v) h[v] = nwp[v] = 0.0f;
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * (D - 2)) : "memory");
        row_lload<VEC, BF>(rows, wn);
        const int nv = (int)(a.vbase[q + 1] - a.vbase[q]);
        int e = 0, xbase = 0;
        int64_t left = cnt;
        // Step sizes of the launch's epochs, lane e holding epoch e's (read with readlane:
        // a scalar memory load inside the loop would put its latency into every step):
        // s_t = alpha / (1 + beta t^gamma) in double, t = epochs done (every rating is
        // updated once per epoch), rounded to float; and s_t lambda, rounded from double.
        const double tl = (double)(a.epoch0 + lane);
        const float s_tab = (float)(a.alpha / (1.0 + a.beta * (tl > 0.0 ? pow(tl, a.gamma) : 0.0)));
        const float sl_tab = (float)((double)s_tab * (double)a.lambda);
        float s = __shfl(s_tab, 0);
        float sl = __shfl(sl_tab, 0);
        int item = 0;  // the item of the current visit (read with it, for the rounding hash)
        int64_t y = 0;
        for (; y < total; ++y) {
            const int u = (int)(y & (D - 1));
            float wv[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) wv[v] = f1 ? nwp[v] : wn[v];
            const RatingRec rn = rec_of(vn);
            const int irow = __builtin_amdgcn_readfirstlane((int)vi.x);
            const uint32_t ifwd = (uint32_t)__builtin_amdgcn_readfirstlane((int)vi.y);
            const int X = xbase + (int)(rc.info & kInfoXMask);
            const int slot = X & (a.slots - 1);
            if (rc.info & kInfoFirst) {
                // This wave's part of visit X starts: wait for the item, from the memory
                // wave (first wave of the visit) or from the wave before.
                const uint32_t pw = (rc.info >> kInfoPrevShift) & kInfoPrevMask;
                const int32_t *word = pw ? &L.flag[pw - 1] : &L.ctl[0];
                const uint64_t t0 = tick(a.timing);
                if (!wait_above(word, X, L, a.abort_flag, lane, a.diag, q, w, (int)pw)) break;
                compiler_fence();
                t_wait += tick(a.timing) - t0;
                lload<VEC>(items + (size_t)slot * kp, h);
                if constexpr (BF) item = __builtin_amdgcn_readfirstlane(L.item[slot]);
                if (a.gstep) {
                    // the visit's step size (t = the global update count before it)
                    s = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(L.ss[slot])));
                    sl = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(L.sc[slot])));
                }
            }
            // Section 2.3: one residual, both vectors from their values before the update.
            float d = 0.0f;
#pragma unroll
            for (int v = 0; v < VEC; ++v) d = fmaf(wv[v], h[v], d);
            d = wave_sum_last(d);
            // Reads for the next step: the row of rating y + 1 (its load completed in the
            // step before), the records of y + 2 and y + D + 1.
            row_lload<VEC, BF>(rows + ((u + 1) & (D - 1)) * rb, wn);
            vn = rec_read(an);
            an = rec_next(an);
            vi = rec_read_rf(ai);
            ai = rec_next(ai);
            const float se = rl_f(s * residual<LOSS>(rc.r, d), 63);
            float nw[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                nw[v] = fmaf(-sl, wv[v], fmaf(se, h[v], wv[v]));
                h[v] = fmaf(se, wv[v], fmaf(-sl, h[v], h[v]));
            }
            // Hand the row on to its next use inside the window (the very next rating takes
            // it in registers), and store it.
            round_row(nw, rc.row, item, a.epoch0 + e);
            const int nxt = (int)(rc.fwd & 255u);
            if (nxt > 1) row_lstore<VEC, BF>(rows + ((u + nxt) & (D - 1)) * rb, nw);
            forwarded += nxt != 0;
            row_gstore<VEC, BF>(wlane + (int64_t)rc.row * rb, nw);
            f1 = nxt == 1;
#pragma unroll
            for (int v = 0; v < VEC; ++v) nwp[v] = nw[v];
            if (rc.info & kInfoLast) {
                lstore<VEC>(items + (size_t)slot * kp, h);
                wait_lgkm();
                if (lane == 0) sync_store(&L.flag[w], X + 1);
            }
            if ((y & (kRecBatch - 1)) == 0) load_batch();
            // Start loading the row of rating ip = y + D into slot u (or into the spare slot
            // if an update inside the window hands it on).
            if (ip < total) {
                const int prv = (int)((ifwd >> 8) & 255u);
                load_row(irow, (prv && prv <= ip) ? D : u);
            } else {
                load_row(0, D);
            }
            ++ip;
            // The row of rating y + 2, read in the next step.  (Not timed: the clock read is
            // a scalar-memory operation, and waiting for it would wait for the LDS reads
            // issued above.)
            asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * (D - 2)) : "memory");
            rc = rn;
            if (--left == 0) {
                left = cnt;
                ++e;
                xbase += nv;
                s = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(s_tab), e & 63));
                sl = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sl_tab), e & 63));
            }
        }
        wait_vm();
        if (viol && lane == 0) atomicAdd(a.counters + 0, (unsigned long long)viol);
        if (a.wstats && lane == 0) {
            unsigned long long *ws = (unsigned long long *)(a.wstats + (int64_t)q * kWStatCount);
            const uint64_t tot = tick(a.timing) - t_start;
            atomicAdd(&ws[kWStatCompTotal], (unsigned long long)tot);
            atomicMax(&ws[kWStatCompMax], (unsigned long long)tot);
            atomicAdd(&ws[kWStatItemWait], (unsigned long long)t_wait);
            atomicAdd(&ws[kWStatRatings], (unsigned long long)y);
            atomicAdd(&ws[kWStatForwarded], (unsigned long long)forwarded);
        }
    }
};

// ---------------------------------------------------------------------------------------
// Memory wave.

__device__ __forceinline__ uint32_t lds_addr(const float *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) float *)p;
}
typedef __attribute__((address_space(3))) void lds_void_t;

// LDS reads of the memory wave, waited for inside the asm block.  Written as asm so that
// the compiler does not put "s_waitcnt vmcnt(0)" in front of them (it cannot tell these
// slots from those the wave's LDS-DMA loads write).  The slots read here are never the
// target of a load in flight: a slot is read before any load into it is issued.
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
__device__ __forceinline__ int lds_read_i32_now(const int32_t *p) {
    int v;
    asm volatile("ds_read_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)"
                 : "=v"(v)
                 : "v"((uint32_t)(uintptr_t)(const __attribute__((address_space(3))) int32_t *)p)
                 : "memory");
    return v;
}

struct MemoryWave {
    const TrainArgs &a;
    const Lds &L;
    const int q, lane, kp, S;
    const int64_t vb;   // first visit record of the worker
    const int nv;       // visits per epoch
    const int V;        // visits of the call
    uint32_t *const abort_flag;
    int Xl = 0, Xr = 0; // visits taken over / passed on
    // visits held (loaded, not yet passed on): lane (X mod S)
    int f_j = 0, f_lw = 0;
    uint32_t f_tk = 0, f_nv = 0;
    // candidates: lane l = visit Xl + l; c_s, c_c: the visit's step size and step size
    // times lambda when t is the global update count
    int c_j = 0, c_lw = 0;
    uint32_t c_tk = 0, c_pv = 0, c_v = 0, c_nvis = 0;
    int64_t c_vs = 0;
    float c_s = 0.0f, c_c = 0.0f;
    int c_state = 0;    // 0 none, 1 record requested, 2 record known, 3 polled
    // items passed on this round: published once their stores are complete
    int pub_j = 0;
    uint32_t pub_tk = 0;
    int npub = 0;
    uint64_t iters = 0, misses = 0, t_mem = 0, hops = 0, viol = 0;
    const uint64_t row_mask;  // lanes that load a vector (16 bytes each)

    __device__ MemoryWave(const TrainArgs &a_, const Lds &L_, int q_, int lane_)
        : a(a_), L(L_), q(q_), lane(lane_), kp(a_.kp), S(a_.slots), vb(a_.vbase[q_]),
          nv((int)(a_.vbase[q_ + 1] - a_.vbase[q_])), V((int)(a_.vbase[q_ + 1] - a_.vbase[q_]) * a_.epochs),
          abort_flag(a_.abort_flag), row_mask((a_.kp >> 2) >= 64 ? ~0ull : ((1ull << (a_.kp >> 2)) - 1ull)) {}

    // Write items back from LDS slots with device-coherent stores: lane t < count gives
    // the item (id) and its slot.  A vector is kp / 4 lanes of 16 bytes, so one
    // instruction moves rpi = 64 / (kp / 4) vectors.
    __device__ __forceinline__ void write_back(int id, int sl, int count) {
        constexpr int kRounds = 8;
        const int lpr = kp >> 2, rpi = 64 / lpr, vbk = lane / lpr, piece = lane - vbk * lpr;
        const bool act = vbk < rpi;
        const uint32_t base = lds_addr(L.items) + (uint32_t)piece * 16u;
        for (int b0 = 0; b0 < count; b0 += kRounds * rpi) {
            int gid[kRounds];
            uint32_t src[kRounds];
#pragma unroll
            for (int r = 0; r < kRounds; ++r) {
                gid[r] = -1;
                src[r] = base;
                if (b0 + r * rpi < count) {
                    const int t = b0 + r * rpi + vbk;
                    const int g = __shfl(id, t & 63), s = __shfl(sl, t & 63);
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
                coherent_store4(a.H + (int64_t)gid[r] * kp + piece * 4, v[r]);
            }
        }
    }

    // Load item `j` into LDS slot `sl` (device-coherent LDS-DMA, 16 bytes per lane).
    __device__ __forceinline__ void load_item(int j, int sl) {
        const float *src = a.H + (int64_t)j * kp + (lane & 63) * 4;
        const uint32_t dst = lds_off(L.items) + (uint32_t)(sl * kp * 4);
        dma16_coherent(src, dst, row_mask);
    }

    __device__ __forceinline__ bool stopping() {
        return sync_load(&L.ctl[1]) != 0 ||
               __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }

    __device__ void run() {
        if (V <= 0) return;
        const uint64_t t_start = tick(a.timing);
        const int Smask = S - 1;
        uint64_t t_prog = wall_clock64();
        while (Xr < V) {
            ++iters;
            bool progress = false;
            // 1. Pass on the visits every wave of which is done (in order).
            {
                const int inflight = Xl - Xr;
                const int X = Xr + lane;
                const int sl = X & Smask;
                const int j = __shfl(f_j, sl), lw = __shfl(f_lw, sl);
                const uint32_t tk = (uint32_t)__shfl((int)f_tk, sl), nvj = (uint32_t)__shfl((int)f_nv, sl);
                bool done = false;
                if (lane < inflight) done = lds_read_i32_now(&L.flag[lw]) > X;
                const uint64_t dm = __builtin_amdgcn_ballot_w64(done);
                const int nr = leading_run(dm);
                if (nr > 0) {
                    write_back(j, sl, nr);
                    if (a.owner && lane < nr) {
                        // the item leaves this worker: its holder word must name it
                        const uint32_t was = atomicExch(a.owner + j, 0xFFFFFFFFu);
                        viol += was != (uint32_t)q;
                    }
                    // hand-offs to a later visit of the same call
                    hops += (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(
                        lane < nr && tk + 1u < (uint32_t)(a.epoch0 + a.epochs) * nvj));
                    pub_j = j;
                    pub_tk = tk + 1u;
                    npub = nr;
                    Xr += nr;
                    progress = true;
                }
            }
            // 2. Take over the candidates found free, in order, as far as slots allow.
            int nl = 0;
            {
                const bool ready = c_state == 3 && c_pv == c_tk;
                nl = leading_run(__builtin_amdgcn_ballot_w64(ready));
                const int room = Xr + S - Xl;
                if (nl > room) nl = room;
                if (nl > V - Xl) nl = V - Xl;
                if (nl < room && nl < V - Xl) {  // the next visit's item is still held elsewhere
                    const int cs = __shfl(c_state, nl & 63);
                    if (cs == 3) ++misses;
                }
                for (int t = 0; t < nl; ++t) {
                    const int j = __shfl(c_j, t);
                    load_item(j, (Xl + t) & Smask);
                }
                if (a.owner && lane < nl) {
                    // the item arrives: no other worker may hold it
                    const uint32_t was = atomicCAS(a.owner + c_j, 0xFFFFFFFFu, (uint32_t)q);
                    viol += was != 0xFFFFFFFFu;
                }
                if (nl > 0) {
                    // holder lanes: slot s takes candidate t = (s - Xl) mod S when t < nl
                    const int t = (lane - Xl) & Smask;
                    const int j = __shfl(c_j, t), lw = __shfl(c_lw, t);
                    const uint32_t tk = (uint32_t)__shfl((int)c_tk, t), nvj = (uint32_t)__shfl((int)c_nvis, t);
                    const float ts = __shfl(c_s, t), tc = __shfl(c_c, t);
                    if (lane < S && t < nl) {
                        f_j = j;
                        f_lw = lw;
                        f_tk = tk;
                        f_nv = nvj;
                        L.item[lane] = j;
                        L.ss[lane] = ts;
                        L.sc[lane] = tc;
                    }
                    if (a.trace) {
                        int64_t base = 0;
                        if (lane == 0) base = (int64_t)atomicAdd((unsigned long long *)a.trace_len,
                                                                 (unsigned long long)nl);
                        base = __shfl(base, 0);
                        if (lane < nl && base + lane < a.trace_cap) {
                            const int X = Xl + lane;
                            int32_t *tr = a.trace + 4 * (base + lane);
                            tr[0] = q;
                            tr[1] = c_j;
                            tr[2] = a.epoch0 + X / nv;
                            tr[3] = (int32_t)c_tk;
                        }
                    }
                    Xl += nl;
                    // shift the candidate window down
                    const int src = lane + nl;
                    const int sj = __shfl(c_j, src & 63), slw = __shfl(c_lw, src & 63),
                              sst = __shfl(c_state, src & 63);
                    const uint32_t stk = (uint32_t)__shfl((int)c_tk, src & 63),
                                   spv = (uint32_t)__shfl((int)c_pv, src & 63),
                                   snv = (uint32_t)__shfl((int)c_nvis, src & 63);
                    const float ss = __shfl(c_s, src & 63), sc = __shfl(c_c, src & 63);
                    const bool in = src < 64;
                    c_j = sj;
                    c_lw = slw;
                    c_tk = stk;
                    c_pv = spv;
                    c_nvis = snv;
                    c_s = ss;
                    c_c = sc;
                    c_state = in ? sst : 0;
                    progress = true;
                }
            }
            // 3. Poll the candidates whose record is known; request the missing records.
            const int X = Xl + lane;
            bool req = false;
            uint32_t e_rel = 0;
            if (X < V) {
                if (c_state >= 2) {
                    c_pv = __hip_atomic_load(a.tok_done + c_j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    c_state = 3;
                } else {
                    e_rel = (uint32_t)X / (uint32_t)nv;
                    const int x = X - (int)e_rel * nv;
                    const int4 r = *(const int4 *)(a.visits + vb + x);
                    c_j = r.x;
                    c_v = (uint32_t)r.y;
                    c_nvis = (uint32_t)r.z;
                    c_lw = r.w;
                    if (a.gstep) c_vs = a.vstart[vb + x];
                    req = true;
                }
            }
            // 4. Wait for every load and store of the round, then publish.
            {
                const uint64_t t0 = tick(a.timing);
                wait_vm();
                t_mem += tick(a.timing) - t0;
            }
            if (req) {
                bool bad = c_j < 0 || c_j >= a.n || c_lw < 0 || c_lw >= a.nw;
                if (__builtin_amdgcn_ballot_w64(bad)) {
                    if (lane == 0) raise_abort(abort_flag, L, 2u);
                    return;
                }
                c_tk = ((uint32_t)a.epoch0 + e_rel) * c_nvis + c_v;
                // t = the global count of updates before the visit, in the ring order
                if (a.gstep) step_size(a, (double)((int64_t)(a.epoch0 + (int)e_rel) * a.nnz + c_vs), c_s, c_c);
                c_state = 2;
            }
            if (npub > 0) {
                if (lane < npub)
                    __hip_atomic_store(a.tok_done + pub_j, pub_tk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                npub = 0;
            }
            if (nl > 0) {
                wait_lgkm();  // the slots' item ids are written before the visits are announced
                if (lane == 0) sync_store(&L.ctl[0], Xl);
            }
            if (progress) {
                t_prog = wall_clock64();
            } else {
                if (stopping()) break;
                if (wall_clock64() - t_prog > kWaitLimitTicks) {
                    const int st0 = __shfl(c_state, 0), j0 = __shfl(c_j, 0);
                    const uint32_t tk0 = (uint32_t)__shfl((int)c_tk, 0), pv0 = (uint32_t)__shfl((int)c_pv, 0);
                    if (lane == 0) {
                        note_timeout(a.diag, q, -1, Xr, Xl, V, st0 * 1000000 + j0);
                        a.diag[6] = (int32_t)tk0;
                        a.diag[7] = (int32_t)pv0;
                        raise_abort(abort_flag, L, 1u);
                    }
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        wait_vm();
        unsigned long long vsum = viol;
        for (int o = 32; o > 0; o >>= 1) vsum += __shfl_xor(vsum, o);
        if (lane == 0) {
            if (vsum) atomicAdd(a.counters + 0, vsum);
            if (hops) atomicAdd(a.counters + 1, (unsigned long long)hops);
        }
        if (a.wstats && lane == 0) {
            unsigned long long *ws = (unsigned long long *)(a.wstats + (int64_t)q * kWStatCount);
            atomicAdd(&ws[kWStatMemTotal], (unsigned long long)(tick(a.timing) - t_start));
            atomicAdd(&ws[kWStatMemIters], (unsigned long long)iters);
            atomicAdd(&ws[kWStatVisits], (unsigned long long)Xl);
            atomicAdd(&ws[kWStatPollMiss], (unsigned long long)misses);
            atomicAdd(&ws[kWStatMemWait], (unsigned long long)t_mem);
        }
    }
};

// ---------------------------------------------------------------------------------------
// Asynchronous schedule: Algorithm 1 with the random-permutation circulation of section
// 3.4.  Every worker has an inbound queue of items in device memory (lock-free: a producer
// reserves a position with an atomic increment of the queue's tail and writes the entry
// (position + 1, holder entry) with one 64-bit device-coherent store; the consumer reads
// positions in order and takes an entry once its position matches).  A worker takes items
// in arrival order; after its last compute wave is done with an item it writes h_j back
// (device-coherent), passes it to the next worker of the item's visiting order for the
// epoch, or parks it after the launch's last epoch.  The visiting order of item j in epoch
// e is a keyed pseudo-random permutation of its holders (a fresh one every epoch), so every
// rating is updated once per epoch and t = e.

// Position -> holder rank of item j's visiting order in epoch e: a keyed bijection of
// [0, nh).  Eight alternating half-steps of a Feistel network (each xors one half of the
// bits with a hash of the other half, so each is invertible) permute [0, 2^b), 2^b >= nh
// the smallest such power of two; values outside [0, nh) are mapped again until one falls
// inside (cycle walking), which keeps the map a bijection of [0, nh).  Fewer than two
// passes are needed on average, and the cost does not grow with nh.  Halves are only a few
// bits wide here (three for 64 holders), and with four half-steps the orders showed it:
// consecutive ranks followed each other about 25% more often than in a uniform
// permutation at 256 holders, many times more at 64; with eight the frequencies of
// consecutive-rank gaps and of rank positions are those of uniform permutations.
__device__ __forceinline__ uint32_t visit_rank(uint32_t seed, int j, int e, uint32_t nh, uint32_t x) {
    if (nh <= 1u) return 0u;
    const int b = 32 - __builtin_clz(nh - 1u);
    const int lo = b >> 1;
    const uint32_t mlo = (1u << lo) - 1u, mhi = (1u << (b - lo)) - 1u;
    const uint32_t key = lowbias32(lowbias32(seed ^ (uint32_t)j) ^ ((uint32_t)e * 0x9E3779B9u));
    do {
        uint32_t L = x >> lo, R = x & mlo;
#pragma unroll
        for (uint32_t r = 0; r < 8u; r += 2u) {
            L ^= lowbias32(R ^ (key + r * 0x9E3779B9u)) & mhi;
            R ^= lowbias32(L ^ (key + (r + 1u) * 0x9E3779B9u)) & mlo;
        }
        x = (L << lo) | R;
    } while (x >= nh);
    return x;
}

// Per-item state words (TrainArgs::istate), read and written device-coherently: the item's
// holder writes them before the item moves on, the next holder reads them after taking it.
__device__ __forceinline__ int4 istate_load(const TrainArgs &a, int j) {
    const uint64_t *p = (const uint64_t *)(a.istate + 4 * (int64_t)j);
    const uint64_t u0 = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t u1 = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_int4((int)(uint32_t)u0, (int)(uint32_t)(u0 >> 32), (int)(uint32_t)u1, (int)(uint32_t)(u1 >> 32));
}
__device__ __forceinline__ void istate_store(const TrainArgs &a, int j, int4 v) {
    uint64_t *p = (uint64_t *)(a.istate + 4 * (int64_t)j);
    __hip_atomic_store(p, (uint64_t)(uint32_t)v.x | ((uint64_t)(uint32_t)v.y << 32), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 1, (uint64_t)(uint32_t)v.z | ((uint64_t)(uint32_t)v.w << 32), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// W's stored row elements of the lane to FP32 registers (global memory).
template <int VEC, bool BF>
__device__ __forceinline__ void row_gload(const char *p, float (&v)[VEC]) {
    if constexpr (!BF) {
        vload<VEC>((const float *)p, v);
    } else if constexpr (VEC == 1) {
        v[0] = __uint_as_float((uint32_t)*(const uint16_t *)p << 16);
    } else if constexpr (VEC == 2) {
        const uint32_t t = *(const uint32_t *)p;
        v[0] = __uint_as_float(t << 16);
        v[1] = __uint_as_float(t & 0xFFFF0000u);
    } else {
        const uint2 t = *(const uint2 *)p;
        v[0] = __uint_as_float(t.x << 16);
        v[1] = __uint_as_float(t.x & 0xFFFF0000u);
        v[2] = __uint_as_float(t.y << 16);
        v[3] = __uint_as_float(t.y & 0xFFFF0000u);
    }
}

// Compute wave of the asynchronous schedule: takes the worker's visits in the order the
// memory wave announces them; for each, runs the SGD updates of its own ratings of the
// item (its rows, ascending) and passes the item to the next wave.  A visit's records are
// read 64 at a time into lane registers (one vector load; lane l holds the l-th); the row
// of the next rating is loaded while the current one is updated (rows of one visit are
// distinct, so the load never overtakes a store of the same row).
template <int VEC, bool BF, int LOSS, bool KEEP, int RND>
struct AsyncComputeWave {
    static constexpr int ES = BF ? 2 : 4;
    const TrainArgs &a;
    const Lds &L;
    const int q, w, lane, kp, loff, rb;
    const RatingRec *rs;  // the wave's records, grouped by local item
    lds_float *const items;
    char *const W;
    const uint32_t lb;    // the lane's byte offset inside a row
    uint64_t nrat = 0, t_wait = 0;
    uint32_t viol = 0;    // ownership checks: ratings of rows the wave does not own
    // KEEP (layouts with a row that holds more than half of a compute wave's share of the
    // ratings): the row of the last update of this wave's last batch, its stored value in the
    // wave's row region of the LDS layout (unused otherwise here) and its index in `kept`
    // (-1: none kept).  A visit whose only rating for this wave is on that row takes the row
    // from here instead of memory: only this wave writes its rows, so the kept copy is the
    // row's current value.  A row rated by nearly every item dominates its wave, which then
    // gets from nearly every item a visit of one rating on that row.  The kernel is compiled
    // with and without this path: its mere presence costs the other layouts a few percent.
    __device__ __forceinline__ lds_float *keep() const {
        return to_lds((float *)(L.rows + (size_t)w * (kAsyncWindow + 1) * kp * ES));
    }

    __device__ AsyncComputeWave(const TrainArgs &a_, const Lds &L_, int q_, int w_, int lane_, int64_t r0)
        : a(a_), L(L_), q(q_), w(w_), lane(lane_), kp(a_.kp), loff(lane_ * VEC), rb(a_.kp * ES), rs(a_.recs + r0),
          items(to_lds(L_.items) + lane_ * VEC), W((char *)a_.W), lb((uint32_t)(lane_ * VEC * ES)) {}
    int kept = -1;  // the kept row's index (a scalar register: the check costs no LDS round trip)

    // The lane's part of row `row` (uniform).
    __device__ __forceinline__ char *lane_row(int row) const { return W + (int64_t)row * rb + lb; }

    // Row addresses of a batch of records: lane l holds the address of record l's row,
    // formed once per batch (one vector multiply-add for 64 rows), and row(x) takes record
    // x's out of the lanes into scalar registers, where the row's load and, later, its store
    // use it with the lane's offset (no 64-bit multiply per access).
    struct RowAddr {
        uint32_t lo, hi;
        __device__ __forceinline__ uint64_t row(int x) const {
            return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)hi, x) << 32) |
                   (uint32_t)__builtin_amdgcn_readlane((int)lo, x);
        }
    };
    // The lane's part of the row at uniform address `base`: global-memory accesses with the
    // row's address in scalar registers and the lane's 32-bit byte offset.
    typedef __attribute__((address_space(1))) char gchar;
    __device__ __forceinline__ void gload(uint64_t base, float (&v)[VEC]) const {
        const gchar *p = (const gchar *)base + lb;
        if constexpr (!BF) {
            if constexpr (VEC == 1) v[0] = *(const __attribute__((address_space(1))) float *)p;
            if constexpr (VEC == 2) {
                const f32x2v t = *(const __attribute__((address_space(1))) f32x2v *)p;
                v[0] = t.x;
                v[1] = t.y;
            }
            if constexpr (VEC == 4) {
                const f32x4v t = *(const __attribute__((address_space(1))) f32x4v *)p;
                v[0] = t.x;
                v[1] = t.y;
                v[2] = t.z;
                v[3] = t.w;
            }
        } else if constexpr (VEC == 1) {
            v[0] = __uint_as_float((uint32_t)*(const __attribute__((address_space(1))) uint16_t *)p << 16);
        } else if constexpr (VEC == 2) {
            const uint32_t t = *(const __attribute__((address_space(1))) uint32_t *)p;
            v[0] = __uint_as_float(t << 16);
            v[1] = __uint_as_float(t & 0xFFFF0000u);
        } else {
            const u32x2v t = *(const __attribute__((address_space(1))) u32x2v *)p;
            v[0] = __uint_as_float(t.x << 16);
            v[1] = __uint_as_float(t.x & 0xFFFF0000u);
            v[2] = __uint_as_float(t.y << 16);
            v[3] = __uint_as_float(t.y & 0xFFFF0000u);
        }
    }
    __device__ __forceinline__ void gstore(uint64_t base, const float (&v)[VEC]) const {
        gchar *p = (gchar *)base + lb;
        if constexpr (!BF) {
            if constexpr (VEC == 1) *(__attribute__((address_space(1))) float *)p = v[0];
            if constexpr (VEC == 2) *(__attribute__((address_space(1))) f32x2v *)p = f32x2v{v[0], v[1]};
            if constexpr (VEC == 4) *(__attribute__((address_space(1))) f32x4v *)p = f32x4v{v[0], v[1], v[2], v[3]};
        } else if constexpr (VEC == 1) {
            *(__attribute__((address_space(1))) uint16_t *)p = (uint16_t)(__float_as_uint(v[0]) >> 16);
        } else if constexpr (VEC == 2) {
            *(__attribute__((address_space(1))) uint32_t *)p = bf_pair<VEC>(v, 0);
        } else {
            *(__attribute__((address_space(1))) u32x2v *)p = u32x2v{bf_pair<VEC>(v, 0), bf_pair<VEC>(v, 2)};
        }
    }
    __device__ __forceinline__ RowAddr row_addresses(int crow) const {
        const uint64_t ad = (uint64_t)(uintptr_t)W + (uint64_t)(uint32_t)crow * (uint64_t)(uint32_t)rb;
        return RowAddr{(uint32_t)ad, (uint32_t)(ad >> 32)};
    }

    // Wait until visit X reaches this wave.  False when the worker stops with no such visit.
    __device__ __forceinline__ bool wait_visit(const int32_t *word, int X) {
        if (sync_load(word) > X) return true;
        const uint64_t t0 = wall_clock64();
        while (sync_load(word) <= X) {
            if (sync_load(&L.ctl[1])) return sync_load(word) > X;
            if (wall_clock64() - t0 > kWaitLimitTicks) {
                if (lane == 0) {
                    note_timeout(a.diag, q, w, X, sync_load(word), 100, sync_load(&L.ctl[0]));
                    raise_abort(a.abort_flag, L, 1u);
                }
                return false;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        return true;
    }

    // One update (section 2.3: one residual, both vectors from their values before it).
    // TO_KEEP: also keep the stored row in LDS as this wave's kept row.
    template <bool TO_KEEP = false>
    __device__ __forceinline__ void update(float (&h)[VEC], const float (&wv)[VEC], int row, uint64_t rowp,
                                           float rating, float s, float sl, int item, int t) {
        float d = 0.0f;
#pragma unroll
        for (int i = 0; i < VEC; ++i) d = fmaf(wv[i], h[i], d);
        d = wave_sum_last(d);
        const float se = rl_f(s * residual<LOSS>(rating, d), 63);
        float nw[VEC];
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            // w + se h - s lambda w as two FMAs, the first after the residual: a product of
            // w alone would be scheduled early, for rows of later ratings, and wait for
            // their loads there.
            nw[i] = fmaf(-sl, wv[i], fmaf(se, h[i], wv[i]));
            h[i] = fmaf(se, wv[i], fmaf(-sl, h[i], h[i]));
        }
        round_stored<VEC, BF, RND>(a, loff, nw, row, item, t);
        gstore(rowp, nw);
        if constexpr (TO_KEEP) {
            lstore<VEC>(keep() + loff, nw);
            kept = row;
        }
    }

    // The wave's record range of visit X, left in LDS by the memory wave ([b, e); b = e when
    // the worker holds no rating of the item or the wave none of its ratings).
    __device__ __forceinline__ void range(int X, int64_t &b, int64_t &e) const {
        const int sl = X & (a.slots - 1);
        const int x = __builtin_amdgcn_readfirstlane(L.sx[sl]);  // -1: the worker holds no rating of the item
        b = e = 0;
        if (x >= 0) {
            const int32_t *rng = (const int32_t *)L.recs;
            b = __builtin_amdgcn_readfirstlane(rng[w * kMaxItemSlots + sl]);
            e = __builtin_amdgcn_readfirstlane(rng[(a.nw + w) * kMaxItemSlots + sl]);
        }
    }

    __device__ void run() {
        const uint64_t t_start = tick(a.timing);
        const int32_t *word = w == 0 ? &L.ctl[0] : &L.flag[w - 1];
        // The first records of a later visit, loaded while this one is updated: `pre` holds
        // them (lane l: record l) for visit pre_X.
        int pre_X = -1;
        u32x2v pre = {0u, 0u};
        for (int X = 0;; ++X) {
            const uint64_t t0 = tick(a.timing);
            if (!wait_visit(word, X)) break;
            compiler_fence();
            t_wait += tick(a.timing) - t0;
            const int sl = X & (a.slots - 1);
            int64_t b, e;
            range(X, b, e);
            if (b < e) {
                const int t = __builtin_amdgcn_readfirstlane(L.se[sl]);
                const int item = __builtin_amdgcn_readfirstlane(L.item[sl]);
                float h[VEC];
                lload<VEC>(items + (size_t)sl * kp, h);
                const float s = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(L.ss[sl])));
                const float slam = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(L.sc[sl])));
                for (int64_t r0 = b; r0 < e; r0 += 64) {
                    const int nb = (int)(e - r0 < 64 ? e - r0 : 64);
                    // lane l: record r0 + l (row, rating)
                    int crow = 0;
                    float crat = 0.0f;
                    if (r0 == b && pre_X == X) {
                        const uint32_t p0 = pre.x, p1 = pre.y;
                        crow = (int)p0;
                        crat = __uint_as_float(p1);
                    } else {
                        if (lane < nb) {
                            const u32x2v rv = *(const u32x2v *)(rs + r0 + lane);
                            const uint32_t v0 = rv.x, v1 = rv.y;
                            crow = (int)v0;
                            crat = __uint_as_float(v1);
                        }
                        // the records are in place here, so that no path into what follows
                        // leaves a load of them pending
                        asm volatile("" : "+v"(crow), "+v"(crat));
                    }
                    if (a.owner) {
                        // every rating of the batch is of a row this wave owns
                        const int64_t lo = a.wave_start[(int64_t)q * a.nw + w], hi = a.wave_start[(int64_t)q * a.nw + w + 1];
                        viol += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(lane < nb && (crow < lo || crow >= hi)));
                    }
                    if (r0 == b) {
                        // The next visit's first records, if it is announced and has ratings
                        // of this wave (else this visit's again: no branch around the load).
                        int64_t pb = b, pe = e;
                        int px = -1;
                        if (sync_load(&L.ctl[0]) > X + 1) {
                            int64_t b1, e1;
                            range(X + 1, b1, e1);
                            if (b1 < e1) {
                                pb = b1;
                                pe = e1;
                                px = X + 1;
                            }
                        }
                        const int pn = (int)(pe - pb < 64 ? pe - pb : 64);
                        if (lane < pn) pre = *(const u32x2v *)(rs + pb + lane);
                        pre_X = px;
                    }
                    if constexpr (KEEP) {
                        if (nb == 1 && __builtin_amdgcn_readfirstlane(crow) == kept) {
                            // one rating, on the row kept from this wave's last batch: no load
                            const RowAddr ra = row_addresses(crow);
                            float wv[VEC];
                            lload<VEC>(keep() + loff, wv);
                            update<true>(h, wv, kept, ra.row(0),
                                         __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(crat))), s, slam,
                                         item, t);
                            continue;
                        }
                    }
                    // Sixteen row buffers: the row of rating l + 16 is loaded while rating l is
                    // updated.  Groups of four updates run in a branch-free body with
                    // unconditional loads (indices past the batch clamped to its last rating),
                    // and the way into the loop leaves the same pattern of loads and stores as
                    // a pass of it, so that the compiler's wait counts stay exact (a
                    // conditional load or store makes it wait for everything).
                    constexpr int NB = 16;
                    float wbuf[NB][VEC];
                    int rbuf[NB];     // row indices (the stochastic rounding key uses them)
                    uint64_t abuf[NB];  // row addresses (uniform)
                    const RowAddr ra = row_addresses(crow);
#pragma unroll
                    for (int k = 0; k < NB; ++k) {
                        rbuf[k] = __builtin_amdgcn_readlane(crow, k < nb ? k : nb - 1);
                        abuf[k] = ra.row(k < nb ? k : nb - 1);
                        gload(abuf[k], wbuf[k]);
                        // every lane, no branch; a different value each time, so that no
                        // store is merged into another
                        if (k + 1 < NB) a.dummy[(int64_t)q * kMaxWaves + w] = (float)k;
                    }
                    int l = 0;
                    for (; l + NB <= nb; l += NB) {
#pragma unroll
                        for (int k = 0; k < NB; ++k) {
                            update(h, wbuf[k], rbuf[k], abuf[k],
                                   __int_as_float(__builtin_amdgcn_readlane(__float_as_int(crat), l + k)), s, slam, item, t);
                            const int nl = l + k + NB;
                            rbuf[k] = __builtin_amdgcn_readlane(crow, nl < nb ? nl : nb - 1);
                            abuf[k] = ra.row(nl < nb ? nl : nb - 1);
                            gload(abuf[k], wbuf[k]);
                        }
                    }
                    if constexpr (KEEP) kept = -1;  // kept only when the batch's last update is below
#pragma unroll
                    for (int k = 0; k < NB - 1; ++k)
                        if (l + k < nb) {
                            const float rk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(crat), l + k));
                            if (KEEP && l + k == nb - 1)
                                update<KEEP>(h, wbuf[k], __builtin_amdgcn_readlane(crow, l + k), abuf[k], rk, s, slam,
                                             item, t);
                            else
                                update(h, wbuf[k], rbuf[k], abuf[k], rk, s, slam, item, t);
                        }
                }
                nrat += (uint64_t)(e - b);
                lstore<VEC>(items + (size_t)sl * kp, h);
                wait_lgkm();
            }
            if (lane == 0) sync_store(&L.flag[w], X + 1);
        }
        wait_vm();
        if (viol && lane == 0) atomicAdd(a.counters + 0, (unsigned long long)viol);
        if (a.wstats && lane == 0) {
            unsigned long long *ws = (unsigned long long *)(a.wstats + (int64_t)q * kWStatCount);
            const uint64_t tot = tick(a.timing) - t_start;
            atomicAdd(&ws[kWStatCompTotal], (unsigned long long)tot);
            atomicMax(&ws[kWStatCompMax], (unsigned long long)tot);
            atomicAdd(&ws[kWStatItemWait], (unsigned long long)t_wait);
            atomicAdd(&ws[kWStatRatings], (unsigned long long)nrat);
        }
    }
};

// Uniform routing (Algorithm 1 as printed): the next worker of item j after its v-th move.
__device__ __forceinline__ int route_uniform(uint32_t seed, int j, int v, int p) {
    const uint32_t k = lowbias32(lowbias32(seed ^ 0x2545F491u ^ (uint32_t)j) + (uint32_t)v * 0x9E3779B9u);
    return (int)(((uint64_t)k * (uint64_t)(uint32_t)p) >> 32);
}

// Payload of a queue entry: the holder entry of the visit, or (uniform routing, for a
// worker holding no rating of the item) kPassBit | item.
constexpr uint32_t kPassBit = 0x80000000u;

// Memory wave of the asynchronous schedules.
//   Queue entries: (position + 1) << 32 | payload (see kPassBit).  Random permutation:
//   items only go to workers holding their ratings, and worker q's queue has room for its
//   local items; uniform routing: any item may come, room for n.
//   Per visit the wave works out t (the epoch, or the number of earlier visits of the item
//   to this worker, or the global update count) and the step size, for the compute waves.
//   Taking an item over costs two rounds of dependent loads after its queue entry: the
//   holder tables of the entry, then the item's state words, its vector (LDS-DMA) and the
//   compute waves' record ranges.
struct AsyncMemoryWave {
    const TrainArgs &a;
    const Lds &L;
    MemoryWave io;        // item loads and write-backs
    const int q, lane, S;
    const bool uni;       // uniform routing
    const int64_t qb;     // inbound queue: [qb, qb + cap)
    const int64_t cap;
    const int64_t vbq;    // the worker's first visit record
    const int nvq;        // the worker's local items
    int Xl = 0, Xr = 0;   // visits taken / passed on
    int64_t head = 0;     // next queue position to take
    // lane s < S: the visit in slot s: item, holder entry (-1 if none), step counter t, the
    // item's state words (epoch or moves, position, visits), its first holder entry and
    // number of holders
    int f_j = 0, f_g = -1, f_t = 0, f_e = 0, f_pos = 0, f_seq = 0, f_hb = 0, f_nh = 0, f_cr = -1;
    // step sizes of t = tbase + lane
    int tbase = 0;
    float s_tab = 0.0f, c_tab = 0.0f;
    uint64_t iters = 0, misses = 0, hops = 0, viol = 0;
    // sums over rounds: free slots, queue length (with collect_stats), rounds whose first
    // queue entry was not yet written while a later one was, visits passed on, visits held
    uint64_t s_room = 0, s_qlen = 0, s_hol = 0, s_nr = 0, s_held = 0;

    __device__ AsyncMemoryWave(const TrainArgs &a_, const Lds &L_, int q_, int lane_)
        : a(a_), L(L_), io(a_, L_, q_, lane_), q(q_), lane(lane_), S(a_.slots), uni(a_.sched == 2),
          qb(a_.sched == 2 ? (int64_t)q_ * a_.n : a_.vbase[q_]),
          cap(a_.sched == 2 ? a_.n : a_.vbase[q_ + 1] - a_.vbase[q_]), vbq(a_.vbase[q_]),
          nvq((int)(a_.vbase[q_ + 1] - a_.vbase[q_])) {
        // the permutation's t is the epoch, within [epoch0, epoch0 + epochs); uniform
        // routing's per-pair counts stay near the epochs done
        tbase = uni ? (a.epoch0 > 32 ? a.epoch0 - 32 : 0) : a.epoch0;
        step_size(a, (double)(tbase + lane), s_tab, c_tab);
    }

    // Items waiting in worker q2's queue (pushed, not yet taken): the load that section 3.3's
    // rule compares.  The two counters are read at slightly different moments, so a head
    // read after the tail can pass it; such a reading counts as an empty queue.
    __device__ __forceinline__ int queue_load(int q2) const {
        const uint32_t tl = __hip_atomic_load(a.qtail + q2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t hd = __hip_atomic_load(a.qhead + q2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int d = (int)(tl - hd);
        return d > 0 ? d : 0;
    }

    // Push the item to worker q2's queue with payload `pay`.
    __device__ __forceinline__ void push(int q2, uint32_t pay) {
        const int64_t b2 = uni ? (int64_t)q2 * a.n : a.vbase[q2];
        const int64_t cap2 = uni ? a.n : a.vbase[q2 + 1] - b2;
        const uint32_t pos = atomicAdd(a.qtail + q2, 1u);
        const uint64_t ent = ((uint64_t)(pos + 1u) << 32) | pay;
        __hip_atomic_store(a.queue + b2 + (int64_t)(pos % (uint64_t)cap2), ent, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }

    // 1. Pass on the visits the last compute wave has finished (in order): write h_j back,
    //    work out the next worker, write the item's state words, then push.
    __device__ __forceinline__ bool pass_on() {
        int nr = sync_load(&L.flag[a.nw - 1]) - Xr;
        if (nr > 64) nr = 64;
        if (nr <= 0) return false;
        s_nr += (uint64_t)nr;
        const int Smask = S - 1;
        const int X = Xr + lane;
        const int sl = X & Smask;
        const int j = __shfl(f_j, sl), g = __shfl(f_g, sl), t = __shfl(f_t, sl), e = __shfl(f_e, sl),
                  pos = __shfl(f_pos, sl), seq = __shfl(f_seq, sl), hb = __shfl(f_hb, sl), nh = __shfl(f_nh, sl),
                  cr = __shfl(f_cr, sl);
        io.write_back(j, sl, nr);
        const bool mine = lane < nr;
        int dest = -1;  // next worker, -1: the item is parked
        uint32_t pay = 0;
        int4 nst = make_int4(0, 0, g >= 0 ? seq + 1 : seq, -1);
        unsigned long long done_upd = 0;
        if (mine) {
            if (uni) {
                if (g >= 0) {
                    if (!a.gstep) a.tvis[g] = t + 1;
                    done_upd = (unsigned long long)a.hcnt[g];
                }
            } else {
                // The next holder: the next position of the epoch's visiting order (or the first
                // of the next epoch once every holder was visited).  With load balancing
                // (section 3.3) two holders not yet visited are candidates, the one held over
                // from the last choice (if any) and the next of the order, and the one whose
                // queue holds fewer items goes next; the other is held over.
                int fp = pos, carry = cr, ne = e;
                if (fp >= nh && carry < 0) {
                    fp = 0;
                    ++ne;
                }
                if (ne < a.epoch0 + a.epochs) {
                    int ra;
                    if (carry >= 0) {
                        ra = carry;
                        carry = -1;
                    } else {
                        ra = (int)visit_rank(a.route_seed, j, ne, (uint32_t)nh, (uint32_t)fp++);
                    }
                    int pick = ra;
                    if (a.balance && fp < nh) {
                        const int rb = (int)visit_rank(a.route_seed, j, ne, (uint32_t)nh, (uint32_t)fp++);
                        const int qa = a.hold[hb + ra], qb = a.hold[hb + rb];
                        const bool take_b = queue_load(qb) < queue_load(qa);
                        pick = take_b ? rb : ra;
                        carry = take_b ? ra : rb;
                    }
                    const int ng = hb + pick;
                    dest = a.hold[ng];
                    pay = (uint32_t)ng;
                }
                nst.x = ne;
                nst.y = fp;
                nst.w = carry;
            }
        }
        if (uni) {
            // updates of these visits, then: keep the items moving until the budget is met
            unsigned long long sum = done_upd;
            for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
            unsigned long long before = 0;
            if (lane == 0) before = atomicAdd(a.upd, sum);
            before = __shfl(before, 0);
            if (mine) {
                nst.x = e;  // moves so far
                if (before + sum < a.budget) {
                    dest = route_uniform(a.route_seed, j, e, a.p);
                    if (a.balance) {
                        // section 3.3: the less loaded of two uniformly drawn workers
                        const int d2 = route_uniform(a.route_seed ^ 0x5BD1E995u, j, e, a.p);
                        if (queue_load(d2) < queue_load(dest)) dest = d2;
                    }
                    nst.x = e + 1;
                    const int g2 = a.hmap[(int64_t)dest * a.n + j];
                    pay = g2 >= 0 ? (uint32_t)g2 : (kPassBit | (uint32_t)j);
                }
            }
        }
        if (mine) istate_store(a, j, nst);
        if (a.owner && mine) {
            // the item leaves this worker: its holder word must name it
            const uint32_t was = atomicExch(a.owner + j, 0xFFFFFFFFu);
            viol += was != (uint32_t)q;
        }
        wait_vm();  // the item vectors and state words are in place before the items move on
        if (mine && dest >= 0) push(dest, pay);
        hops += (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(mine && dest >= 0));
        const int np = __popcll(__builtin_amdgcn_ballot_w64(mine && dest < 0));
        if (np > 0 && lane == 0) atomicAdd(a.parked, (uint32_t)np);
        Xr += nr;
        return true;
    }

    // 2. Take over arrived items, in arrival order, as far as slots allow.
    __device__ __forceinline__ bool take_over() {
        int room = Xr + S - Xl;
        if (room > 64) room = 64;
        s_held += (uint64_t)(Xl - Xr);
        if (room > 0) s_room += (uint64_t)room;
        if (a.timing && cap > 0) {
            const int ql = (int)(__hip_atomic_load(a.qtail + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                                 (uint32_t)head);
            s_qlen += (uint64_t)(ql > 0 ? ql : 0);
        }
        if (room <= 0 || cap <= 0) return false;
        const int Smask = S - 1;
        uint64_t ent = 0;
        bool valid = false;
        if (lane < room) {
            ent = __hip_atomic_load(a.queue + qb + (head + lane) % cap, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            valid = (uint32_t)(ent >> 32) == (uint32_t)(head + lane + 1);
        }
        const uint64_t vb = __builtin_amdgcn_ballot_w64(valid);
        const int nt = leading_run(vb);
        if (nt <= 0) {
            ++misses;
            s_hol += vb != 0;
            return false;
        }
        const bool mine = lane < nt;
        // the holder tables of the entry
        int j = 0, g = -1, x = -1, t = 0, cnt = 0;
        if (mine) {
            const uint32_t pay = (uint32_t)ent;
            if (pay & kPassBit) {
                j = (int)(pay & ~kPassBit);
            } else {
                g = (int)pay;
                j = a.hitem[g];
                x = a.hx[g];
                cnt = a.hcnt[g];
                if (uni) t = a.tvis[g];
            }
        }
        // the item's vector and state words
        for (int k = 0; k < nt; ++k) io.load_item(__shfl(j, k), (Xl + k) & Smask);
        int4 st = make_int4(0, 0, 0, 0);
        int hb = 0, nh = 0;
        if (mine) {
            st = istate_load(a, j);
            if (!uni) {
                const int64_t h0 = a.hoff[j];
                hb = (int)h0;
                nh = (int)(a.hoff[j + 1] - h0);
                t = st.x;  // the epoch
            }
        }
        {
            // Every compute wave's record range of the new visits, into LDS (the record ring
            // of the ring kernel's layout, unused here): one batched load here instead of a
            // dependent load at the start of every visit in every compute wave.
            int32_t *rng = (int32_t *)L.recs;
            const int sl = (Xl + lane) & Smask;
            for (int w2 = 0; w2 < a.nw; ++w2) {
                int bw = 0, ew = 0;
                if (mine && x >= 0) {
                    const int64_t v = vbq + x;
                    bw = a.xoff[v * a.nw + w2];
                    ew = x + 1 < nvq ? a.xoff[(v + 1) * a.nw + w2]
                                     : (int)(a.rbase[(int64_t)q * a.nw + w2 + 1] - a.rbase[(int64_t)q * a.nw + w2]);
                }
                if (mine) {
                    rng[w2 * kMaxItemSlots + sl] = bw;
                    rng[(a.nw + w2) * kMaxItemSlots + sl] = ew;
                }
            }
        }
        if (a.owner && mine) {
            // the item arrives: no other worker may hold it
            const uint32_t was = atomicCAS(a.owner + j, 0xFFFFFFFFu, (uint32_t)q);
            viol += was != 0xFFFFFFFFu;
        }
        // step size of the visit: from the table, else computed
        double tg = (double)t;
        if (a.gstep && mine && g >= 0) {
            // the global count of updates before the visit (visits are counted in the order
            // they are taken, which is an order that every row and item sees)
            tg = (double)atomicAdd(a.counters + 2, (unsigned long long)cnt);
            t = (int)(uint32_t)(unsigned long long)tg;
        }
        const int ti = t - tbase;
        float sv = __shfl(s_tab, ti & 63), cv = __shfl(c_tab, ti & 63);
        if (mine && (a.gstep || ti < 0 || ti >= 64)) step_size(a, tg, sv, cv);
        if (mine) {
            const int sl = (Xl + lane) & Smask;
            L.sx[sl] = x;
            L.se[sl] = t;
            L.ss[sl] = sv;
            L.sc[sl] = cv;
            L.item[sl] = j;
        }
        {
            const int k = (lane - Xl) & Smask;
            const int tj = __shfl(j, k), tg2 = __shfl(g, k), tt = __shfl(t, k), te = __shfl(st.x, k),
                      tp = __shfl(st.y, k), ts = __shfl(st.z, k), thb = __shfl(hb, k), tnh = __shfl(nh, k),
                      tcr = __shfl(st.w, k);
            if (lane < S && k < nt) {
                f_cr = tcr;
                f_j = tj;
                f_g = tg2;
                f_t = tt;
                f_e = te;
                f_pos = tp;
                f_seq = ts;
                f_hb = thb;
                f_nh = tnh;
            }
        }
        if (a.trace) {
            // the visits that update something (uniform routing also visits workers holding
            // no rating of the item)
            const uint64_t rec = __builtin_amdgcn_ballot_w64(mine && g >= 0);
            const int nrec = __popcll(rec);
            int64_t base = 0;
            if (lane == 0 && nrec > 0)
                base = (int64_t)atomicAdd((unsigned long long *)a.trace_len, (unsigned long long)nrec);
            base = __shfl(base, 0);
            const int rank = __popcll(rec & ((1ull << lane) - 1ull));
            if (mine && g >= 0 && base + rank < a.trace_cap) {
                int32_t *tr = a.trace + 4 * (base + rank);
                tr[0] = q;
                tr[1] = j;
                tr[2] = t;
                tr[3] = st.z;
            }
        }
        head += nt;
        Xl += nt;
        if (a.balance && lane == 0)
            __hip_atomic_store(a.qhead + q, (uint32_t)head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_vm();    // the item vectors are in LDS
        wait_lgkm();  // and so are the slots' descriptions
        if (lane == 0) sync_store(&L.ctl[0], Xl);
        return true;
    }

    __device__ void run() {
        const uint64_t t_start = tick(a.timing);
        uint64_t t_prog = wall_clock64();
        while (true) {
            ++iters;
            bool progress = pass_on();
            progress = take_over() || progress;
            // Done when every item has stopped moving and nothing is held.
            if (Xr == Xl &&
                (int64_t)__hip_atomic_load(a.parked, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= a.active)
                break;
            if (progress) {
                t_prog = wall_clock64();
            } else {
                if (sync_load(&L.ctl[1]) != 0 ||
                    __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                    break;
                if (wall_clock64() - t_prog > kWaitLimitTicks) {
                    if (lane == 0) {
                        note_timeout(a.diag, q, -1, Xr, Xl, (int)head, (int)__hip_atomic_load(
                                         a.parked, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                        raise_abort(a.abort_flag, L, 1u);
                    }
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        wait_vm();
        if (lane == 0) sync_store(&L.ctl[1], 1);  // compute waves: no more visits
        // per-lane counts (violations) summed over the wave
        unsigned long long vsum = viol;
        for (int o = 32; o > 0; o >>= 1) vsum += __shfl_xor(vsum, o);
        if (lane == 0) {
            if (vsum) atomicAdd(a.counters + 0, vsum);
            if (hops) atomicAdd(a.counters + 1, (unsigned long long)hops);
        }
        if (a.wstats && lane == 0) {
            unsigned long long *ws = (unsigned long long *)(a.wstats + (int64_t)q * kWStatCount);
            atomicAdd(&ws[kWStatMemTotal], (unsigned long long)(tick(a.timing) - t_start));
            atomicAdd(&ws[kWStatMemIters], (unsigned long long)iters);
            atomicAdd(&ws[kWStatVisits], (unsigned long long)Xl);
            atomicAdd(&ws[kWStatPollMiss], (unsigned long long)misses);
            atomicAdd(&ws[kWStatRoom], (unsigned long long)s_room);
            atomicAdd(&ws[kWStatQueueLen], (unsigned long long)s_qlen);
            atomicAdd(&ws[kWStatBlocked], (unsigned long long)s_hol);
            atomicAdd(&ws[kWStatPassed], (unsigned long long)s_nr);
            atomicAdd(&ws[kWStatHeld], (unsigned long long)s_held);
            // hardware register XCC_ID (bits 3:0): the die this workgroup was placed on
            a.wstats[(int64_t)q * kWStatCount + kWStatXcd] = (int64_t)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);
        }
    }
};

template <int VEC, int D, bool BF, int LOSS, bool KEEP, int RND>
__global__ __launch_bounds__(64 * (kMaxWavesAsync + 1)) void k_worker_async(TrainArgs a) {
    extern __shared__ float4 lds4[];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x;
    const Lds L = lds_layout(lds4, a.kp, a.nw, a.slots, D, BF ? 2 : 4);
    if (threadIdx.x < kMaxWaves + 1) L.flag[threadIdx.x] = 0;
    if (threadIdx.x < 2) L.ctl[threadIdx.x] = 0;
    __syncthreads();
    if (q >= a.p || a.epochs <= 0) return;
    if (wave < a.nw) {
        AsyncComputeWave<VEC, BF, LOSS, KEEP, RND> cw(a, L, q, wave, lane, a.rbase[(int64_t)q * a.nw + wave]);
        cw.run();
    } else if (wave == a.nw) {
        AsyncMemoryWave mw(a, L, q, lane);
        mw.run();
    }
}

// Seeding: the first worker of every item (sort key; p for an item without ratings) and the
// payload of its queue entry.  Random permutation: the holder at position 0 of the item's
// visiting order for epoch a.epoch0 (payload: that holder entry).  Uniform routing: a
// uniformly random worker, the item's next move (payload: the holder entry there, or the
// item with kPassBit).
__global__ void k_seed_first(TrainArgs a, int64_t n, uint32_t *key, uint32_t *val, uint32_t *first) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += stride) {
        val[j] = (uint32_t)j;
        int4 st = *(const int4 *)(a.istate + 4 * j);
        const int64_t hb = a.hoff[j], nh = a.hoff[j + 1] - hb;
        if (nh <= 0) {
            key[j] = (uint32_t)a.p;
            first[j] = 0;
            continue;
        }
        if (a.sched == 2) {
            const int dest = route_uniform(a.route_seed, (int)j, st.x, a.p);
            const int g = a.hmap[(int64_t)dest * n + j];
            key[j] = (uint32_t)dest;
            first[j] = g >= 0 ? (uint32_t)g : (kPassBit | (uint32_t)j);
            st.x += 1;
        } else {
            const int64_t g = hb + visit_rank(a.route_seed, (int)j, a.epoch0, (uint32_t)nh, 0u);
            key[j] = (uint32_t)a.hold[g];
            first[j] = (uint32_t)g;
            st.x = a.epoch0;
            st.y = 1;   // position 0 of the visiting order is this first visit
            st.w = -1;
        }
        *(int4 *)(a.istate + 4 * j) = st;
    }
}

__global__ void k_seed_write(TrainArgs a, int64_t n, const uint32_t *key_s, const uint32_t *val_s,
                             const uint32_t *first) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t q = key_s[i];
        if (q >= (uint32_t)a.p) continue;
        int64_t lo = 0, hi = i;  // first position of worker q in the sorted keys
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (key_s[mid] < q) lo = mid + 1; else hi = mid;
        }
        const uint32_t pos = (uint32_t)(i - lo);
        const int64_t qb = a.sched == 2 ? (int64_t)q * a.n : a.vbase[q];
        a.queue[qb + pos] = ((uint64_t)(pos + 1u) << 32) | first[val_s[i]];
        atomicAdd(a.qtail + q, 1u);
    }
}

// One worker: workgroup q of the problem described by `a` (RND: the bfloat16 rounding rule,
// fixed at compile time so that the update loop has no branch on it).
template <int VEC, int D, bool BF, int LOSS, int RND>
__device__ __forceinline__ void worker_body(const TrainArgs &a, int q) {
    extern __shared__ float4 lds4[];
    // The wave index is the same in every lane: say so, so that everything derived from it
    // lives in scalar registers.
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const Lds L = lds_layout(lds4, a.kp, a.nw, a.slots, D, BF ? 2 : 4);
    if (threadIdx.x < kMaxWaves + 1) L.flag[threadIdx.x] = 0;
    if (threadIdx.x < 2) L.ctl[threadIdx.x] = 0;
    __syncthreads();
    if (q >= a.p || a.epochs <= 0) return;
    if (wave < a.nw) {
        const int64_t i0 = a.rbase[(int64_t)q * a.nw + wave], i1 = a.rbase[(int64_t)q * a.nw + wave + 1];
        ComputeWave<VEC, D, BF, LOSS, RND> cw(a, L, q, wave, lane, i0, i1 - i0);
        cw.run();
    } else if (wave == a.nw) {
        MemoryWave mw(a, L, q, lane);
        mw.run();
    }
}

template <int VEC, int D, bool BF, int LOSS, int RND>
__global__ __launch_bounds__(1024) void k_worker(TrainArgs a) {
    worker_body<VEC, D, BF, LOSS, RND>(a, blockIdx.x);
}

// Several independent problems in one launch: workgroup g runs worker g - wg0 of problem
// wg_prob[g]; every problem has its own layout, factors and item counters.  Built for five
// waves per SIMD (at most 96 registers a lane), so that two workers of eight compute waves
// and a memory wave each (18 waves) share a CU: a batch gains more from workers than from
// registers.
template <int VEC, int D, bool BF, int RND>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5))) void k_worker_batch(const TrainArgs *__restrict__ descs,
                                                       const int32_t *__restrict__ wg_prob) {
    const TrainArgs a = descs[wg_prob[blockIdx.x]];
    worker_body<VEC, D, BF, 0, RND>(a, (int)blockIdx.x - a.wg0);  // batches use the square loss
}

// A batched launch when `descs` is given (a.p then = total workgroups; square loss only),
// else one problem.
template <int VEC, int D, bool BF, int LOSS, int RND>
hipError_t launch_r(const TrainArgs &a, const TrainArgs *descs, const int32_t *wg_prob, hipStream_t st) {
    const size_t lds = lds_bytes(a.kp, a.nw, a.slots, D, BF ? 2 : 4);
    if constexpr (LOSS == 0) {
        if (descs) {
            hipLaunchKernelGGL((k_worker_batch<VEC, D, BF, RND>), dim3(a.p), dim3(64 * (a.nw + 1)), lds, st, descs,
                               wg_prob);
            return hipGetLastError();
        }
    } else {
        if (descs) return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((k_worker<VEC, D, BF, LOSS, RND>), dim3(a.p), dim3(64 * (a.nw + 1)), lds, st, a);
    return hipGetLastError();
}
template <int VEC, int D, bool BF, int LOSS>
hipError_t launch_t(const TrainArgs &a, const TrainArgs *descs, const int32_t *wg_prob, hipStream_t st) {
    if (BF && a.rounding == 1) return launch_r<VEC, D, BF, LOSS, 1>(a, descs, wg_prob, st);
    return launch_r<VEC, D, BF, LOSS, 0>(a, descs, wg_prob, st);
}

template <int VEC, bool BF, int LOSS>
const void *pick_d(int window) {
    if (window <= 8) return (const void *)k_worker<VEC, 8, BF, LOSS, 0>;
    if (window <= 16) return (const void *)k_worker<VEC, 16, BF, LOSS, 0>;
    return (const void *)k_worker<VEC, 32, BF, LOSS, 0>;
}

template <bool BF, int LOSS>
const void *pick_kernel(int kp, int window) {
    if (kp <= 64) return pick_d<1, BF, LOSS>(window);
    if (kp <= 128) return pick_d<2, BF, LOSS>(window);
    return pick_d<4, BF, LOSS>(window);
}

template <int VEC, bool BF>
const void *pick_batch_d(int window) {
    if (window <= 8) return (const void *)k_worker_batch<VEC, 8, BF, 0>;
    if (window <= 16) return (const void *)k_worker_batch<VEC, 16, BF, 0>;
    return (const void *)k_worker_batch<VEC, 32, BF, 0>;
}

template <bool BF>
const void *pick_batch(int kp, int window) {
    if (kp <= 64) return pick_batch_d<1, BF>(window);
    if (kp <= 128) return pick_batch_d<2, BF>(window);
    return pick_batch_d<4, BF>(window);
}

template <int VEC, bool BF, int LOSS>
hipError_t launch_v(const TrainArgs &a, const TrainArgs *d, const int32_t *g, hipStream_t st) {
    if (a.window <= 8) return launch_t<VEC, 8, BF, LOSS>(a, d, g, st);
    if (a.window <= 16) return launch_t<VEC, 16, BF, LOSS>(a, d, g, st);
    return launch_t<VEC, 32, BF, LOSS>(a, d, g, st);
}

template <bool BF, int LOSS>
hipError_t launch_b(const TrainArgs &a, const TrainArgs *d, const int32_t *g, hipStream_t st) {
    if (a.kp <= 64) return launch_v<1, BF, LOSS>(a, d, g, st);
    if (a.kp <= 128) return launch_v<2, BF, LOSS>(a, d, g, st);
    return launch_v<4, BF, LOSS>(a, d, g, st);
}

}  // namespace

namespace {
template <bool BF, int LOSS>
const void *pick_async(int kp) {
    if (kp <= 64) return (const void *)k_worker_async<1, kAsyncWindow, BF, LOSS, false, 0>;
    if (kp <= 128) return (const void *)k_worker_async<2, kAsyncWindow, BF, LOSS, false, 0>;
    return (const void *)k_worker_async<4, kAsyncWindow, BF, LOSS, false, 0>;
}
}  // namespace

size_t train_lds_bytes(int32_t kp, int32_t nw, int32_t slots, int32_t window, int32_t wbytes) {
    return lds_bytes(kp, nw, slots, window, wbytes);
}

hipError_t train_max_workers(int32_t kp, int32_t nw, int32_t slots, int32_t window, int32_t wbytes,
                             int32_t *max_workers, bool async, int32_t loss, bool batch) {
    int dev = 0, cus = 0, nb = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (async) window = kAsyncWindow;
    const void *kern =
        batch ? (wbytes == 2 ? pick_batch<true>(kp, window) : pick_batch<false>(kp, window)) :
        loss == 1 ? (async ? (wbytes == 2 ? pick_async<true, 1>(kp) : pick_async<false, 1>(kp))
                           : (wbytes == 2 ? pick_kernel<true, 1>(kp, window) : pick_kernel<false, 1>(kp, window)))
                  : (async ? (wbytes == 2 ? pick_async<true, 0>(kp) : pick_async<false, 0>(kp))
                           : (wbytes == 2 ? pick_kernel<true, 0>(kp, window) : pick_kernel<false, 0>(kp, window)));
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, 64 * (nw + 1), lds_bytes(kp, nw, slots, window, wbytes));
    if (e != hipSuccess) return e;
    *max_workers = nb * cus;
    return hipSuccess;
}

hipError_t launch_train(const TrainArgs &a, hipStream_t st) {
    if (a.loss == 1)
        return a.wbytes == 2 ? launch_b<true, 1>(a, nullptr, nullptr, st) : launch_b<false, 1>(a, nullptr, nullptr, st);
    return a.wbytes == 2 ? launch_b<true, 0>(a, nullptr, nullptr, st) : launch_b<false, 0>(a, nullptr, nullptr, st);
}

namespace {
template <int VEC, int D, bool BF, int LOSS>
hipError_t launch_async_t(const TrainArgs &a, hipStream_t st) {
    const size_t lds = lds_bytes(a.kp, a.nw, a.slots, D, BF ? 2 : 4);
    if (a.nw < 1 || a.nw > kMaxWavesAsync) return hipErrorInvalidValue;  // the kernel's launch bound
    // variants: with the kept-row path or not; bfloat16 storage per rounding rule
    const dim3 g(a.p), b(64 * (a.nw + 1));
    if (BF && a.rounding == 1) {
        if (a.keep_rows) hipLaunchKernelGGL((k_worker_async<VEC, D, BF, LOSS, true, 1>), g, b, lds, st, a);
        else hipLaunchKernelGGL((k_worker_async<VEC, D, BF, LOSS, false, 1>), g, b, lds, st, a);
    } else {
        if (a.keep_rows) hipLaunchKernelGGL((k_worker_async<VEC, D, BF, LOSS, true, 0>), g, b, lds, st, a);
        else hipLaunchKernelGGL((k_worker_async<VEC, D, BF, LOSS, false, 0>), g, b, lds, st, a);
    }
    return hipGetLastError();
}
template <int VEC, bool BF, int LOSS>
hipError_t launch_async_v(const TrainArgs &a, hipStream_t st) {
    return launch_async_t<VEC, kAsyncWindow, BF, LOSS>(a, st);  // the row window of the LDS layout is not used here
}
template <bool BF, int LOSS>
hipError_t launch_async_k(const TrainArgs &a, hipStream_t st) {
    if (a.kp <= 64) return launch_async_v<1, BF, LOSS>(a, st);
    if (a.kp <= 128) return launch_async_v<2, BF, LOSS>(a, st);
    return launch_async_v<4, BF, LOSS>(a, st);
}
hipError_t launch_async_b(const TrainArgs &a, hipStream_t st) {
    if (a.loss == 1) return a.wbytes == 2 ? launch_async_k<true, 1>(a, st) : launch_async_k<false, 1>(a, st);
    return a.wbytes == 2 ? launch_async_k<true, 0>(a, st) : launch_async_k<false, 0>(a, st);
}
}  // namespace

size_t async_scratch_bytes(int64_t n, int32_t p) {
    size_t sort_bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (uint32_t *)nullptr, (uint32_t *)nullptr,
                                             (uint32_t *)nullptr, (uint32_t *)nullptr, (int)(n > 0 ? n : 1), 0, 32);
    (void)p;
    return (size_t)(5 * (n > 0 ? n : 1)) * 4 + sort_bytes + 256;
}

hipError_t seed_train_async(const TrainArgs &a, void *scratch, size_t scratch_bytes, hipStream_t st) {
    const int64_t n = a.n;
    if (scratch_bytes < async_scratch_bytes(n, a.p)) return hipErrorInvalidValue;
    uint32_t *key = (uint32_t *)scratch, *val = key + n, *key_s = val + n, *val_s = key_s + n;
    uint32_t *first = val_s + n;
    void *tmp = (void *)(((uintptr_t)(first + n) + 255) & ~(uintptr_t)255);
    size_t tmp_bytes = scratch_bytes - ((char *)tmp - (char *)scratch);
    hipError_t e;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_seed_first, dim3(grid > 0 ? grid : 1), dim3(256), 0, st, a, n, key, val, first);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key, key_s, val, val_s, (int)n, 0, 32, st)) !=
        hipSuccess)
        return e;
    hipLaunchKernelGGL(k_seed_write, dim3(grid > 0 ? grid : 1), dim3(256), 0, st, a, n, key_s, val_s, first);
    return hipGetLastError();
}

hipError_t launch_train_async(const TrainArgs &a, hipStream_t st) { return launch_async_b(a, st); }

namespace {
// Per-launch resets of a batch's problems: block b clears problem b's abort word, its
// eight diagnostic words and its workers' statistics.
__global__ void k_batch_reset(const TrainArgs *descs, int nprob) {
    const int b = blockIdx.x;
    if (b >= nprob) return;
    const TrainArgs a = descs[b];
    if (threadIdx.x == 0) *a.abort_flag = 0u;
    if (threadIdx.x < 8) a.diag[threadIdx.x] = 0;
    if (threadIdx.x < 2) a.counters[threadIdx.x] = 0ull;
    const int64_t nst = (int64_t)kWStatCount * a.p;
    for (int64_t i = threadIdx.x; i < nst; i += blockDim.x) a.wstats[i] = 0;
}

__global__ void k_batch_epochs(TrainArgs *descs, int nprob, int32_t epochs, int32_t advance) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nprob) return;
    descs[b].epoch0 += advance;
    descs[b].epochs = epochs;
}
}  // namespace

hipError_t launch_batch_reset(const TrainArgs *d_descs, int32_t nprob, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_reset, dim3(nprob), dim3(64), 0, st, d_descs, (int)nprob);
    return hipGetLastError();
}

hipError_t launch_batch_epochs(TrainArgs *d_descs, int32_t nprob, int32_t epochs, int32_t advance, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_epochs, dim3((nprob + 63) / 64), dim3(64), 0, st, d_descs, (int)nprob, epochs, advance);
    return hipGetLastError();
}

hipError_t launch_train_batch(const TrainArgs &shape, int32_t workgroups, const TrainArgs *d_descs,
                              const int32_t *d_wg_prob, hipStream_t st) {
    TrainArgs a = shape;
    a.p = workgroups;
    return a.wbytes == 2 ? launch_b<true, 0>(a, d_descs, d_wg_prob, st) : launch_b<false, 0>(a, d_descs, d_wg_prob, st);
}

}  // namespace nomad
