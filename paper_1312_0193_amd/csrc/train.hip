// NOMAD worker kernel: one wavefront = one worker (Algorithm 1), persistent for a whole
// nomad_train_epochs call.
//
// Worker q walks its chunks in plan order, epoch after epoch.  At the first chunk of a
// block (q, g) it waits until group g has completed every earlier visit of the epoch
// (its ticket), which makes worker q the sole owner of the group's item vectors h_j
// (owner-computes rule, section 3.1).  It stages the chunk's rows w_i and items h_j in
// LDS, runs the SGD updates of section 2.3 over the chunk's ratings in plan order,
// writes back what the next chunk does not carry, and after the last chunk of the block
// publishes the items and passes the group on by advancing its ticket.
//
// Memory ordering of a hand-off: item vectors are written with device-coherent
// stores (agent scope, sc1) and the ticket is advanced with a device-coherent store
// only after "s_waitcnt vmcnt(0)" has seen those stores complete; the next owner polls
// the ticket with device-coherent loads and then reads the items with device-coherent
// loads.  Rows w_i are private to their worker (always the same wavefront, hence the
// same CU and XCD) and use ordinary cached loads and stores.
#include <cmath>

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

// Device-coherent (agent scope) item loads/stores.
template <int VEC>
__device__ __forceinline__ void coherent_load(const float *p, float (&v)[VEC]) {
    if constexpr (VEC == 1) {
        uint32_t t = __hip_atomic_load((uint32_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v[0] = __builtin_bit_cast(float, t);
    } else {
#pragma unroll
        for (int h = 0; h < VEC / 2; ++h) {
            uint64_t t = __hip_atomic_load((uint64_t *)p + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            v[2 * h] = __builtin_bit_cast(float, (uint32_t)t);
            v[2 * h + 1] = __builtin_bit_cast(float, (uint32_t)(t >> 32));
        }
    }
}
template <int VEC>
__device__ __forceinline__ void coherent_store(float *p, const float (&v)[VEC]) {
    if constexpr (VEC == 1) {
        __hip_atomic_store((uint32_t *)p, __builtin_bit_cast(uint32_t, v[0]), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
#pragma unroll
        for (int h = 0; h < VEC / 2; ++h) {
            uint64_t t = (uint64_t)__builtin_bit_cast(uint32_t, v[2 * h]) |
                         ((uint64_t)__builtin_bit_cast(uint32_t, v[2 * h + 1]) << 32);
            __hip_atomic_store((uint64_t *)p + h, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int VEC>
__device__ __forceinline__ void global_read(const float *p, float (&v)[VEC]) { lds_read<VEC>(p, v); }
template <int VEC>
__device__ __forceinline__ void global_write(float *p, const float (&v)[VEC]) { lds_write<VEC>(p, v); }

__device__ __forceinline__ void wait_vm_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Seconds-scale bound on any single wait, so that a broken schedule ends the kernel
// instead of hanging the device (100 MHz constant clock).
constexpr uint64_t kWaitLimitTicks = 20ull * 100000000ull;

template <int VEC, int NR16>
__global__ __launch_bounds__(64) void k_train(TrainArgs a, uint32_t *abort_flag) {
    extern __shared__ float4 lds4[];
    float *lds = reinterpret_cast<float *>(lds4);
    const int q = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t c0 = a.wck[q], c1 = a.wck[q + 1];
    const int64_t nck = c1 - c0;
    if (nck <= 0 || a.epochs <= 0) return;
    const int kp = a.kp;
    const int nslot = a.rmax + a.tmax;
    const bool on = lane * VEC < kp;
    const int off = lane * VEC;
    const int64_t total = nck * (int64_t)a.epochs;

    for (int64_t it = 0; it < total; ++it) {
        const int64_t e = it / nck;
        const int64_t c = c0 + (it - e * nck);
        const ChunkRec ck = a.chunks[c];
        const uint32_t info = ck.info;
        const int nrat = info & 255, nr = (info >> 8) & 255, nt = (info >> 16) & 255;
        const uint32_t flags = info >> 24;
        float *cur = lds + (size_t)(it & 1) * nslot * kp;
        float *prv = lds + (size_t)((it & 1) ^ 1) * nslot * kp;
        const bool first_it = it == 0, last_it = it == total - 1;
        const int64_t ep = a.epoch0 + e;
        const float s = (float)(a.alpha / (1.0 + a.beta * pow((double)ep, a.gamma)));
        const float shrink = 1.0f - s * a.lambda;
        const uint32_t ticket = (uint32_t)(ep * (int64_t)ck.nblk + ck.vblk);

        SlotRec sr{0, -1, 0};
        if (lane < nr + nt) sr = a.slots[ck.slot + lane];
        const int s_id = sr.id, s_src = sr.src, s_keep = sr.keep;
        RatingRec rr{0, 0.0f};
        if (lane < nrat) rr = a.ratings[ck.rat + lane];
        {
            // Plan validation: a malformed plan ends the kernel instead of touching
            // memory outside the factors or the LDS staging area.
            const bool is_row = lane < nr;
            const int cap = is_row ? a.rmax : a.tmax;
            const int64_t lim = is_row ? a.m : a.n;
            bool bad = nr > a.rmax || nt > a.tmax || nrat > kMaxRatingsPerChunk;
            if (lane < nr + nt) bad |= s_id < 0 || s_id >= lim || s_src >= cap;
            if (lane < nrat) bad |= (int)(rr.slots & 255) >= nr || (int)(rr.slots >> 8) >= nt;
            if (__builtin_amdgcn_ballot_w64(bad) != 0) {
                if (lane == 0)
                    __hip_atomic_store(abort_flag, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
        }

        if (flags & kFirstOfBlock) {
            uint32_t *gd = a.grp_done + ck.group;
            if (__hip_atomic_load(gd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ticket) {
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(gd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ticket) {
                    __builtin_amdgcn_s_sleep(2);
                    if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
                    if (wall_clock64() - t0 > kWaitLimitTicks) {
                        __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        return;
                    }
                }
            }
            if (a.trace && lane == 0) {
                int64_t slot = atomicAdd((unsigned long long *)a.trace_len, 1ull);
                if (slot < a.trace_cap) {
                    a.trace[4 * slot + 0] = q;
                    a.trace[4 * slot + 1] = ck.group;
                    a.trace[4 * slot + 2] = (int32_t)ep;
                    a.trace[4 * slot + 3] = (int32_t)ticket;
                }
            }
        }

        // Stage rows.
        for (int x = 0; x < nr; ++x) {
            const int id = rl_i(s_id, x), src = rl_i(s_src, x);
            float v[VEC] = {};
            if (on) {
                if (!first_it && src >= 0) lds_read<VEC>(prv + src * kp + off, v);
                else global_read<VEC>(a.W + (int64_t)id * kp + off, v);
                lds_write<VEC>(cur + x * kp + off, v);
            }
        }
        // Stage items (owned by this worker until the group is passed on).
        for (int x = 0; x < nt; ++x) {
            const int id = rl_i(s_id, nr + x), src = rl_i(s_src, nr + x);
            float v[VEC] = {};
            if (on) {
                if (src >= 0) lds_read<VEC>(prv + (a.rmax + src) * kp + off, v);
                else coherent_load<VEC>(a.H + (int64_t)id * kp + off, v);
                lds_write<VEC>(cur + (a.rmax + x) * kp + off, v);
            }
        }

        // SGD over the chunk's ratings, in plan order.
        const int r_sl = (int)rr.slots;
        const float r_val = rr.r;
        int cur_ts = -1;
        float h[VEC] = {};
        for (int x = 0; x < nrat; ++x) {
            const int sl = rl_i(r_sl, x);
            const float r = rl_f(r_val, x);
            const int rs = sl & 255, ts = sl >> 8;
            if (ts != cur_ts) {
                if (cur_ts >= 0 && on) lds_write<VEC>(cur + (a.rmax + cur_ts) * kp + off, h);
                if (on) lds_read<VEC>(cur + (a.rmax + ts) * kp + off, h);
                cur_ts = ts;
            }
            float w[VEC] = {};
            if (on) lds_read<VEC>(cur + rs * kp + off, w);
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
            if (on) lds_write<VEC>(cur + rs * kp + off, w);
        }
        if (cur_ts >= 0 && on) lds_write<VEC>(cur + (a.rmax + cur_ts) * kp + off, h);

        // Write back what the next chunk does not carry.
        for (int x = 0; x < nr; ++x) {
            const int id = rl_i(s_id, x), keep = rl_i(s_keep, x);
            if ((last_it || !keep) && on) {
                float v[VEC];
                lds_read<VEC>(cur + x * kp + off, v);
                global_write<VEC>(a.W + (int64_t)id * kp + off, v);
            }
        }
        for (int x = 0; x < nt; ++x) {
            const int id = rl_i(s_id, nr + x), keep = rl_i(s_keep, nr + x);
            if ((last_it || !keep) && on) {
                float v[VEC];
                lds_read<VEC>(cur + (a.rmax + x) * kp + off, v);
                coherent_store<VEC>(a.H + (int64_t)id * kp + off, v);
            }
        }
        if (flags & kLastOfBlock) {
            wait_vm_all();
            if (lane == 0)
                __hip_atomic_store(a.grp_done + ck.group, ticket + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
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
    return (size_t)2 * (size_t)(rmax + tmax) * (size_t)kp * sizeof(float);
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

// The abort flag lives in a small device buffer owned by the caller (TrainArgs::trace
// pointers are optional); it is passed through `a.trace_len`'s neighbour in the API.
hipError_t launch_train(const TrainArgs &a, int32_t p, hipStream_t st) {
    const size_t lds = train_lds_bytes(a.kp, a.rmax, a.tmax);
    uint32_t *abort_flag = a.grp_done + p;  // one extra word after the tickets
    if (a.kp <= 16) return launch_t<1, 1>(a, p, lds, abort_flag, st);
    if (a.kp <= 32) return launch_t<1, 2>(a, p, lds, abort_flag, st);
    if (a.kp <= 64) return launch_t<1, 4>(a, p, lds, abort_flag, st);
    if (a.kp <= 128) return launch_t<2, 4>(a, p, lds, abort_flag, st);
    return launch_t<4, 4>(a, p, lds, abort_flag, st);
}

}  // namespace nomad
