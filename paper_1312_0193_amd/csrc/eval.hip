// Test RMSE (section 5.1) and objective J(W,H) (eq. obj_fcn, per-rating form, with the
// context's per-rating loss) with FP64 dot products and compensated (Neumaier) sums.  The entry-to-thread assignment and the
// reduction tree are fixed, so the result does not depend on timing.
#include "nomad_internal.h"

namespace nomad {
namespace {

constexpr int kBlocks = 1024;
constexpr int kThreads = 256;

struct Comp {
    double s, c;
};

__device__ __forceinline__ void neu_add(Comp &a, double x) {
    double t = a.s + x;
    if (fabs(a.s) >= fabs(x)) a.c += (a.s - t) + x;
    else a.c += (x - t) + a.s;
    a.s = t;
}

__device__ __forceinline__ Comp neu_merge(Comp a, Comp b) {
    neu_add(a, b.s);
    a.c += b.c;
    return a;
}

// Element l of row i of W stored as FP32 (wbytes 4) or bfloat16 (wbytes 2).
__device__ __forceinline__ double w_at(const void *W, int32_t wbytes, int64_t x) {
    if (wbytes == 2) return (double)__uint_as_float((uint32_t)((const uint16_t *)W)[x] << 16);
    return (double)((const float *)W)[x];
}

__global__ __launch_bounds__(kThreads) void k_eval_partial(const void *W, int32_t wbytes, const float *H, int32_t k,
                                                          int32_t kp, int64_t m, int64_t n, int64_t nnz,
                                                          const int32_t *row, const int32_t *col,
                                                          const float *val, double lambda, int32_t loss,
                                                          Comp *part, int32_t *bad) {
    __shared__ Comp sq[kThreads], ob[kThreads];
    Comp a{0.0, 0.0}, b{0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += stride) {
        const int32_t i = row[e], j = col[e];
        if (i < 0 || i >= m || j < 0 || j >= n) {
            atomicOr(bad, 1);
            continue;
        }
        const int64_t wi = (int64_t)i * kp;
        const float *h = H + (int64_t)j * kp;
        double d = 0.0, ww = 0.0, hh = 0.0;
        for (int32_t l = 0; l < k; ++l) {
            const double wl = w_at(W, wbytes, wi + l), hl = (double)h[l];
            d += wl * hl;
            ww += wl * wl;
            hh += hl * hl;
        }
        const double err = (double)val[e] - d;
        neu_add(a, err * err);
        if (loss == 1) {
            // logistic loss log(1 + exp(z)), z = -r d, as max(z, 0) + log1p(exp(-|z|))
            const double z = -(double)val[e] * d;
            neu_add(b, (z > 0.0 ? z : 0.0) + log1p(exp(-fabs(z))) + 0.5 * lambda * (ww + hh));
        } else {
            neu_add(b, 0.5 * (err * err + lambda * (ww + hh)));
        }
    }
    sq[threadIdx.x] = a;
    ob[threadIdx.x] = b;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sq[threadIdx.x] = neu_merge(sq[threadIdx.x], sq[threadIdx.x + w]);
            ob[threadIdx.x] = neu_merge(ob[threadIdx.x], ob[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sq[0];
        part[2 * blockIdx.x + 1] = ob[0];
    }
}

__global__ __launch_bounds__(kThreads) void k_eval_final(const Comp *part, int nparts, double *out) {
    __shared__ Comp sq[kThreads], ob[kThreads];
    Comp a{0.0, 0.0}, b{0.0, 0.0};
    for (int x = threadIdx.x; x < nparts; x += blockDim.x) {
        a = neu_merge(a, part[2 * x]);
        b = neu_merge(b, part[2 * x + 1]);
    }
    sq[threadIdx.x] = a;
    ob[threadIdx.x] = b;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sq[threadIdx.x] = neu_merge(sq[threadIdx.x], sq[threadIdx.x + w]);
            ob[threadIdx.x] = neu_merge(ob[threadIdx.x], ob[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sq[0].s + sq[0].c;
        out[1] = ob[0].s + ob[0].c;
    }
}

// The results of a reduction for a caller's device buffer: RMSE, J and the bad-index flag
// (1.0 if an entry's index was out of range, else 0.0).
__global__ void k_eval_out(const double *sums, const int32_t *bad, int64_t nnz, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    out[0] = nnz > 0 ? sqrt(sums[0] / (double)nnz) : NAN;
    out[1] = nnz > 0 ? sums[1] : 0.0;
    out[2] = *bad ? 1.0 : 0.0;
}

__global__ void k_clear_word(int32_t *w) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *w = 0;
}

// Scratch of the allocation-free evaluation (nomad_eval_rmse_noalloc): one Neumaier pair
// per block of the partial pass and per sum, the two final sums and the bad-index word.
// Each device that runs the library holds its own copy until the process ends; its
// address comes from hipGetSymbolAddress (the name itself is a host-side stand-in).
constexpr int kNoallocMaxBlocks = 16384;
constexpr int64_t kNoallocEntriesPerBlock = 8192;
constexpr size_t kNoallocScratchBytes = sizeof(Comp) * 2 * kNoallocMaxBlocks + 2 * sizeof(double) + 64;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

// FP32 rows of width k -> bfloat16 rows of width kp (nearest-even; the pad is left alone).
__global__ void k_to_bf16(const float *src, int32_t k, uint16_t *dst, int32_t kp, int64_t rows) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < rows * k; x += stride) {
        const int64_t i = x / k, l = x - i * k;
        const uint32_t u = __float_as_uint(src[x]);
        dst[i * kp + l] = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
    }
}

// bfloat16 rows of width kp -> FP32 rows of width k (exact).
__global__ void k_from_bf16(const uint16_t *src, int32_t kp, float *dst, int32_t k, int64_t rows) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < rows * k; x += stride) {
        const int64_t i = x / k, l = x - i * k;
        dst[x] = __uint_as_float((uint32_t)src[i * kp + l] << 16);
    }
}

}  // namespace

hipError_t to_bf16(const float *src, int32_t k, uint16_t *dst, int32_t kp, int64_t rows, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_bf16, dim3(2048), dim3(256), 0, st, src, k, dst, kp, rows);
    return hipGetLastError();
}

hipError_t from_bf16(const uint16_t *src, int32_t kp, float *dst, int32_t k, int64_t rows, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_from_bf16, dim3(2048), dim3(256), 0, st, src, kp, dst, k, rows);
    return hipGetLastError();
}

size_t eval_scratch_bytes() { return sizeof(Comp) * 2 * kBlocks + 2 * sizeof(double) + 64; }

int64_t noalloc_max_nnz() { return (int64_t)kNoallocMaxBlocks * kNoallocEntriesPerBlock; }
size_t noalloc_scratch_bytes() { return kNoallocScratchBytes; }

hipError_t noalloc_scratch_address(void **ptr) {
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

hipError_t eval_sums_noalloc(const void *W, int32_t wbytes, const float *H, int32_t k, int32_t kp, int64_t m,
                             int64_t n, int64_t nnz, const int32_t *row, const int32_t *col, const float *val,
                             double lambda, int32_t loss, void *scratch_ptr, double *d_out, hipStream_t st) {
    // one block of the partial pass per kNoallocEntriesPerBlock entries (the caller has
    // checked nnz <= noalloc_max_nnz())
    const int64_t want = (nnz + kNoallocEntriesPerBlock - 1) / kNoallocEntriesPerBlock;
    const int blocks = (int)(want < 1 ? 1 : want);
    Comp *part = (Comp *)scratch_ptr;
    double *sums = (double *)(part + 2 * kNoallocMaxBlocks);
    int32_t *bad = (int32_t *)(sums + 2);
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(64), 0, st, bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_eval_partial, dim3(blocks), dim3(kThreads), 0, st, W, wbytes, H, k, kp, m, n, nnz, row,
                       col, val, lambda, loss, part, bad);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_eval_final, dim3(1), dim3(kThreads), 0, st, part, blocks, sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_eval_out, dim3(1), dim3(64), 0, st, sums, bad, nnz, d_out);
    return hipGetLastError();
}

hipError_t eval_sums(const void *W, int32_t wbytes, const float *H, int32_t k, int32_t kp, int64_t m, int64_t n,
                     int64_t nnz, const int32_t *row, const int32_t *col, const float *val,
                     double lambda, int32_t loss, double *h_sq_err, double *h_obj, int *h_bad_index, void *scratch,
                     size_t scratch_bytes, hipStream_t st) {
    if (scratch_bytes < eval_scratch_bytes()) return hipErrorInvalidValue;
    Comp *part = (Comp *)scratch;
    double *out = (double *)(part + 2 * kBlocks);
    int32_t *bad = (int32_t *)(out + 2);
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(int32_t), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_eval_partial, dim3(kBlocks), dim3(kThreads), 0, st, W, wbytes, H, k, kp, m, n, nnz, row,
                       col, val, lambda, loss, part, bad);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_eval_final, dim3(1), dim3(kThreads), 0, st, part, kBlocks, out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double h_out[2];
    int32_t h_bad = 0;
    if ((e = hipMemcpyAsync(h_out, out, sizeof(h_out), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&h_bad, bad, sizeof(h_bad), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    *h_sq_err = h_out[0];
    *h_obj = h_out[1];
    *h_bad_index = h_bad;
    return hipSuccess;
}

}  // namespace nomad
