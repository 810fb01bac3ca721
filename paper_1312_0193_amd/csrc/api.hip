// C ABI of libnomad.so (declared in include/nomad.h).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <utility>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "nomad.h"
#include "nomad_internal.h"

using nomad::Plan;

struct nomad_ctx {
    nomad_config cfg{};
    int64_t m = 0, n = 0, nnz = 0;
    int32_t k = 0, kp = 0, p = 0;
    int32_t nw = 0, slots = 0;         // compute waves and item slots per worker
    int32_t window = 0;                // rows a compute wave keeps in flight
    int32_t keep_rows = 0;             // asynchronous schedules: some compute wave owns a single row
    int32_t cus = 0, max_lds = 0;
    hipStream_t stream = nullptr;
    int device = 0;                    // the device current at nomad_init
    Plan plan;
    void *W = nullptr;                 // m x kp, FP32 or bfloat16 (row stride kp, padding kept at 0)
    float *H = nullptr;                // n x kp FP32
    int32_t wbytes = 4;                // bytes per stored element of W
    uint32_t *tok_done = nullptr;      // n item counters + 1 abort word
    float *dummy = nullptr;            // target of the workers' placeholder stores
    int32_t *diag = nullptr;           // 8 words describing a wait that ran out of time
    int64_t epochs_done = 0;
    std::vector<int64_t> row_start;
    int64_t *wstats = nullptr;         // p x kWStatCount per-worker counters of the last call
    int32_t *trace = nullptr;
    int64_t *trace_len = nullptr;
    int64_t trace_cap = 0;
    int64_t trace_count = 0;
    void *eval_scratch = nullptr;
    size_t eval_scratch_bytes = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<hipEvent_t> lev;       // around each training launch of a call (pairs)
    double layout_seconds = 0.0;
    std::string err;
    // Asynchronous schedule: inbound queues, item state, seeding scratch.
    uint64_t *queue = nullptr;
    uint32_t *qtail = nullptr, *qhead = nullptr, *parked = nullptr;
    int32_t *istate = nullptr, *tvis = nullptr;   // per item state words (n x 4), per holder visits
    unsigned long long *upd = nullptr;
    int64_t queue_len = 0;
    void *async_scratch = nullptr;
    size_t async_scratch_bytes = 0;
    // Ownership checks and counters: [0] violations, [1] hops (both per call), [2] global
    // update count (since nomad_init).
    uint32_t *holder = nullptr;
    unsigned long long *counters = nullptr;
    // A launch that ran out of time or found a malformed layout leaves the factors and the
    // items' state undefined: every later call that needs them is refused.
    bool failed = false;
    // A batch (nomad_init_batched): its problems, each a full context of its own, trained
    // together by one launch.
    std::vector<nomad_ctx *> members;
    nomad_ctx *owner = nullptr;        // set in a problem of a batch
    nomad::Shape shape{};
    nomad::TrainArgs *d_descs = nullptr;  // per problem: its launch arguments
    int32_t *d_wg = nullptr;           // per workgroup: its problem
    std::vector<int32_t> wg0;          // per problem: its first workgroup
    int32_t total_wg = 0;
    hipGraphExec_t graph = nullptr;    // a batch's captured launch sequence (nomad_batch_graph)
    int32_t graph_epochs = 0;          // the epochs it runs
};

namespace {

thread_local std::string g_last_error;

// Device address of the allocation-free evaluation's scratch array, per device: looked up
// once per device (with that device current) by the first nomad_init on it.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

void prepare_noalloc_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return;
    void *ptr = nullptr;
    const hipError_t e = nomad::noalloc_scratch_address(&ptr);
    g_scratch_err[dev] = e;
    if (e == hipSuccess) g_scratch_ptr[dev] = ptr;
}

nomad_status fail(nomad_ctx *ctx, nomad_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
nomad_status fail(nomad_ctx *ctx, nomad_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    if (ctx) ctx->err = buf;
    return st;
}

nomad_status hip_fail(nomad_ctx *ctx, hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory)
        return fail(ctx, NOMAD_ENOMEM, "%s: device allocation failed (%s)", what, hipGetErrorString(e));
    return fail(ctx, NOMAD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPTRY(ctx, expr, what)                             \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return hip_fail((ctx), _e, (what)); \
    } while (0)

void release(nomad_ctx *c) {
    if (!c) return;
    for (nomad_ctx *m : c->members) {
        release(m);
        delete m;
    }
    c->members.clear();
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
    (void)hipFree(c->d_descs);
    (void)hipFree(c->d_wg);
    (void)hipFree(c->queue);
    (void)hipFree(c->qtail);
    (void)hipFree(c->qhead);
    (void)hipFree(c->parked);
    (void)hipFree(c->istate);
    (void)hipFree(c->tvis);
    (void)hipFree(c->holder);
    (void)hipFree(c->counters);
    (void)hipFree(c->upd);
    (void)hipFree(c->async_scratch);
    nomad::free_plan(&c->plan);
    (void)hipFree(c->W);
    (void)hipFree(c->H);
    (void)hipFree(c->tok_done);
    (void)hipFree(c->dummy);
    (void)hipFree(c->diag);
    (void)hipFree(c->trace);
    (void)hipFree(c->trace_len);
    (void)hipFree(c->wstats);
    (void)hipFree(c->eval_scratch);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    for (hipEvent_t ev : c->lev) (void)hipEventDestroy(ev);
    c->lev.clear();
}

// Launch shape: compute waves, item slots and row window of a worker (LDS-fitted as the
// configuration asks), and how many workers can be resident at once.
nomad_status choose_shape(const nomad_config *cfg, int32_t kp, int32_t wbytes, nomad::Shape *out, nomad_ctx *ec,
                          bool batch = false) {
    // Workers, compute waves per worker and item slots.  By default one worker runs on
    // every CU with eight compute waves (four under the asynchronous schedules), and holds
    // up to 64 items (fewer if LDS is short).
    int dev = 0, max_lds = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(ec, NOMAD_EDEVICE, "nomad_init: no usable HIP device");
    const bool async = cfg->sched == NOMAD_SCHED_PERM || cfg->sched == NOMAD_SCHED_UNIFORM;
    const int32_t nw = cfg->waves_per_worker > 0 ? cfg->waves_per_worker
                                                 : (async ? nomad::kDefaultWavesAsync : nomad::kDefaultWaves);
    if (nw < 1 || nw > (async ? nomad::kMaxWavesAsync : nomad::kMaxWaves))
        return fail(ec, NOMAD_EINVAL, "nomad_init: waves_per_worker=%d outside [1,%d]%s", nw,
                    async ? nomad::kMaxWavesAsync : nomad::kMaxWaves, async ? " (asynchronous schedules)" : "");
    if (cfg->window < 0 || cfg->window > nomad::kMaxWindow)
        return fail(ec, NOMAD_EINVAL, "nomad_init: window=%d outside [0,%d]", cfg->window, nomad::kMaxWindow);
    // Item slots and the compute waves' row windows share the LDS: by default deep windows
    // come first, then item slots.
    int32_t slots = cfg->item_slots;
    int32_t window = cfg->window <= 0 ? nomad::kMaxWindow : (cfg->window <= 8 ? 8 : (cfg->window <= 16 ? 16 : 32));
    if (async) window = nomad::kAsyncWindow;  // the asynchronous kernel keeps its rows in registers
    const bool auto_window = cfg->window <= 0 && !async;
    auto fits = [&](int32_t s_, int32_t w_) {
        return nomad::train_lds_bytes(kp, nw, s_, w_, wbytes) <= (size_t)max_lds;
    };
    if (slots <= 0) {
        slots = nomad::kMaxItemSlots;
        while (!fits(slots, window)) {
            if (slots > 32) slots >>= 1;
            else if (auto_window && window > 16) window >>= 1;
            else if (slots > 16) slots >>= 1;
            else if (auto_window && window > 8) window >>= 1;
            else if (slots > 8) slots >>= 1;
            else break;
        }
    } else if (auto_window) {
        while (!fits(slots, window) && window > 8) window >>= 1;
    }
    if (slots < 1 || slots > nomad::kMaxItemSlots || (slots & (slots - 1)) != 0)
        return fail(ec, NOMAD_EINVAL, "nomad_init: item_slots=%d must be a power of two in [1,%d]", slots,
                    nomad::kMaxItemSlots);
    const size_t lds = nomad::train_lds_bytes(kp, nw, slots, window, wbytes);
    if (lds > (size_t)max_lds)
        return fail(ec, NOMAD_EINVAL, "nomad_init: %d compute waves, %d item slots and a window of %d rows need "
                    "%zu bytes of LDS for padded k=%d, device allows %d", nw, slots, window, lds, kp, max_lds);
    int32_t maxw = 0;
    hipError_t he = nomad::train_max_workers(kp, nw, slots, window, wbytes, &maxw, async, cfg->loss, batch);
    if (he != hipSuccess) return hip_fail(ec, he, "nomad_init: occupancy query");
    out->kp = kp;
    out->nw = nw;
    out->slots = slots;
    out->window = window;
    out->maxw = maxw;
    out->cus = cus;
    out->max_lds = max_lds;
    return NOMAD_OK;
}

}  // namespace

extern "C" {

void nomad_config_default(nomad_config *cfg) {
    if (!cfg) return;
    memset(cfg, 0, sizeof(*cfg));
    cfg->k = 0;
    cfg->lambda = 0.05f;
    cfg->alpha = 0.01f;
    cfg->beta = 0.0f;
    cfg->gamma = 1.5f;
    cfg->sched = NOMAD_SCHED_RING;
    cfg->dtype = NOMAD_FP32;
    cfg->rounding = NOMAD_ROUND_RNE;
    cfg->workers = 0;
    cfg->waves_per_worker = 0;
    cfg->item_slots = 0;
    cfg->window = 0;
    cfg->record_trace = 0;
    cfg->collect_stats = 0;
    cfg->debug_ownership = 0;
    cfg->t_source = 0;
    cfg->balance = 0;
    cfg->transpose = 0;
    cfg->loss = NOMAD_LOSS_SQUARE;
    cfg->seed = 0;
}

// nomad_init with an optional launch shape imposed (the problems of a batch share one).
static nomad_status init_impl(nomad_ctx **out, const nomad_config *cfg, int64_t m, int64_t n, int64_t nnz,
                              const int32_t *d_row, const int32_t *d_col, const float *d_val, const float *d_W0,
                              const float *d_H0, void *hip_stream, const nomad::Shape *forced) {
    if (!out) return fail(nullptr, NOMAD_EINVAL, "nomad_init: out is NULL");
    *out = nullptr;
    if (!cfg) return fail(nullptr, NOMAD_EINVAL, "nomad_init: cfg is NULL");
    if (cfg->k < 1 || cfg->k > nomad::kMaxK)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: k=%d outside [1,%d]", cfg->k, nomad::kMaxK);
    if (!(cfg->lambda >= 0.0f) || !std::isfinite(cfg->lambda))
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: lambda must be finite and >= 0");
    if (!std::isfinite(cfg->alpha) || !std::isfinite(cfg->beta) || !std::isfinite(cfg->gamma) ||
        cfg->alpha < 0.0f || cfg->beta < 0.0f || cfg->gamma < 0.0f)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: step-size parameters must be finite and >= 0");
    if (m < 1 || n < 1 || m > INT32_MAX || n > INT32_MAX)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: m=%lld, n=%lld must be in [1, 2^31)", (long long)m,
                    (long long)n);
    if (nnz < 0 || nnz > (int64_t)UINT32_MAX)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: nnz=%lld outside [0, 2^32)", (long long)nnz);
    if (nnz > 0 && (!d_row || !d_col || !d_val))
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: rating arrays are NULL");
    if (!d_W0 || !d_H0) return fail(nullptr, NOMAD_EINVAL, "nomad_init: initial factors are NULL");
    if (cfg->sched != NOMAD_SCHED_RING && cfg->sched != NOMAD_SCHED_PERM && cfg->sched != NOMAD_SCHED_UNIFORM)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: schedule %d is not one of NOMAD_SCHED_RING, NOMAD_SCHED_PERM, "
                    "NOMAD_SCHED_UNIFORM", cfg->sched);
    if (cfg->dtype != NOMAD_FP32 && cfg->dtype != NOMAD_BF16)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: storage type %d is not one of NOMAD_FP32, NOMAD_BF16",
                    cfg->dtype);
    if (cfg->rounding != NOMAD_ROUND_RNE && cfg->rounding != NOMAD_ROUND_STOCHASTIC)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: rounding %d is not one of NOMAD_ROUND_RNE, "
                    "NOMAD_ROUND_STOCHASTIC", cfg->rounding);
    if (cfg->debug_ownership != 0 && cfg->debug_ownership != 1)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: debug_ownership=%d is not 0 or 1", cfg->debug_ownership);
    if (cfg->t_source != 0 && cfg->t_source != 1)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: t_source=%d is not 0 or 1", cfg->t_source);
    if (cfg->balance != 0 && cfg->balance != 1)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: balance=%d is not 0 or 1", cfg->balance);
    if (cfg->transpose != 0 && cfg->transpose != 1)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: transpose=%d is not 0 or 1", cfg->transpose);
    if (cfg->transpose == 1 && forced)
        return fail(nullptr, NOMAD_ENOTIMPL, "nomad_init_batched: transpose=1 is per problem only");
    if (cfg->loss != NOMAD_LOSS_SQUARE && cfg->loss != NOMAD_LOSS_LOGISTIC)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init: loss=%d is not a nomad_loss", cfg->loss);
    if (cfg->loss != NOMAD_LOSS_SQUARE && forced)
        return fail(nullptr, NOMAD_ENOTIMPL, "nomad_init_batched: batches use the square loss");
    if (cfg->balance == 1 && cfg->sched == NOMAD_SCHED_RING)
        return fail(nullptr, NOMAD_ENOTIMPL, "nomad_init: balance=1 needs an asynchronous schedule (the ring order "
                    "is fixed)");
    if (cfg->t_source == 1 && forced)
        return fail(nullptr, NOMAD_ENOTIMPL, "nomad_init_batched: t_source=1 (global update count) is per problem only");

    nomad_ctx *c = new (std::nothrow) nomad_ctx();
    if (!c) return fail(nullptr, NOMAD_ENOMEM, "nomad_init: host allocation failed");
    c->cfg = *cfg;
    c->m = m;
    c->n = n;
    c->nnz = nnz;
    c->k = cfg->k;
    c->kp = forced ? forced->kp : nomad::padded_k(cfg->k);
    c->wbytes = cfg->dtype == NOMAD_BF16 ? 2 : 4;
    c->stream = (hipStream_t)hip_stream;

    auto bail = [&](nomad_status st) {
        g_last_error = c->err;
        release(c);
        delete c;
        return st;
    };

    nomad::Shape sh;
    if (forced) {
        sh = *forced;
    } else {
        nomad_config shaped = *cfg;
        const bool async = cfg->sched == NOMAD_SCHED_PERM || cfg->sched == NOMAD_SCHED_UNIFORM;
        if (async && cfg->waves_per_worker <= 0 && nnz > 0) {
            // a row holding more than half of a four-wave share of the ratings: six waves
            int64_t md = 0;
            int dev = 0, cus = 0;
            hipError_t e0 = nomad::max_row_degree(d_row, nnz, m, c->stream, &md);
            if (e0 == hipSuccess) e0 = hipGetDevice(&dev);
            if (e0 == hipSuccess) e0 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e0 != hipSuccess) return bail(hip_fail(c, e0, "nomad_init: row degrees"));
            const double pw = cfg->workers > 0 ? cfg->workers : cus;
            if (2.0 * (double)md * pw * nomad::kDefaultWavesAsync > (double)nnz)
                shaped.waves_per_worker = nomad::kDenseWavesAsync;
        }
        const nomad_status ss = choose_shape(&shaped, c->kp, c->wbytes, &sh, c);
        if (ss != NOMAD_OK) return bail(ss);
    }
    const int32_t nw = sh.nw, slots = sh.slots, window = sh.window, maxw = sh.maxw, cus = sh.cus, max_lds = sh.max_lds;
    int32_t p = cfg->workers;
    if (p <= 0) p = maxw < cus ? maxw : cus;
    if (p < 1 || p > nomad::kMaxWorkers)
        return bail(fail(c, NOMAD_EINVAL, "nomad_init: workers=%d outside [1,%d]", p, nomad::kMaxWorkers));
    if (p > maxw)
        return bail(fail(c, NOMAD_EDEVICE, "nomad_init: %d workers cannot all be resident (device holds %d "
                         "with %d compute waves and %d item slots)", p, maxw, nw, slots));
    c->p = p;
    c->nw = nw;
    c->slots = slots;
    c->window = window;
    c->cfg.window = window;
    c->cus = cus;
    c->max_lds = max_lds;
    c->cfg.workers = p;
    c->cfg.waves_per_worker = nw;
    c->cfg.item_slots = slots;

    hipError_t e;
    if ((e = hipGetDevice(&c->device)) != hipSuccess) return bail(hip_fail(c, e, "nomad_init: device"));
    prepare_noalloc_scratch(c->device);
    if ((e = hipMalloc(&c->W, (size_t)c->wbytes * (size_t)m * c->kp)) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: W"));
    if ((e = hipMalloc(&c->H, sizeof(float) * (size_t)n * c->kp)) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: H"));
    if ((e = hipMalloc(&c->tok_done, sizeof(uint32_t) * (size_t)(n + 1))) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: item counters"));
    if ((e = hipMalloc(&c->dummy, sizeof(float) * nomad::kMaxWaves * (size_t)p)) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: scratch words"));
    if ((e = hipMalloc(&c->diag, sizeof(int32_t) * 8)) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: diagnostics"));
    if ((e = hipMalloc(&c->wstats, sizeof(int64_t) * nomad::kWStatCount * (size_t)p)) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: worker counters"));
    if ((e = hipMalloc(&c->counters, sizeof(unsigned long long) * 4)) != hipSuccess ||
        (e = hipMemsetAsync(c->counters, 0, sizeof(unsigned long long) * 4, c->stream)) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: counters"));
    if (cfg->debug_ownership &&
        ((e = hipMalloc(&c->holder, sizeof(uint32_t) * (size_t)n)) != hipSuccess ||
         (e = hipMemsetAsync(c->holder, 0xFF, sizeof(uint32_t) * (size_t)n, c->stream)) != hipSuccess))
        return bail(hip_fail(c, e, "nomad_init: holder words"));
    c->eval_scratch_bytes = nomad::eval_scratch_bytes();
    if ((e = hipMalloc(&c->eval_scratch, c->eval_scratch_bytes)) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: scratch"));
    if ((e = hipEventCreate(&c->ev0)) != hipSuccess || (e = hipEventCreate(&c->ev1)) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: events"));
    hipStream_t st = c->stream;
    if ((e = hipMemsetAsync(c->W, 0, (size_t)c->wbytes * (size_t)m * c->kp, st)) != hipSuccess ||
        (e = hipMemsetAsync(c->H, 0, sizeof(float) * (size_t)n * c->kp, st)) != hipSuccess ||
        (e = hipMemsetAsync(c->tok_done, 0, sizeof(uint32_t) * (size_t)(n + 1), st)) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: clear"));
    if ((e = c->wbytes == 2
                 ? nomad::to_bf16(d_W0, c->k, (uint16_t *)c->W, c->kp, m, st)
                 : hipMemcpy2DAsync(c->W, sizeof(float) * c->kp, d_W0, sizeof(float) * c->k, sizeof(float) * c->k, m,
                                    hipMemcpyDeviceToDevice, st)) != hipSuccess ||
        (e = hipMemcpy2DAsync(c->H, sizeof(float) * c->kp, d_H0, sizeof(float) * c->k, sizeof(float) * c->k, n,
                              hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: copy initial factors"));

    if ((e = hipEventRecord(c->ev0, st)) != hipSuccess) return bail(hip_fail(c, e, "nomad_init: event"));
    int code = 0;
    char msg[256] = {0};
    e = nomad::build_plan(&c->plan, m, n, nnz, d_row, d_col, d_val, p, nw, window, cfg->seed, st, &code, msg,
                          sizeof(msg));
    if (e != hipSuccess) return bail(hip_fail(c, e, "nomad_init: layout"));
    if (code != 0) return bail(fail(c, (nomad_status)code, "nomad_init: %s", msg));
    if (cfg->sched == NOMAD_SCHED_RING && cfg->t_source == 1 &&
        (e = nomad::build_visit_starts(&c->plan, cfg->seed, st)) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: visit positions"));
    if (cfg->sched == NOMAD_SCHED_PERM || cfg->sched == NOMAD_SCHED_UNIFORM) {
        if (c->plan.nvisits >= (int64_t)INT32_MAX)
            return bail(fail(c, NOMAD_EINVAL, "nomad_init: %lld (worker, item) visits per epoch are too many for the "
                             "asynchronous schedules", (long long)c->plan.nvisits));
        if (cfg->sched == NOMAD_SCHED_UNIFORM && (int64_t)p * n >= (int64_t)INT32_MAX)
            return bail(fail(c, NOMAD_EINVAL, "nomad_init: uniform routing needs workers x items < 2^31"));
        if ((e = nomad::build_async_tables(&c->plan, st)) != hipSuccess)
            return bail(hip_fail(c, e, "nomad_init: asynchronous tables"));
        if (cfg->sched == NOMAD_SCHED_UNIFORM && (e = nomad::build_holder_map(&c->plan, st)) != hipSuccess)
            return bail(hip_fail(c, e, "nomad_init: holder map"));
        const int64_t nv = c->plan.nvisits > 0 ? c->plan.nvisits : 1;
        // permutation: a worker's queue holds its local items; uniform routing: any item
        c->queue_len = cfg->sched == NOMAD_SCHED_UNIFORM ? (int64_t)p * n : nv;
        c->async_scratch_bytes = nomad::async_scratch_bytes(n, p);
        if ((e = hipMalloc(&c->queue, sizeof(uint64_t) * (size_t)c->queue_len)) != hipSuccess ||
            (e = hipMalloc(&c->tvis, sizeof(int32_t) * (size_t)nv)) != hipSuccess ||
            (e = hipMalloc(&c->upd, sizeof(unsigned long long))) != hipSuccess ||
            (e = hipMemsetAsync(c->tvis, 0, sizeof(int32_t) * (size_t)nv, st)) != hipSuccess ||
            (e = hipMalloc(&c->qtail, sizeof(uint32_t) * (size_t)p)) != hipSuccess ||
            (e = hipMalloc(&c->qhead, sizeof(uint32_t) * (size_t)p)) != hipSuccess ||
            (e = hipMalloc(&c->parked, sizeof(uint32_t))) != hipSuccess ||
            (e = hipMalloc(&c->istate, sizeof(int32_t) * 4 * (size_t)n)) != hipSuccess ||
            (e = hipMalloc(&c->async_scratch, c->async_scratch_bytes)) != hipSuccess ||
            (e = hipMemsetAsync(c->istate, 0, sizeof(int32_t) * 4 * (size_t)n, st)) != hipSuccess)
            return bail(hip_fail(c, e, "nomad_init: queues"));
    }
    if ((e = hipEventRecord(c->ev1, st)) != hipSuccess || (e = hipEventSynchronize(c->ev1)) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: event"));
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
    c->layout_seconds = ms * 1e-3;
    c->row_start.resize(p + 1);
    if ((e = hipMemcpy(c->row_start.data(), c->plan.row_start, sizeof(int64_t) * (p + 1), hipMemcpyDeviceToHost)) !=
        hipSuccess)
        return bail(hip_fail(c, e, "nomad_init: partition copy"));
    // A row holding more than half of a compute wave's share of the ratings dominates its
    // wave: most of the wave's visits are then a single rating on that row, and the kernel
    // with the kept-row path for such visits is the one launched.
    c->keep_rows = (cfg->sched == NOMAD_SCHED_PERM || cfg->sched == NOMAD_SCHED_UNIFORM) && nnz > 0 &&
                   2.0 * (double)c->plan.max_row_degree * p * nw > (double)nnz;
    *out = c;
    return NOMAD_OK;
}

nomad_status nomad_init(nomad_ctx **out, const nomad_config *cfg, int64_t m, int64_t n, int64_t nnz,
                        const int32_t *d_row, const int32_t *d_col, const float *d_val, const float *d_W0,
                        const float *d_H0, void *hip_stream) {
    // Transposed: NOMAD on A^T, whose rows are A's columns (section 3.1's symmetric choice).
    if (cfg && cfg->transpose == 1)
        return init_impl(out, cfg, n, m, nnz, d_col, d_row, d_val, d_H0, d_W0, hip_stream, nullptr);
    return init_impl(out, cfg, m, n, nnz, d_row, d_col, d_val, d_W0, d_H0, hip_stream, nullptr);
}

// Launch arguments of context c that do not depend on the call.
static void fill_args(nomad_ctx *c, nomad::TrainArgs &a) {
    a.m = c->m;
    a.n = c->n;
    a.nnz = c->nnz;
    a.wave_start = c->plan.wave_start;
    a.vstart = c->plan.vstart;
    a.owner = c->holder;
    a.counters = c->counters;
    a.gstep = c->cfg.t_source == 1 ? 1 : 0;
    a.loss = c->cfg.loss;
    a.W = c->W;
    a.H = c->H;
    a.recs = c->plan.recs;
    a.rbase = c->plan.rbase;
    a.visits = c->plan.visits;
    a.vbase = c->plan.vbase;
    a.tok_done = c->tok_done;
    a.abort_flag = c->tok_done + c->n;
    a.dummy = c->dummy;
    a.diag = c->diag;
    a.kp = c->kp;
    a.keep_rows = c->keep_rows;
    a.wbytes = c->wbytes;
    a.rounding = c->cfg.rounding == NOMAD_ROUND_STOCHASTIC ? 1 : 0;
    a.sr_seed = (uint32_t)c->cfg.seed;
    a.p = c->p;
    a.nw = c->nw;
    a.slots = c->slots;
    a.window = c->window;
    a.lambda = c->cfg.lambda;
    a.alpha = c->cfg.alpha;
    a.beta = c->cfg.beta;
    a.gamma = c->cfg.gamma;
    a.wstats = c->wstats;
    a.timing = c->cfg.collect_stats != 0;
}

// Checks before a call of `epochs` epochs on context c.
static nomad_status check_epochs(nomad_ctx *c, int32_t epochs, const char *who) {
    if (c->epochs_done + epochs > (int64_t)INT32_MAX / 2)
        return fail(c, NOMAD_EINVAL, "%s: epoch counter would overflow", who);
    if ((int64_t)nomad::kMaxEpochsPerLaunch * c->plan.max_worker_visits >= (int64_t)INT32_MAX)
        return fail(c, NOMAD_EINVAL, "%s: %lld visits per epoch on the busiest worker are too many", who,
                    (long long)c->plan.max_worker_visits);
    return NOMAD_OK;
}

// The abort word of context c after a launch: NOMAD_OK, or the failure it records.
static nomad_status check_abort(nomad_ctx *c, const char *who) {
    uint32_t aborted = 0;
    HIPTRY(c, hipMemcpy(&aborted, c->tok_done + c->n, sizeof(uint32_t), hipMemcpyDeviceToHost), "train: flag");
    if (aborted) c->failed = true;
    if (aborted == 2)
        return fail(c, NOMAD_EDEVICE, "%s: malformed layout detected; the factors are undefined", who);
    if (aborted) {
        int32_t d[8] = {0};
        (void)hipMemcpy(d, c->diag, sizeof(d), hipMemcpyDeviceToHost);
        return fail(c, NOMAD_EDEVICE, "%s: a worker waited beyond the time limit (worker %d, wave %d, %d %d %d %d "
                    "%d %d); the factors are undefined", who, d[0] - 1, d[1], d[2], d[3], d[4], d[5], d[6], d[7]);
    }
    return NOMAD_OK;
}

// nomad_train_epochs of a batch: every problem runs `epochs` epochs, all in one launch per
// kMaxEpochsPerLaunch epochs.
static nomad_status train_batch(nomad_ctx *c, int32_t epochs, nomad_stats *out) {
    for (nomad_ctx *m : c->members) {
        const nomad_status st = check_epochs(m, epochs, "nomad_train_epochs");
        if (st != NOMAD_OK) return fail(c, st, "%s", m->err.c_str());
    }
    hipStream_t st = c->stream;
    double seconds = 0.0;
    if (epochs > 0 && c->graph && epochs == c->graph_epochs) {
        // The captured sequence: the problems' launch arguments as of now, then the graph
        // (resets, then per launch its epoch count and the workers).
        const size_t np = c->members.size();
        std::vector<nomad::TrainArgs> h(np);
        for (size_t b = 0; b < np; ++b) {
            fill_args(c->members[b], h[b]);
            h[b].epoch0 = (int32_t)c->members[b]->epochs_done;
            h[b].epochs = 0;
            h[b].wg0 = c->wg0[b];
        }
        HIPTRY(c, hipMemcpyAsync(c->d_descs, h.data(), sizeof(nomad::TrainArgs) * np, hipMemcpyHostToDevice, st),
               "train: arguments");
        HIPTRY(c, hipEventRecord(c->ev0, st), "train: event");
        HIPTRY(c, hipGraphLaunch(c->graph, st), "train: graph launch");
        HIPTRY(c, hipEventRecord(c->ev1, st), "train: event");
        HIPTRY(c, hipEventSynchronize(c->ev1), "train: kernel");
        float ms = 0.0f;
        HIPTRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1), "train: timing");
        seconds = ms * 1e-3;
        for (size_t b = 0; b < np; ++b) {
            const nomad_status ab = check_abort(c->members[b], "nomad_train_epochs");
            if (ab != NOMAD_OK) {
                c->failed = true;
                return fail(c, ab, "problem %zu of the batch: %s", b, c->members[b]->err.c_str());
            }
        }
        for (nomad_ctx *m : c->members) m->epochs_done += epochs;
        c->epochs_done += epochs;
    } else if (epochs > 0) {
        const size_t np = c->members.size();
        std::vector<nomad::TrainArgs> h(np);
        for (nomad_ctx *m : c->members) {
            HIPTRY(c, hipMemsetAsync(m->tok_done + m->n, 0, sizeof(uint32_t), st), "train: reset");
            HIPTRY(c, hipMemsetAsync(m->diag, 0, sizeof(int32_t) * 8, st), "train: reset");
            HIPTRY(c, hipMemsetAsync(m->wstats, 0, sizeof(int64_t) * nomad::kWStatCount * (size_t)m->p, st),
                   "train: reset");
            HIPTRY(c, hipMemsetAsync(m->counters, 0, sizeof(unsigned long long) * 2, st), "train: reset");
        }
        HIPTRY(c, hipEventRecord(c->ev0, st), "train: event");
        for (int32_t done = 0; done < epochs;) {
            const int32_t ne = std::min(epochs - done, (int32_t)nomad::kMaxEpochsPerLaunch);
            for (size_t b = 0; b < np; ++b) {
                nomad::TrainArgs a{};
                fill_args(c->members[b], a);
                a.epoch0 = (int32_t)(c->members[b]->epochs_done + done);
                a.epochs = ne;
                a.wg0 = c->wg0[b];
                h[b] = a;
            }
            HIPTRY(c, hipMemcpyAsync(c->d_descs, h.data(), sizeof(nomad::TrainArgs) * np, hipMemcpyHostToDevice, st),
                   "train: arguments");
            HIPTRY(c, nomad::launch_train_batch(h[0], c->total_wg, c->d_descs, c->d_wg, st), "train: launch");
            // the host arguments are rewritten by the next launch
            HIPTRY(c, hipStreamSynchronize(st), "train: kernel");
            done += ne;
        }
        HIPTRY(c, hipEventRecord(c->ev1, st), "train: event");
        HIPTRY(c, hipEventSynchronize(c->ev1), "train: kernel");
        float ms = 0.0f;
        HIPTRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1), "train: timing");
        seconds = ms * 1e-3;
        for (size_t b = 0; b < np; ++b) {
            const nomad_status ab = check_abort(c->members[b], "nomad_train_epochs");
            if (ab != NOMAD_OK) {
                c->failed = true;
                return fail(c, ab, "problem %zu of the batch: %s", b, c->members[b]->err.c_str());
            }
        }
        for (nomad_ctx *m : c->members) m->epochs_done += epochs;
        c->epochs_done += epochs;
    }
    if (out) {
        memset(out, 0, sizeof(*out));
        out->seconds = seconds;
        out->updates = (uint64_t)c->nnz * (uint64_t)epochs;
        out->epochs_done = (uint64_t)c->epochs_done;
        out->layout_seconds = c->layout_seconds;
        if (epochs > 0)
            for (nomad_ctx *m : c->members) {
                unsigned long long ctr[2] = {0, 0};
                HIPTRY(c, hipMemcpy(ctr, m->counters, sizeof(ctr), hipMemcpyDeviceToHost), "train: counters");
                out->violations += ctr[0];
                out->hops += ctr[1];
            }
    }
    return NOMAD_OK;
}

nomad_status nomad_train_epochs(nomad_ctx *c, int32_t epochs, nomad_stats *out) {
    if (!c) return fail(nullptr, NOMAD_ESTATE, "nomad_train_epochs: NULL context");
    if (c->owner) return fail(c, NOMAD_ESTATE, "nomad_train_epochs: this problem belongs to a batch; train the batch");
    if (epochs < 0) return fail(c, NOMAD_EINVAL, "nomad_train_epochs: epochs=%d < 0", epochs);
    if (c->failed)
        return fail(c, NOMAD_ESTATE, "nomad_train_epochs: an earlier launch failed; the factors are undefined "
                    "(destroy the context and build a new one)");
    if (!c->members.empty()) return train_batch(c, epochs, out);
    {
        const nomad_status ce = check_epochs(c, epochs, "nomad_train_epochs");
        if (ce != NOMAD_OK) return ce;
    }
    if (out) memset(out, 0, sizeof(*out));
    hipStream_t st = c->stream;
    double seconds = 0.0;
    if (epochs > 0 && c->nnz == 0) {
        // No ratings: every epoch is empty and no item has a worker to visit.
        c->trace_count = 0;
        c->epochs_done += epochs;
    } else if (epochs > 0) {
        nomad::TrainArgs a{};
        fill_args(c, a);
        if (c->cfg.record_trace) {
            // uniform routing visits holders a random number of times: room for three times
            // the expected count
            const int64_t need = c->plan.nvisits * (int64_t)epochs * (c->cfg.sched == NOMAD_SCHED_UNIFORM ? 3 : 1) +
                                 (c->cfg.sched == NOMAD_SCHED_UNIFORM ? 1024 : 0);
            if (need > c->trace_cap) {
                (void)hipFree(c->trace);
                c->trace = nullptr;
                c->trace_cap = 0;
                HIPTRY(c, hipMalloc(&c->trace, sizeof(int32_t) * 4 * (size_t)(need > 0 ? need : 1)), "trace");
                c->trace_cap = need;
            }
            if (!c->trace_len) HIPTRY(c, hipMalloc(&c->trace_len, sizeof(int64_t)), "trace");
            HIPTRY(c, hipMemsetAsync(c->trace_len, 0, sizeof(int64_t), st), "trace");
            a.trace = c->trace;
            a.trace_len = c->trace_len;
            a.trace_cap = c->trace_cap;
        }
        HIPTRY(c, hipMemsetAsync(c->tok_done + c->n, 0, sizeof(uint32_t), st), "train: reset");
        HIPTRY(c, hipMemsetAsync(c->diag, 0, sizeof(int32_t) * 8, st), "train: reset");
        HIPTRY(c, hipMemsetAsync(c->wstats, 0, sizeof(int64_t) * nomad::kWStatCount * (size_t)c->p, st), "train: reset");
        HIPTRY(c, hipMemsetAsync(c->counters, 0, sizeof(unsigned long long) * 2, st), "train: reset");
        const bool async = c->cfg.sched == NOMAD_SCHED_PERM || c->cfg.sched == NOMAD_SCHED_UNIFORM;
        const bool uniform = c->cfg.sched == NOMAD_SCHED_UNIFORM;
        if (async) {
            a.sched = uniform ? 2 : 1;
            a.tvis = c->tvis;
            a.hcnt = c->plan.hcnt;
            a.upd = c->upd;
            a.budget = (unsigned long long)c->nnz * (unsigned long long)epochs;
            a.hold = c->plan.hold;
            a.hx = c->plan.hx;
            a.hitem = c->plan.hitem;
            a.hoff = c->plan.hoff;
            a.xoff = c->plan.xoff;
            a.queue = c->queue;
            a.qtail = c->qtail;
            a.qhead = c->qhead;
            a.balance = c->cfg.balance ? 1 : 0;
            a.istate = c->istate;
            a.hmap = c->plan.hmap;
            a.parked = c->parked;
            a.active = c->plan.active;
            a.route_seed = (uint32_t)(c->cfg.seed >> 32) ^ (uint32_t)c->cfg.seed ^ 0x6a09e667u;
        }
        if (uniform) HIPTRY(c, hipMemsetAsync(c->upd, 0, sizeof(unsigned long long), st), "train: reset");
        // Launches of at most kMaxEpochsPerLaunch epochs (one launch per call for uniform
        // routing, which stops on its update budget instead).
        // Each training launch is timed on its own (the seeding kernels and resets of the
        // asynchronous schedules are not part of it).
        int32_t launches = 0;
        for (int32_t done = 0; done < epochs;) {
            const int32_t ne = uniform ? epochs : std::min(epochs - done, (int32_t)nomad::kMaxEpochsPerLaunch);
            a.epoch0 = (int32_t)(c->epochs_done + done);
            a.epochs = ne;
            while ((int32_t)c->lev.size() < 2 * (launches + 1)) {
                hipEvent_t ev = nullptr;
                HIPTRY(c, hipEventCreate(&ev), "train: event");
                c->lev.push_back(ev);
            }
            if (async) {
                HIPTRY(c, hipMemsetAsync(c->queue, 0, sizeof(uint64_t) * (size_t)c->queue_len, st), "train: reset");
                HIPTRY(c, hipMemsetAsync(c->qtail, 0, sizeof(uint32_t) * (size_t)c->p, st), "train: reset");
                HIPTRY(c, hipMemsetAsync(c->qhead, 0, sizeof(uint32_t) * (size_t)c->p, st), "train: reset");
                HIPTRY(c, hipMemsetAsync(c->parked, 0, sizeof(uint32_t), st), "train: reset");
                HIPTRY(c, nomad::seed_train_async(a, c->async_scratch, c->async_scratch_bytes, st), "train: seeding");
                HIPTRY(c, hipEventRecord(c->lev[2 * launches], st), "train: event");
                HIPTRY(c, nomad::launch_train_async(a, st), "train: launch");
            } else {
                HIPTRY(c, hipEventRecord(c->lev[2 * launches], st), "train: event");
                HIPTRY(c, nomad::launch_train(a, st), "train: launch");
            }
            HIPTRY(c, hipEventRecord(c->lev[2 * launches + 1], st), "train: event");
            ++launches;
            done += ne;
            if (done < epochs) {
                // a launch that stopped early ends the call: the next one would wait again
                const nomad_status ab = check_abort(c, "nomad_train_epochs");
                if (ab != NOMAD_OK) return ab;
            }
        }
        HIPTRY(c, hipEventSynchronize(c->lev[2 * launches - 1]), "train: kernel");
        for (int32_t l = 0; l < launches; ++l) {
            float ms = 0.0f;
            HIPTRY(c, hipEventElapsedTime(&ms, c->lev[2 * l], c->lev[2 * l + 1]), "train: timing");
            seconds += ms * 1e-3;
        }
        {
            const nomad_status ab = check_abort(c, "nomad_train_epochs");
            if (ab != NOMAD_OK) return ab;
        }
        if (c->cfg.record_trace) {
            HIPTRY(c, hipMemcpy(&c->trace_count, c->trace_len, sizeof(int64_t), hipMemcpyDeviceToHost), "trace");
            if (c->trace_count > c->trace_cap) c->trace_count = c->trace_cap;
        }
        c->epochs_done += epochs;
    }
    if (out) {
        out->seconds = seconds;
        out->updates = (uint64_t)c->nnz * (uint64_t)epochs;
        if (epochs > 0 && c->nnz > 0) {
            unsigned long long ctr[2] = {0, 0};
            HIPTRY(c, hipMemcpy(ctr, c->counters, sizeof(ctr), hipMemcpyDeviceToHost), "train: counters");
            out->violations = ctr[0];
            out->hops = ctr[1];
        }
        if (c->cfg.sched == NOMAD_SCHED_UNIFORM && epochs > 0 && c->nnz > 0) {
            unsigned long long u = 0;
            HIPTRY(c, hipMemcpy(&u, c->upd, sizeof(u), hipMemcpyDeviceToHost), "train: update count");
            out->updates = (uint64_t)u;
        }
        out->epochs_done = (uint64_t)c->epochs_done;
        out->layout_seconds = c->layout_seconds;
    }
    return NOMAD_OK;
}

nomad_status nomad_eval_rmse(nomad_ctx *c, int64_t nnz, const int32_t *d_row, const int32_t *d_col,
                             const float *d_val, double *rmse_out, double *objective_out) {
    if (!c) return fail(nullptr, NOMAD_ESTATE, "nomad_eval_rmse: NULL context");
    if (!c->members.empty())
        return fail(c, NOMAD_ESTATE, "nomad_eval_rmse: a batch; use nomad_batch_problem for one of its problems");
    if (!rmse_out) return fail(c, NOMAD_EINVAL, "nomad_eval_rmse: rmse_out is NULL");
    if (c->failed) return fail(c, NOMAD_ESTATE, "nomad_eval_rmse: an earlier launch failed; the factors are undefined");
    if (nnz < 0) return fail(c, NOMAD_EINVAL, "nomad_eval_rmse: nnz < 0");
    if (nnz > 0 && (!d_row || !d_col || !d_val)) return fail(c, NOMAD_EINVAL, "nomad_eval_rmse: NULL arrays");
    if (c->cfg.transpose == 1) std::swap(d_row, d_col);  // the context holds A^T
    double sq = 0.0, obj = 0.0;
    int bad = 0;
    if (nnz > 0) {
        HIPTRY(c, nomad::eval_sums(c->W, c->wbytes, c->H, c->k, c->kp, c->m, c->n, nnz, d_row, d_col, d_val,
                                   c->cfg.lambda, c->cfg.loss, &sq,
                                   &obj, &bad, c->eval_scratch, c->eval_scratch_bytes, c->stream),
               "eval");
        if (bad) return fail(c, NOMAD_EINVAL, "nomad_eval_rmse: rating index out of range");
    }
    *rmse_out = nnz > 0 ? std::sqrt(sq / (double)nnz) : NAN;
    if (objective_out) *objective_out = nnz > 0 ? obj : 0.0;
    return NOMAD_OK;
}

nomad_status nomad_eval_rmse_noalloc(nomad_ctx *c, int64_t nnz, const int32_t *d_row, const int32_t *d_col,
                                     const float *d_val, double *d_out) {
    if (!c) return fail(nullptr, NOMAD_ESTATE, "nomad_eval_rmse_noalloc: NULL context");
    if (!c->members.empty())
        return fail(c, NOMAD_ESTATE, "nomad_eval_rmse_noalloc: a batch; use nomad_batch_problem for one of its problems");
    if (c->failed)
        return fail(c, NOMAD_ESTATE, "nomad_eval_rmse_noalloc: an earlier launch failed; the factors are undefined");
    if (!d_out) return fail(c, NOMAD_EINVAL, "nomad_eval_rmse_noalloc: d_out is NULL");
    if (nnz < 0) return fail(c, NOMAD_EINVAL, "nomad_eval_rmse_noalloc: nnz < 0");
    if (nnz > nomad::noalloc_max_nnz())
        return fail(c, NOMAD_EINVAL, "nomad_eval_rmse_noalloc: nnz=%lld exceeds %lld, the most entries whose partial "
                    "sums its fixed %zu-byte scratch holds (use nomad_eval_rmse)", (long long)nnz,
                    (long long)nomad::noalloc_max_nnz(), nomad::noalloc_scratch_bytes());
    if (nnz > 0 && (!d_row || !d_col || !d_val)) return fail(c, NOMAD_EINVAL, "nomad_eval_rmse_noalloc: NULL arrays");
    if (c->cfg.transpose == 1) std::swap(d_row, d_col);  // the context holds A^T
    void *ptr = nullptr;
    if (c->device >= 0 && c->device < kMaxDevices) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        ptr = g_scratch_ptr[c->device];
        if (!ptr)
            return fail(c, NOMAD_EDEVICE, "nomad_eval_rmse_noalloc: no scratch address on device %d (%s)", c->device,
                        hipGetErrorString(g_scratch_err[c->device]));
    } else {
        return fail(c, NOMAD_EDEVICE, "nomad_eval_rmse_noalloc: device %d is beyond the %d the library tracks",
                    c->device, kMaxDevices);
    }
    HIPTRY(c, nomad::eval_sums_noalloc(c->W, c->wbytes, c->H, c->k, c->kp, c->m, c->n, nnz, d_row, d_col, d_val,
                                       c->cfg.lambda, c->cfg.loss, ptr, d_out, c->stream),
           "nomad_eval_rmse_noalloc");
    return NOMAD_OK;
}

nomad_status nomad_get_factors(nomad_ctx *c, float *d_W, float *d_H) {
    if (!c) return fail(nullptr, NOMAD_ESTATE, "nomad_get_factors: NULL context");
    if (!c->members.empty())
        return fail(c, NOMAD_ESTATE, "nomad_get_factors: a batch; use nomad_batch_problem for one of its problems");
    if (!d_W || !d_H) return fail(c, NOMAD_EINVAL, "nomad_get_factors: NULL output");
    if (c->failed) return fail(c, NOMAD_ESTATE, "nomad_get_factors: an earlier launch failed; the factors are undefined");
    if (c->cfg.transpose == 1) std::swap(d_W, d_H);  // the context's row factors are A's H
    if (c->wbytes == 2)
        HIPTRY(c, nomad::from_bf16((const uint16_t *)c->W, c->kp, d_W, c->k, c->m, c->stream), "get_factors");
    else
        HIPTRY(c, hipMemcpy2DAsync(d_W, sizeof(float) * c->k, c->W, sizeof(float) * c->kp, sizeof(float) * c->k, c->m,
                                   hipMemcpyDeviceToDevice, c->stream),
               "get_factors");
    HIPTRY(c, hipMemcpy2DAsync(d_H, sizeof(float) * c->k, c->H, sizeof(float) * c->kp, sizeof(float) * c->k, c->n,
                               hipMemcpyDeviceToDevice, c->stream),
           "get_factors");
    HIPTRY(c, hipStreamSynchronize(c->stream), "get_factors");
    return NOMAD_OK;
}

nomad_status nomad_get_partition(nomad_ctx *c, int32_t *p_out, int64_t *h_row_start, int64_t cap) {
    if (!c) return fail(nullptr, NOMAD_ESTATE, "nomad_get_partition: NULL context");
    if (!c->members.empty())
        return fail(c, NOMAD_ESTATE, "nomad_get_partition: a batch; use nomad_batch_problem for one of its problems");
    if (p_out) *p_out = c->p;
    if (h_row_start) {
        if (cap < c->p + 1) return fail(c, NOMAD_EINVAL, "nomad_get_partition: cap < p + 1");
        memcpy(h_row_start, c->row_start.data(), sizeof(int64_t) * (c->p + 1));
    }
    return NOMAD_OK;
}

nomad_status nomad_get_config(nomad_ctx *c, nomad_config *h_cfg) {
    if (!c) return fail(nullptr, NOMAD_ESTATE, "nomad_get_config: NULL context");
    if (!h_cfg) return fail(c, NOMAD_EINVAL, "nomad_get_config: h_cfg is NULL");
    *h_cfg = c->cfg;
    return NOMAD_OK;
}

nomad_status nomad_get_trace(nomad_ctx *c, int64_t *len, int32_t *h_buf, int64_t cap) {
    if (!c) return fail(nullptr, NOMAD_ESTATE, "nomad_get_trace: NULL context");
    if (!c->members.empty())
        return fail(c, NOMAD_ESTATE, "nomad_get_trace: a batch; use nomad_batch_problem for one of its problems");
    if (!len) return fail(c, NOMAD_EINVAL, "nomad_get_trace: len is NULL");
    *len = c->trace_count;
    if (h_buf && c->trace_count > 0) {
        int64_t cnt = cap < c->trace_count ? cap : c->trace_count;
        HIPTRY(c, hipMemcpy(h_buf, c->trace, sizeof(int32_t) * 4 * (size_t)cnt, hipMemcpyDeviceToHost), "trace");
    }
    return NOMAD_OK;
}

nomad_status nomad_get_worker_stats(nomad_ctx *c, int64_t *h_stats, int64_t cap) {
    if (!c) return fail(nullptr, NOMAD_ESTATE, "nomad_get_worker_stats: NULL context");
    if (!c->members.empty())
        return fail(c, NOMAD_ESTATE, "nomad_get_worker_stats: a batch; use nomad_batch_problem for one of its problems");
    if (!h_stats || cap < (int64_t)nomad::kWStatCount * c->p)
        return fail(c, NOMAD_EINVAL, "nomad_get_worker_stats: need room for %d values", nomad::kWStatCount * c->p);
    HIPTRY(c, hipMemcpy(h_stats, c->wstats, sizeof(int64_t) * nomad::kWStatCount * (size_t)c->p, hipMemcpyDeviceToHost),
           "worker stats");
    return NOMAD_OK;
}

nomad_status nomad_init_batched(nomad_ctx **out, int32_t nprob, const nomad_problem_desc *descs,
                                const nomad_config *common, void *hip_stream) {
    if (!out) return fail(nullptr, NOMAD_EINVAL, "nomad_init_batched: out is NULL");
    *out = nullptr;
    if (!common || !descs) return fail(nullptr, NOMAD_EINVAL, "nomad_init_batched: NULL argument");
    if (nprob < 1) return fail(nullptr, NOMAD_EINVAL, "nomad_init_batched: nprob=%d < 1", nprob);
    if (common->record_trace) return fail(nullptr, NOMAD_ENOTIMPL, "nomad_init_batched: traces are per problem only");
    if (common->sched != NOMAD_SCHED_RING)
        return fail(nullptr, NOMAD_ENOTIMPL, "nomad_init_batched: batches run the ring schedule");
    if (common->dtype != NOMAD_FP32 && common->dtype != NOMAD_BF16)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init_batched: storage type %d is not one of NOMAD_FP32, NOMAD_BF16",
                    common->dtype);
    int32_t kp = 0;
    uint64_t total_nnz = 0;
    for (int32_t b = 0; b < nprob; ++b) {
        if (descs[b].k < 1 || descs[b].k > nomad::kMaxK)
            return fail(nullptr, NOMAD_EINVAL, "nomad_init_batched: problem %d: k=%d outside [1,%d]", b, descs[b].k,
                        nomad::kMaxK);
        if (descs[b].nnz < 0) return fail(nullptr, NOMAD_EINVAL, "nomad_init_batched: problem %d: nnz < 0", b);
        kp = std::max(kp, nomad::padded_k(descs[b].k));
        total_nnz += (uint64_t)descs[b].nnz;
    }
    // With the window left to the library, a batch takes the smallest one: problems are
    // many and mostly small, so more (resident) workers beat deeper row windows.
    nomad_config shape_cfg = *common;
    if (shape_cfg.window <= 0) shape_cfg.window = 8;
    nomad::Shape sh;
    {
        const nomad_status ss = choose_shape(&shape_cfg, kp, common->dtype == NOMAD_BF16 ? 2 : 4, &sh, nullptr, true);
        if (ss != NOMAD_OK) return ss;
    }
    int32_t T = common->workers > 0 ? common->workers : std::min(sh.maxw, nomad::kMaxWorkers);
    if (T > sh.maxw)
        return fail(nullptr, NOMAD_EDEVICE, "nomad_init_batched: %d workers cannot all be resident (device holds %d)",
                    T, sh.maxw);
    if (nprob > T)
        return fail(nullptr, NOMAD_EINVAL, "nomad_init_batched: %d problems need at least one worker each; %d fit",
                    nprob, T);
    // Workers per problem in proportion to its ratings (at least one each), largest
    // remainders first.
    std::vector<int32_t> pb(nprob, 1);
    {
        std::vector<double> quota(nprob, 1.0);
        int32_t used = 0;
        for (int32_t b = 0; b < nprob; ++b) {
            quota[b] = total_nnz ? (double)T * (double)descs[b].nnz / (double)total_nnz : 1.0;
            pb[b] = std::max(1, (int32_t)quota[b]);
            used += pb[b];
        }
        while (used > T) {  // only possible through the "at least one" rule
            int32_t best = -1;
            for (int32_t b = 0; b < nprob; ++b)
                if (pb[b] > 1 && (best < 0 || pb[b] - quota[b] > pb[best] - quota[best])) best = b;
            --pb[best];
            --used;
        }
        while (used < T && total_nnz) {
            int32_t best = 0;
            for (int32_t b = 1; b < nprob; ++b)
                if (quota[b] - pb[b] > quota[best] - pb[best]) best = b;
            ++pb[best];
            ++used;
        }
    }
    nomad_ctx *c = new (std::nothrow) nomad_ctx();
    if (!c) return fail(nullptr, NOMAD_ENOMEM, "nomad_init_batched: host allocation failed");
    auto bail = [&](nomad_status st) {
        g_last_error = c->err;
        release(c);
        delete c;
        return st;
    };
    c->cfg = *common;
    c->cfg.workers = T;
    c->cfg.waves_per_worker = sh.nw;
    c->cfg.item_slots = sh.slots;
    c->cfg.window = sh.window;
    c->stream = (hipStream_t)hip_stream;
    c->shape = sh;
    c->kp = kp;
    c->nw = sh.nw;
    c->slots = sh.slots;
    c->window = sh.window;
    std::vector<int32_t> wg_prob;
    for (int32_t b = 0; b < nprob; ++b) {
        nomad_config cb = *common;
        cb.k = descs[b].k;
        cb.lambda = descs[b].lambda;
        cb.alpha = descs[b].alpha;
        cb.beta = descs[b].beta;
        cb.gamma = descs[b].gamma;
        cb.workers = pb[b];
        nomad_ctx *m = nullptr;
        const nomad_status st = init_impl(&m, &cb, descs[b].m, descs[b].n, descs[b].nnz, descs[b].d_row,
                                          descs[b].d_col, descs[b].d_val, descs[b].d_W0, descs[b].d_H0, hip_stream, &sh);
        if (st != NOMAD_OK) return bail(fail(c, st, "nomad_init_batched: problem %d: %s", b, g_last_error.c_str()));
        m->owner = c;
        c->members.push_back(m);
        c->wg0.push_back((int32_t)wg_prob.size());
        for (int32_t q = 0; q < pb[b]; ++q) wg_prob.push_back(b);
        c->nnz += descs[b].nnz;
        c->layout_seconds += m->layout_seconds;
    }
    c->total_wg = (int32_t)wg_prob.size();
    c->p = c->total_wg;
    hipError_t e;
    if ((e = hipMalloc(&c->d_descs, sizeof(nomad::TrainArgs) * (size_t)nprob)) != hipSuccess ||
        (e = hipMalloc(&c->d_wg, sizeof(int32_t) * wg_prob.size())) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init_batched: launch tables"));
    if ((e = hipMemcpy(c->d_wg, wg_prob.data(), sizeof(int32_t) * wg_prob.size(), hipMemcpyHostToDevice)) !=
        hipSuccess)
        return bail(hip_fail(c, e, "nomad_init_batched: launch tables"));
    if ((e = hipEventCreate(&c->ev0)) != hipSuccess || (e = hipEventCreate(&c->ev1)) != hipSuccess)
        return bail(hip_fail(c, e, "nomad_init_batched: events"));
    *out = c;
    return NOMAD_OK;
}

nomad_status nomad_batch_problem(nomad_ctx *c, int32_t b, nomad_ctx **problem) {
    if (!problem) return fail(c, NOMAD_EINVAL, "nomad_batch_problem: problem is NULL");
    *problem = nullptr;
    if (!c || c->members.empty()) return fail(c, NOMAD_ESTATE, "nomad_batch_problem: not a batch");
    if (b < 0 || b >= (int32_t)c->members.size())
        return fail(c, NOMAD_EINVAL, "nomad_batch_problem: b=%d outside [0,%zu)", b, c->members.size());
    *problem = c->members[b];
    return NOMAD_OK;
}

nomad_status nomad_batch_graph(nomad_ctx *c, int32_t epochs) {
    if (!c || c->members.empty()) return fail(c, NOMAD_ESTATE, "nomad_batch_graph: not a batch");
    if (epochs < 0) return fail(c, NOMAD_EINVAL, "nomad_batch_graph: epochs=%d < 0", epochs);
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
    c->graph_epochs = 0;
    if (epochs == 0) return NOMAD_OK;
    const int32_t np = (int32_t)c->members.size();
    nomad::TrainArgs shape{};
    fill_args(c->members[0], shape);  // the launch shape all problems share
    // Capture on a private stream (the batch's may be the null stream, which cannot be
    // captured); the graph is replayed on the batch's stream.
    hipStream_t cs = nullptr;
    HIPTRY(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "nomad_batch_graph: stream");
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        e = nomad::launch_batch_reset(c->d_descs, np, cs);
        int32_t prev = 0;
        for (int32_t done = 0; e == hipSuccess && done < epochs;) {
            const int32_t ne = std::min(epochs - done, (int32_t)nomad::kMaxEpochsPerLaunch);
            e = nomad::launch_batch_epochs(c->d_descs, np, ne, prev, cs);
            if (e == hipSuccess) e = nomad::launch_train_batch(shape, c->total_wg, c->d_descs, c->d_wg, cs);
            prev = ne;
            done += ne;
        }
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        c->graph = nullptr;
        return hip_fail(c, e, "nomad_batch_graph: capture");
    }
    c->graph_epochs = epochs;
    return NOMAD_OK;
}

nomad_status nomad_tune_batched(int32_t nprob, const nomad_problem_desc *descs, const nomad_config *common,
                                void *hip_stream, nomad_tune_progress progress, void *user, nomad_config *best,
                                double *best_seconds) {
    if (!common || !best) return fail(nullptr, NOMAD_EINVAL, "nomad_tune_batched: NULL config");
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(nullptr, NOMAD_EDEVICE, "nomad_tune_batched: no usable HIP device");
    // Candidates: one or two workers per CU, four or eight compute waves (the row window
    // stays the batch's default unless set); a field the caller set stays as set.
    std::vector<int32_t> ws, nws, wins;
    if (common->workers > 0) ws = {common->workers}; else ws = {cus, 2 * cus};
    if (common->waves_per_worker > 0) nws = {common->waves_per_worker}; else nws = {4, 8};
    wins = {common->window};
    double tbest = 0.0;
    bool found = false;
    std::string last;
    for (int32_t w : ws)
        for (int32_t nw : nws)
            for (int32_t win : wins) {
                nomad_config cfg = *common;
                cfg.workers = w;
                cfg.waves_per_worker = nw;
                cfg.window = win;
                nomad_ctx *c = nullptr;
                const nomad_status si = nomad_init_batched(&c, nprob, descs, &cfg, hip_stream);
                if (si != NOMAD_OK) {
                    last = g_last_error;  // the shape does not fit (LDS, residency): next one
                    if (progress) progress(&cfg, si, 0.0, user);
                    continue;
                }
                // the faster of two epochs (the first also loads the kernel's code)
                double t = 0.0;
                bool ok = true;
                for (int r = 0; r < 2 && ok; ++r) {
                    nomad_stats stt{};
                    ok = nomad_train_epochs(c, 1, &stt) == NOMAD_OK;
                    if (ok) t = r == 0 ? stt.seconds : std::min(t, stt.seconds);
                }
                if (!ok) last = c->err;
                nomad_destroy(c);
                if (progress) progress(&cfg, ok ? NOMAD_OK : NOMAD_EDEVICE, t, user);
                if (ok && (!found || t < tbest)) {
                    found = true;
                    tbest = t;
                    *best = cfg;
                }
            }
    if (!found) return fail(nullptr, NOMAD_EDEVICE, "nomad_tune_batched: no launch shape worked (%s)", last.c_str());
    if (best_seconds) *best_seconds = tbest;
    return NOMAD_OK;
}

void nomad_destroy(nomad_ctx *c) {
    if (!c || c->owner) return;  // a problem of a batch goes with its batch
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    release(c);
    delete c;
}

const char *nomad_last_error(const nomad_ctx *c) {
    if (c) return c->err.c_str();
    return g_last_error.c_str();
}

}  // extern "C"
