/*
 * NOMAD oracle -- a plain, slow, FP64 CPU implementation of what the NOMAD hot path
 * computes (Yun, Yu, Hsieh, Vishwanathan, Dhillon: "NOMAD: Non-locking, stOchastic
 * Multi-machine algorithm for Asynchronous and Decentralized matrix completion").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  The product path (the HIP library) never
 * calls it, includes it, or shares a line of code, a header or a table with it.
 *
 * Everything is IEEE double precision, single threaded, written for readability:
 * no blocking, fusion or reordering beyond what the paper states.
 *
 * What each function follows:
 *   orc_update       -- SGD updates eq. (w_update)/(h_update), section 2.3, applied to the
 *                       per-rating loss of eq. (obj_fcn) in its simplified per-rating form.
 *                       Readings: descent direction (the printed bracket is the negative
 *                       gradient of the squared loss, so the update adds it), w_i (not w_j)
 *                       in the h-update, one residual shared by both updates, and the h
 *                       step uses the pre-update w_i (simultaneous update).
 *   orc_residual, orc_loss, orc_update_loss -- the same update for a general separable
 *                       loss (section 2 states the method for any; the conclusion writes the
 *                       objective as a sum of per-rating terms): e = -d loss / d <w,h>.
 *                       Square loss (the paper's) and the logistic loss of labels +-1.
 *                       orc_train_ring_loss, orc_replay_loss and orc_objective_loss take
 *                       the loss; the functions without the suffix use the square loss.
 *   orc_step         -- step-size schedule eq. (stepsize_method), section 5.1, with the
 *                       exponent generalised to gamma (the paper uses 1.5).
 *   orc_partition    -- row partition I_1..I_p of section 3.1, in the "same number of
 *                       ratings per set" form given in that section's footnote.
 *   orc_owner0       -- initial uniformly random queue of each item (Algorithm 1, queue
 *                       initialisation), realised by the splitmix64 mixing function
 *                       (Steele, Lea, Flood 2014; Vigna's splitmix64.c).
 *   orc_train_ring   -- Algorithm 1 with a fixed token-passing order: every worker q at
 *                       sub-step s works on the items first placed at worker (q+s) mod p,
 *                       in ascending item order; items move from worker q to q-1.
 *   orc_train_ring_interleaved -- the same per-worker and per-item orders executed under
 *                       a random asynchronous interleaving (serializability, section 1
 *                       and section 4.4).
 *   orc_train_perm   -- Algorithm 1 with the random-permutation circulation of section 3.4:
 *                       each item visits every worker holding its ratings once per epoch, in
 *                       uniformly random order, workers take turns at random.  With
 *                       balance = 1, section 3.3's dynamic load balancing: of two candidate
 *                       holders not yet visited the one with the shorter queue comes next.
 *   orc_balanced_pick -- that choice on its own: the less loaded of two candidates.
 *   orc_train_uniform -- Algorithm 1 literally: recipient uniform over all p workers, t is
 *                       the per-(worker,item) visit count, stop after a number of updates.
 *                       With balance = 1 (section 3.3) the recipient is the less loaded of
 *                       two workers drawn uniformly.  With slots > 0 the turns follow time
 *                       instead of a uniform draw (see orc_train_uniform).
 *   orc_train_ring_gcount -- the ring order with t read as the global count of updates
 *                       applied before the visit (the alternative reading of t in the step
 *                       size of section 5.1).
 *   orc_train_threaded -- Algorithm 1 run literally by one POSIX thread per worker, each
 *                       with a mutex-protected FIFO queue and uniformly random recipients
 *                       (the CPU throughput baseline; its interleaving depends on timing).
 *   orc_replay       -- re-execute a recorded sequence of (worker, item, t, seq) visits.
 *   orc_train_ring_bf16 -- the ring order with the rows w_i stored in bfloat16 (the
 *                       storage form of the benchmark's BF16 configuration; the paper
 *                       itself works in FP32/FP64): the update is computed in FP64 from
 *                       the stored values, rounded to FP32, then to bfloat16 (nearest-even,
 *                       or stochastically with a counter hash).  Parity unpinned beyond
 *                       the rounding primitives: there is no closed form for a BF16 SGD
 *                       trajectory.
 *   orc_rmse / orc_objective -- test RMSE of section 5.1 and J(W,H) of eq. (obj_fcn),
 *                       with FP64 dot products and Neumaier-compensated sums.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <sched.h>
#include <time.h>

#include <stdio.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EDEADLOCK (-3)

typedef struct {
    int64_t updates;     /* SGD updates applied */
    int64_t visits;      /* (worker, item) visits that applied at least one update */
    int64_t violations;  /* updates whose row or item was not owned by the worker */
    int64_t hops;        /* item transfers between workers */
    int64_t max_queue;   /* longest queue seen when an item was pushed (asynchronous emulations) */
} orc_stats;

/* ------------------------------------------------------------------------------- */
/* Counter-based mixing function splitmix64 (published definition).                 */
/* ------------------------------------------------------------------------------- */
uint64_t orc_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Worker whose queue receives item j at start-up: uniform over 0..p-1. */
int32_t orc_owner0(uint64_t seed, int64_t j, int32_t p)
{
    return (int32_t)(orc_splitmix64(seed ^ (uint64_t)j) % (uint64_t)p);
}

/* s_t = alpha / (1 + beta * t^gamma). */
double orc_step(double alpha, double beta, double gamma, double t)
{
    return alpha / (1.0 + beta * pow(t, gamma));
}

/* The residual e = -d loss(r, d) / d d of one rating at prediction d = <w, h>.  The
 * method takes any separable loss (section 2; the objective as a sum of per-rating terms in
 * the conclusion); loss 0 is the square loss (r - d)^2 / 2 the paper works with, so
 * e = r - d; loss 1 is the logistic loss log(1 + exp(-r d)) of labels r = +-1, so
 * e = r / (1 + exp(r d)). */
double orc_residual(double r, double d, int32_t loss)
{
    if (loss == 1) return r / (1.0 + exp(r * d));
    return r - d;
}

/* The per-rating loss itself (without the regulariser): (r - d)^2 / 2, or
 * log(1 + exp(-r d)) written as max(z, 0) + log1p(exp(-|z|)) with z = -r d. */
double orc_loss(double r, double d, int32_t loss)
{
    if (loss == 1) {
        double z = -r * d;
        return (z > 0.0 ? z : 0.0) + log1p(exp(-fabs(z)));
    }
    return 0.5 * (r - d) * (r - d);
}

/* One SGD update on rating r of (w, h) with step s (section 2.3: one residual, both
 * vectors from their values before the update), for the given loss. */
void orc_update_loss(int32_t k, double *w, double *h, double r, double s, double lambda, int32_t loss)
{
    double d = 0.0;
    for (int32_t l = 0; l < k; ++l) d += w[l] * h[l];
    double e = orc_residual(r, d, loss);
    for (int32_t l = 0; l < k; ++l) {
        double wl = w[l], hl = h[l];
        w[l] = wl + s * (e * hl - lambda * wl);
        h[l] = hl + s * (e * wl - lambda * hl);
    }
}

/* The square-loss update. */
void orc_update(int32_t k, double *w, double *h, double r, double s, double lambda)
{
    orc_update_loss(k, w, h, r, s, lambda, 0);
}

/* row_start[q] = smallest i with (#ratings in rows < i) >= ceil(q*nnz/p), q = 1..p-1;
 * row_start[0] = 0 and row_start[p] = m. */
int orc_partition(int64_t m, int64_t nnz, const int32_t *row, int32_t p, int64_t *row_start)
{
    if (p <= 0 || m < 0 || nnz < 0) return ORC_EINVAL;
    int64_t *deg = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
    if (!deg) return ORC_ENOMEM;
    for (int64_t e = 0; e < nnz; ++e) {
        if (row[e] < 0 || row[e] >= m) { free(deg); return ORC_EINVAL; }
        deg[row[e]]++;
    }
    row_start[0] = 0;
    row_start[p] = m;
    int64_t i = 0, prefix = 0; /* prefix = #ratings in rows < i */
    for (int32_t q = 1; q < p; ++q) {
        int64_t target = (q * nnz + p - 1) / p; /* ceil(q*nnz/p) */
        while (prefix < target) { prefix += deg[i]; ++i; }
        row_start[q] = i;
    }
    free(deg);
    return ORC_OK;
}

/* Worker that owns row i: the q with row_start[q] <= i < row_start[q+1]. */
static int32_t worker_of_row(const int64_t *row_start, int32_t p, int64_t i)
{
    int32_t lo = 0, hi = p - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) / 2;
        if (row_start[mid] <= i) lo = mid; else hi = mid - 1;
    }
    /* skip empty workers that share the same start */
    while (lo + 1 < p && row_start[lo + 1] <= i) ++lo;
    return lo;
}

/* ------------------------------------------------------------------------------- */
/* The partitioned data: each worker's ratings grouped by item, ascending row.       */
/* ------------------------------------------------------------------------------- */
typedef struct {
    int32_t i, j, q, s; /* row, item, owning worker, ring sub-step (g(j) - q) mod p */
    double r;
} rating;

typedef struct {
    int32_t q, j;       /* worker and item */
    int64_t begin, end; /* its ratings: ratings[begin..end) */
    int32_t v;          /* ordinal of this visit among the item's visits in one ring epoch */
} visit;

typedef struct {
    int64_t m, n, nnz;
    int32_t p;
    int64_t *row_start;
    rating *ratings;  /* sorted by (q, s, j, i) */
    visit *visits;    /* one per nonempty (q, j), in the same order */
    int64_t nvisit;
    int64_t *wvis;    /* worker q's visits: visits[wvis[q]..wvis[q+1]) */
    int32_t *nhold;   /* number of workers holding ratings of item j */
    /* per item, its visits in ring order: ivis[istart[j]..istart[j+1]) index visits[] */
    int64_t *istart, *ivis;
    int32_t loss;     /* the per-rating loss of the updates (orc_residual); 0 unless set */
} layout;

static int cmp_qsji(const void *a, const void *b)
{
    const rating *x = (const rating *)a, *y = (const rating *)b;
    if (x->q != y->q) return x->q < y->q ? -1 : 1;
    if (x->s != y->s) return x->s < y->s ? -1 : 1;
    if (x->j != y->j) return x->j < y->j ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    return 0;
}

static void layout_free(layout *L)
{
    free(L->row_start); free(L->ratings); free(L->visits); free(L->wvis);
    free(L->nhold); free(L->istart); free(L->ivis);
    memset(L, 0, sizeof(*L));
}

static int layout_build(layout *L, int64_t m, int64_t n, int64_t nnz, const int32_t *row,
                        const int32_t *col, const float *val, int32_t p, uint64_t seed)
{
    memset(L, 0, sizeof(*L));
    if (p <= 0 || m < 0 || n < 0 || nnz < 0) return ORC_EINVAL;
    L->m = m; L->n = n; L->nnz = nnz; L->p = p;
    L->row_start = (int64_t *)malloc(sizeof(int64_t) * ((size_t)p + 1));
    L->ratings = (rating *)malloc(sizeof(rating) * ((size_t)nnz + 1));
    L->wvis = (int64_t *)calloc((size_t)p + 1, sizeof(int64_t));
    L->nhold = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    L->istart = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!L->row_start || !L->ratings || !L->wvis || !L->nhold || !L->istart) {
        layout_free(L); return ORC_ENOMEM;
    }
    for (int64_t e = 0; e < nnz; ++e) {
        if (row[e] < 0 || row[e] >= m || col[e] < 0 || col[e] >= n) { layout_free(L); return ORC_EINVAL; }
    }
    int rc = orc_partition(m, nnz, row, p, L->row_start);
    if (rc) { layout_free(L); return rc; }
    for (int64_t e = 0; e < nnz; ++e) {
        rating *x = &L->ratings[e];
        x->i = row[e]; x->j = col[e]; x->r = (double)val[e];
        x->q = worker_of_row(L->row_start, p, row[e]);
        int32_t g = orc_owner0(seed, col[e], p);
        x->s = (int32_t)(((int64_t)g - x->q + p) % p);
    }
    qsort(L->ratings, (size_t)nnz, sizeof(rating), cmp_qsji);
    /* duplicates are not allowed: Omega is a set of (i, j) positions */
    for (int64_t e = 1; e < nnz; ++e) {
        if (L->ratings[e].i == L->ratings[e - 1].i && L->ratings[e].j == L->ratings[e - 1].j) {
            layout_free(L); return ORC_EINVAL;
        }
    }
    /* visits: maximal runs of equal (q, j) */
    int64_t nv = 0;
    for (int64_t e = 0; e < nnz; ++e)
        if (e == 0 || L->ratings[e].q != L->ratings[e - 1].q || L->ratings[e].j != L->ratings[e - 1].j) ++nv;
    L->visits = (visit *)malloc(sizeof(visit) * ((size_t)nv + 1));
    L->ivis = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nv + 1));
    if (!L->visits || !L->ivis) { layout_free(L); return ORC_ENOMEM; }
    nv = 0;
    for (int64_t e = 0; e < nnz; ++e) {
        if (e == 0 || L->ratings[e].q != L->ratings[e - 1].q || L->ratings[e].j != L->ratings[e - 1].j) {
            if (nv > 0) L->visits[nv - 1].end = e;
            L->visits[nv].q = L->ratings[e].q;
            L->visits[nv].j = L->ratings[e].j;
            L->visits[nv].begin = e;
            ++nv;
        }
    }
    if (nv > 0) L->visits[nv - 1].end = nnz;
    L->nvisit = nv;
    for (int64_t v = 0; v < nv; ++v) { L->wvis[L->visits[v].q + 1]++; L->nhold[L->visits[v].j]++; }
    for (int32_t q = 0; q < p; ++q) L->wvis[q + 1] += L->wvis[q];
    /* per item: its visits ordered by ring sub-step (the order the ring schedule meets them) */
    for (int64_t j = 0; j < n; ++j) L->istart[j + 1] = L->istart[j] + L->nhold[j];
    int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!fill) { layout_free(L); return ORC_ENOMEM; }
    for (int64_t v = 0; v < nv; ++v) {
        int32_t j = L->visits[v].j;
        L->ivis[L->istart[j] + fill[j]++] = v;
    }
    /* insertion sort each item's visits by sub-step s (distinct per item) */
    for (int64_t j = 0; j < n; ++j) {
        int64_t a = L->istart[j], b = L->istart[j + 1];
        for (int64_t x = a + 1; x < b; ++x) {
            int64_t key = L->ivis[x];
            int32_t ks = L->ratings[L->visits[key].begin].s;
            int64_t y = x - 1;
            while (y >= a && L->ratings[L->visits[L->ivis[y]].begin].s > ks) {
                L->ivis[y + 1] = L->ivis[y]; --y;
            }
            L->ivis[y + 1] = key;
        }
        for (int64_t x = a; x < b; ++x) L->visits[L->ivis[x]].v = (int32_t)(x - a);
    }
    free(fill);
    return ORC_OK;
}

/* Progress report of long runs (off by default): a line on stderr every `every` updates,
 * counted over all runs in progress (several may run at once in different threads). */
static int64_t g_progress_every = 0, g_progress_next = 0, g_progress_done = 0;

void orc_set_progress(int64_t every)
{
    __atomic_store_n(&g_progress_done, 0, __ATOMIC_RELAXED);
    __atomic_store_n(&g_progress_next, every, __ATOMIC_RELAXED);
    __atomic_store_n(&g_progress_every, every, __ATOMIC_RELAXED);
}

static void progress_add(int64_t updates)
{
    const int64_t every = __atomic_load_n(&g_progress_every, __ATOMIC_RELAXED);
    if (every <= 0) return;
    const int64_t done = __atomic_add_fetch(&g_progress_done, updates, __ATOMIC_RELAXED);
    int64_t next = __atomic_load_n(&g_progress_next, __ATOMIC_RELAXED);
    if (done >= next && __atomic_compare_exchange_n(&g_progress_next, &next, done + every, 0, __ATOMIC_RELAXED,
                                                    __ATOMIC_RELAXED)) {
        fprintf(stderr, "[oracle] %lld updates applied\n", (long long)done);
        fflush(stderr);
    }
}

/* Apply one visit: worker q holding item j runs SGD over its ratings of j. */
static void apply_visit(const layout *L, const visit *V, int32_t k, double *W, double *H,
                        double lambda, double s, int32_t holder_ok, orc_stats *st)
{
    double *h = H + (int64_t)V->j * k;
    for (int64_t e = V->begin; e < V->end; ++e) {
        const rating *x = &L->ratings[e];
        int own_row = (x->i >= L->row_start[V->q] && x->i < L->row_start[V->q + 1]);
        if (st && (!own_row || !holder_ok)) st->violations++;
        orc_update_loss(k, W + (int64_t)x->i * k, h, x->r, s, lambda, L->loss);
        if (st) st->updates++;
    }
    if (st && V->end > V->begin) st->visits++;
    if (st) progress_add(V->end - V->begin);  /* (the threaded run passes no stats) */
}

static int check_common(int32_t k, int32_t p, int32_t epochs)
{
    return (k <= 0 || p <= 0 || epochs < 0) ? ORC_EINVAL : ORC_OK;
}

/* Fixed token-passing order.  For e in epochs, s in 0..p-1, q in 0..p-1: worker q
 * processes, in ascending item order, the items of group (q+s) mod p; t = epoch0 + e
 * (every rating is updated exactly once per epoch). */
int orc_train_ring_loss(int64_t m, int64_t n, int64_t nnz, const int32_t *row, const int32_t *col,
                        const float *val, int32_t k, double lambda, double alpha, double beta,
                        double gamma, int32_t p, uint64_t seed, int32_t epoch0, int32_t epochs,
                        double *W, double *H, orc_stats *st, int32_t loss)
{
    int rc = check_common(k, p, epochs);
    if (rc) return rc;
    if (loss != 0 && loss != 1) return ORC_EINVAL;
    layout L;
    rc = layout_build(&L, m, n, nnz, row, col, val, p, seed);
    if (rc) return rc;
    L.loss = loss;
    if (st) memset(st, 0, sizeof(*st));
    /* cursor[q] walks worker q's visits, which are sorted by sub-step */
    int64_t *cursor = (int64_t *)malloc(sizeof(int64_t) * ((size_t)p + 1));
    if (!cursor) { layout_free(&L); return ORC_ENOMEM; }
    for (int32_t e = 0; e < epochs; ++e) {
        double s_t = orc_step(alpha, beta, gamma, (double)(epoch0 + e));
        for (int32_t q = 0; q < p; ++q) cursor[q] = L.wvis[q];
        for (int32_t sub = 0; sub < p; ++sub) {
            for (int32_t q = 0; q < p; ++q) {
                while (cursor[q] < L.wvis[q + 1] &&
                       L.ratings[L.visits[cursor[q]].begin].s == sub) {
                    apply_visit(&L, &L.visits[cursor[q]], k, W, H, lambda, s_t, 1, st);
                    cursor[q]++;
                }
            }
        }
    }
    free(cursor);
    layout_free(&L);
    return ORC_OK;
}

int orc_train_ring(int64_t m, int64_t n, int64_t nnz, const int32_t *row, const int32_t *col,
                   const float *val, int32_t k, double lambda, double alpha, double beta,
                   double gamma, int32_t p, uint64_t seed, int32_t epoch0, int32_t epochs,
                   double *W, double *H, orc_stats *st)
{
    return orc_train_ring_loss(m, n, nnz, row, col, val, k, lambda, alpha, beta, gamma, p, seed, epoch0, epochs,
                               W, H, st, 0);
}

/* The ring order with t = the number of updates applied before the visit (globally,
 * starting from t0): every rating of a visit uses the count at the visit's start. */
int orc_train_ring_gcount(int64_t m, int64_t n, int64_t nnz, const int32_t *row, const int32_t *col,
                          const float *val, int32_t k, double lambda, double alpha, double beta,
                          double gamma, int32_t p, uint64_t seed, int64_t t0, int32_t epochs,
                          double *W, double *H, orc_stats *st)
{
    int rc = check_common(k, p, epochs);
    if (rc) return rc;
    layout L;
    rc = layout_build(&L, m, n, nnz, row, col, val, p, seed);
    if (rc) return rc;
    if (st) memset(st, 0, sizeof(*st));
    int64_t *cursor = (int64_t *)malloc(sizeof(int64_t) * ((size_t)p + 1));
    if (!cursor) { layout_free(&L); return ORC_ENOMEM; }
    int64_t t = t0;
    for (int32_t e = 0; e < epochs; ++e) {
        for (int32_t q = 0; q < p; ++q) cursor[q] = L.wvis[q];
        for (int32_t sub = 0; sub < p; ++sub) {
            for (int32_t q = 0; q < p; ++q) {
                while (cursor[q] < L.wvis[q + 1] &&
                       L.ratings[L.visits[cursor[q]].begin].s == sub) {
                    const visit *V = &L.visits[cursor[q]];
                    apply_visit(&L, V, k, W, H, lambda, orc_step(alpha, beta, gamma, (double)t), 1, st);
                    t += V->end - V->begin;
                    cursor[q]++;
                }
            }
        }
    }
    free(cursor);
    layout_free(&L);
    return ORC_OK;
}

/* The ring schedule's per-worker and per-item orders, executed under a random
 * interleaving of the workers: a worker may take its next visit as soon as the item's
 * previous visit (in ring order) is done.  Serializability says the result equals
 * orc_train_ring bit for bit. */
int orc_train_ring_interleaved(int64_t m, int64_t n, int64_t nnz, const int32_t *row,
                               const int32_t *col, const float *val, int32_t k, double lambda,
                               double alpha, double beta, double gamma, int32_t p, uint64_t seed,
                               int32_t epoch0, int32_t epochs, uint64_t interleave_seed,
                               double *W, double *H, orc_stats *st)
{
    int rc = check_common(k, p, epochs);
    if (rc) return rc;
    layout L;
    rc = layout_build(&L, m, n, nnz, row, col, val, p, seed);
    if (rc) return rc;
    if (st) memset(st, 0, sizeof(*st));
    int64_t *pos = (int64_t *)calloc((size_t)p, sizeof(int64_t));  /* visits done by q, all epochs */
    int64_t *done = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t)); /* visits done on item j */
    int32_t *live = (int32_t *)malloc(sizeof(int32_t) * (size_t)p);
    if (!pos || !done || !live) { free(pos); free(done); free(live); layout_free(&L); return ORC_ENOMEM; }
    int32_t nlive = 0;
    for (int32_t q = 0; q < p; ++q)
        if (L.wvis[q + 1] > L.wvis[q] && epochs > 0) live[nlive++] = q;
    uint64_t ctr = 0;
    int64_t misses = 0;
    while (nlive > 0) {
        int32_t pick = (int32_t)(orc_splitmix64(interleave_seed + ctr++) % (uint64_t)nlive);
        int32_t q = live[pick];
        int64_t per = L.wvis[q + 1] - L.wvis[q];
        int64_t e = pos[q] / per;
        const visit *V = &L.visits[L.wvis[q] + pos[q] % per];
        int64_t ticket = e * L.nhold[V->j] + V->v;
        if (done[V->j] != ticket) {
            if (++misses > 64LL * p + 1024) {
                /* scan: is any live worker able to move? */
                int any = 0;
                for (int32_t x = 0; x < nlive && !any; ++x) {
                    int32_t qq = live[x];
                    int64_t pp = L.wvis[qq + 1] - L.wvis[qq];
                    const visit *VV = &L.visits[L.wvis[qq] + pos[qq] % pp];
                    if (done[VV->j] == (pos[qq] / pp) * L.nhold[VV->j] + VV->v) any = 1;
                }
                if (!any) { rc = ORC_EDEADLOCK; break; }
                misses = 0;
            }
            continue;
        }
        misses = 0;
        apply_visit(&L, V, k, W, H, lambda, orc_step(alpha, beta, gamma, (double)(epoch0 + e)), 1, st);
        done[V->j]++;
        pos[q]++;
        if (pos[q] == per * epochs) live[pick] = live[--nlive];
    }
    free(pos); free(done); free(live);
    layout_free(&L);
    return rc;
}

/* ------------------------------------------------------------------------------- */
/* bfloat16 storage: the upper 16 bits of an IEEE single.                            */
/* ------------------------------------------------------------------------------- */

/* Integer hash "lowbias32" (C. Wellons, hash-prospector, 2018). */
uint32_t orc_lowbias32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

/* The 16 random bits of element l of the update of rating (i, j) in epoch t: a key
 * c = lowbias32(seed ^ i*0x9E3779B1 ^ j*0x85EBCA77 ^ t*0xC2B2AE3D) (32-bit arithmetic),
 * then the word lowbias32(c + l/2), whose low half serves even l and high half odd l. */
uint32_t orc_sr_bits(uint32_t seed, int64_t i, int64_t j, int64_t t, int32_t l)
{
    const uint32_t key = seed ^ ((uint32_t)i * 0x9E3779B1U) ^ ((uint32_t)j * 0x85EBCA77U) ^
                         ((uint32_t)t * 0xC2B2AE3DU);
    const uint32_t c = orc_lowbias32(key);
    const uint32_t word = orc_lowbias32(c + (uint32_t)(l >> 1));
    return (l & 1) ? (word >> 16) : (word & 0xFFFFU);
}

/* x rounded to FP32, then to bfloat16: rounding = 0 nearest-even (ties to the even
 * bfloat16), 1 stochastic (the 16 discarded bits are compared with `bits`: the magnitude
 * rounds up with probability equal to the discarded fraction).  Returns the bfloat16
 * value as a double.  Finite inputs only. */
double orc_round_bf16(double x, int32_t rounding, uint32_t bits)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if (rounding == 0)
        u = u + 0x7FFFU + ((u >> 16) & 1U);
    else
        u = u + (bits & 0xFFFFU);
    u &= 0xFFFF0000U;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* The ring order (as orc_train_ring) with w_i stored in bfloat16: W is rounded to
 * bfloat16 (nearest-even) on entry, and every update's new w_i is rounded with
 * orc_round_bf16 before it is stored; h_j, the residual and the update are FP64. */
int orc_train_ring_bf16(int64_t m, int64_t n, int64_t nnz, const int32_t *row, const int32_t *col,
                        const float *val, int32_t k, double lambda, double alpha, double beta,
                        double gamma, int32_t p, uint64_t seed, int32_t epoch0, int32_t epochs,
                        int32_t rounding, uint32_t sr_seed, double *W, double *H, orc_stats *st)
{
    int rc = check_common(k, p, epochs);
    if (rc) return rc;
    if (rounding != 0 && rounding != 1) return ORC_EINVAL;
    layout L;
    rc = layout_build(&L, m, n, nnz, row, col, val, p, seed);
    if (rc) return rc;
    if (st) memset(st, 0, sizeof(*st));
    for (int64_t x = 0; x < m * (int64_t)k; ++x) W[x] = orc_round_bf16(W[x], 0, 0);
    int64_t *cursor = (int64_t *)malloc(sizeof(int64_t) * ((size_t)p + 1));
    if (!cursor) { layout_free(&L); return ORC_ENOMEM; }
    for (int32_t e = 0; e < epochs; ++e) {
        const int64_t t = epoch0 + e;
        double s_t = orc_step(alpha, beta, gamma, (double)t);
        for (int32_t q = 0; q < p; ++q) cursor[q] = L.wvis[q];
        for (int32_t sub = 0; sub < p; ++sub) {
            for (int32_t q = 0; q < p; ++q) {
                while (cursor[q] < L.wvis[q + 1] &&
                       L.ratings[L.visits[cursor[q]].begin].s == sub) {
                    const visit *V = &L.visits[cursor[q]];
                    double *h = H + (int64_t)V->j * k;
                    for (int64_t x = V->begin; x < V->end; ++x) {
                        const rating *r = &L.ratings[x];
                        double *w = W + (int64_t)r->i * k;
                        orc_update(k, w, h, r->r, s_t, lambda);
                        for (int32_t l = 0; l < k; ++l)
                            w[l] = orc_round_bf16(w[l], rounding,
                                                  rounding ? orc_sr_bits(sr_seed, r->i, r->j, t, l) : 0);
                        if (st) st->updates++;
                    }
                    if (st && V->end > V->begin) st->visits++;
                    cursor[q]++;
                }
            }
        }
    }
    free(cursor);
    layout_free(&L);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------- */
/* Asynchronous emulation: FIFO queue per worker (linked through next[]), a seeded   */
/* scheduler picks uniformly among workers whose queue is not empty.                 */
/* ------------------------------------------------------------------------------- */
typedef struct {
    int32_t *head, *tail, *next; /* per-worker FIFO of items; next[j] links items */
    int32_t *ne, *ne_pos;        /* list of workers with a non-empty queue */
    int32_t nne;
} queues;

static int queues_init(queues *Q, int32_t p, int64_t n)
{
    Q->head = (int32_t *)malloc(sizeof(int32_t) * (size_t)p);
    Q->tail = (int32_t *)malloc(sizeof(int32_t) * (size_t)p);
    Q->next = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    Q->ne = (int32_t *)malloc(sizeof(int32_t) * (size_t)p);
    Q->ne_pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)p);
    if (!Q->head || !Q->tail || !Q->next || !Q->ne || !Q->ne_pos) return ORC_ENOMEM;
    for (int32_t q = 0; q < p; ++q) { Q->head[q] = Q->tail[q] = -1; Q->ne_pos[q] = -1; }
    Q->nne = 0;
    return ORC_OK;
}

static void queues_free(queues *Q)
{
    free(Q->head); free(Q->tail); free(Q->next); free(Q->ne); free(Q->ne_pos);
}

static void q_push(queues *Q, int32_t q, int32_t j)
{
    Q->next[j] = -1;
    if (Q->tail[q] < 0) {
        Q->head[q] = Q->tail[q] = j;
        Q->ne_pos[q] = Q->nne;
        Q->ne[Q->nne++] = q;
    } else {
        Q->next[Q->tail[q]] = j;
        Q->tail[q] = j;
    }
}

static int32_t q_pop(queues *Q, int32_t q)
{
    int32_t j = Q->head[q];
    Q->head[q] = Q->next[j];
    if (Q->head[q] < 0) {
        Q->tail[q] = -1;
        int32_t at = Q->ne_pos[q], last = Q->ne[--Q->nne];
        Q->ne[at] = last; Q->ne_pos[last] = at; Q->ne_pos[q] = -1;
    }
    return j;
}

/* Remove item j from worker q's queue (it is in it). */
static void q_remove(queues *Q, int32_t q, int32_t j)
{
    if (Q->head[q] == j) { (void)q_pop(Q, q); return; }
    int32_t prev = Q->head[q];
    while (Q->next[prev] != j) prev = Q->next[prev];
    Q->next[prev] = Q->next[j];
    if (Q->tail[q] == j) Q->tail[q] = prev;
}

/* Queue length of worker q. */
static int64_t q_len(const queues *Q, const int32_t *next, int32_t q)
{
    int64_t len = 0;
    for (int32_t j = Q->head[q]; j >= 0; j = next[j]) ++len;
    return len;
}

/* Section 3.3's dynamic load balancing reduced to one choice: of two candidate workers
 * a (the first drawn) and b, the one whose queue holds fewer items; a on a tie. */
int32_t orc_balanced_pick(int32_t a, int64_t len_a, int32_t b, int64_t len_b)
{
    return len_b < len_a ? b : a;
}

/* Index (into L->visits) of worker q's visit of item j, or -1 if q holds no rating of j. */
static int64_t find_visit(const layout *L, int32_t j, int32_t q)
{
    for (int64_t x = L->istart[j]; x < L->istart[j + 1]; ++x)
        if (L->visits[L->ivis[x]].q == q) return L->ivis[x];
    return -1;
}

/* Random-permutation circulation.  Each item starts at worker owner0(j); on every pop
 * the worker processes its ratings of the item (once per epoch), then sends it to a
 * uniformly random holder of the item's ratings that it has not visited in its current
 * epoch; when every holder has been visited, the item's epoch advances (t = epoch0 +
 * item epoch) and all holders become eligible again.  Items retire after `epochs`. */
/* trace (nullable): 4 ints per visit that applies updates, in execution order: worker,
 * item, t, visit number of the item (as orc_replay reads them), at most trace_cap visits;
 * *trace_len receives the count. */
static void trace_put(int32_t *trace, int64_t cap, int64_t *len, int32_t q, int32_t j, int64_t t, int64_t seq)
{
    if (trace && *len < cap) {
        int32_t *r = trace + 4 * *len;
        r[0] = q; r[1] = j; r[2] = (int32_t)t; r[3] = (int32_t)seq;
    }
    ++*len;
}

int orc_train_perm(int64_t m, int64_t n, int64_t nnz, const int32_t *row, const int32_t *col,
                   const float *val, int32_t k, double lambda, double alpha, double beta,
                   double gamma, int32_t p, uint64_t seed, int32_t epoch0, int32_t epochs,
                   uint64_t sched_seed, double *W, double *H, orc_stats *st,
                   int32_t *trace, int64_t trace_cap, int64_t *trace_len, int32_t balance)
{
    int rc = check_common(k, p, epochs);
    if (rc) return rc;
    layout L;
    rc = layout_build(&L, m, n, nnz, row, col, val, p, seed);
    if (rc) return rc;
    if (st) memset(st, 0, sizeof(*st));
    queues Q;
    int32_t *ep = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *left = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));   /* holders not yet visited */
    uint8_t *seen = (uint8_t *)calloc((size_t)L.nvisit + 1, 1);          /* per visit: done this epoch */
    int32_t *holder = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * ((size_t)p + 1));
    int64_t *nvisits = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *carry = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1)); /* held-over candidate visit, -1 none */
    if (queues_init(&Q, p, n) || !ep || !left || !seen || !holder || !cand || !nvisits || !carry) {
        queues_free(&Q); free(ep); free(left); free(seen); free(holder); free(cand); free(nvisits); free(carry);
        layout_free(&L); return ORC_ENOMEM;
    }
    for (int64_t j = 0; j < n; ++j) carry[j] = -1;
    int64_t tlen = 0;
    uint64_t ctr = 0;
    for (int64_t j = 0; j < n; ++j) {
        left[j] = L.nhold[j];
        holder[j] = -1;
        if (L.nhold[j] > 0 && epochs > 0) {
            holder[j] = orc_owner0(seed, j, p);
            q_push(&Q, holder[j], (int32_t)j);
        }
    }
    while (Q.nne > 0) {
        int32_t q = Q.ne[orc_splitmix64(sched_seed + ctr++) % (uint64_t)Q.nne];
        int32_t j = q_pop(&Q, q);
        int64_t vi = find_visit(&L, j, q);
        if (vi >= 0 && !seen[vi]) {
            apply_visit(&L, &L.visits[vi], k, W, H, lambda,
                        orc_step(alpha, beta, gamma, (double)(epoch0 + ep[j])), holder[j] == q, st);
            trace_put(trace, trace_cap, &tlen, q, j, epoch0 + ep[j], nvisits[j]++);
            seen[vi] = 1;
            left[j]--;
        }
        if (left[j] == 0) {
            ep[j]++;
            if (ep[j] == epochs) { holder[j] = -1; continue; }
            left[j] = L.nhold[j];
            for (int64_t x = L.istart[j]; x < L.istart[j + 1]; ++x) seen[L.ivis[x]] = 0;
        }
        int32_t nc = 0;
        for (int64_t x = L.istart[j]; x < L.istart[j + 1]; ++x)
            if (!seen[L.ivis[x]] && L.ivis[x] != carry[j]) cand[nc++] = L.ivis[x];
        int32_t dst;
        if (!balance) {
            dst = L.visits[cand[orc_splitmix64(sched_seed + ctr++) % (uint64_t)nc]].q;
        } else {
            /* two candidates not yet visited: the held-over one (or, if none, a first random
             * draw) and a random draw from the rest; the less loaded goes next, the other is
             * held over for the next choice (with nothing else left, the held-over one goes) */
            int64_t a = carry[j];
            if (a < 0 && nc > 0) {
                int32_t pick = (int32_t)(orc_splitmix64(sched_seed + ctr++) % (uint64_t)nc);
                a = cand[pick];
                cand[pick] = cand[--nc];
            }
            if (nc == 0) {
                dst = L.visits[a].q;
                carry[j] = -1;
            } else {
                int64_t b = cand[orc_splitmix64(sched_seed + ctr++) % (uint64_t)nc];
                int32_t qa = L.visits[a].q, qb = L.visits[b].q;
                dst = orc_balanced_pick(qa, q_len(&Q, Q.next, qa), qb, q_len(&Q, Q.next, qb));
                carry[j] = dst == qa ? b : a;
            }
        }
        holder[j] = dst;
        if (st) st->hops++;
        q_push(&Q, dst, j);
        if (st) { int64_t len = q_len(&Q, Q.next, dst); if (len > st->max_queue) st->max_queue = len; }
    }
    queues_free(&Q); free(ep); free(left); free(seen); free(holder); free(cand); free(nvisits); free(carry);
    layout_free(&L);
    if (trace_len) *trace_len = tlen;
    return ORC_OK;
}

/* Algorithm 1 literally: recipient uniform over all p workers; t = number of earlier
 * updates of the (i, j) pair = earlier visits of item j to worker q (visit_count, p*n
 * entries, in/out, may carry over from an earlier call); stop once `max_updates`
 * updates were applied (checked after each visit).
 *
 * Whose turn it is: with slots = 0 a worker drawn uniformly among those with a non-empty
 * queue.  With slots > 0, time decides, as it does for workers running in parallel: every
 * worker serves `slots` items at once; a visit takes visit_cost plus one unit per rating
 * it updates (units of one update) and the item reaches its next queue hop_time after the
 * visit ends; a worker takes its items in the order they arrive, and the next visit is the
 * one that can start first (the earliest time at which some worker has a free slot and an
 * item that has arrived; the lower worker, then the lower item, on a tie).  Which ratings
 * receive how many of the budget's updates depends on this: under the uniform draw a long
 * visit costs a worker one turn like a short one. */
int orc_train_uniform(int64_t m, int64_t n, int64_t nnz, const int32_t *row, const int32_t *col,
                      const float *val, int32_t k, double lambda, double alpha, double beta,
                      double gamma, int32_t p, uint64_t seed, int64_t max_updates,
                      uint64_t sched_seed, int32_t *visit_count, double *W, double *H,
                      orc_stats *st, int32_t *trace, int64_t trace_cap, int64_t *trace_len,
                      int32_t balance, int32_t slots, double visit_cost, double hop_time)
{
    int rc = check_common(k, p, 0);
    if (rc) return rc;
    layout L;
    rc = layout_build(&L, m, n, nnz, row, col, val, p, seed);
    if (rc) return rc;
    if (st) memset(st, 0, sizeof(*st));
    queues Q;
    int64_t *nvisits = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (queues_init(&Q, p, n) || !nvisits) { queues_free(&Q); free(nvisits); layout_free(&L); return ORC_ENOMEM; }
    int64_t tlen = 0;
    uint64_t ctr = 0;
    int64_t applied = 0;
    if (max_updates > 0 && nnz > 0)
        for (int64_t j = 0; j < n; ++j) q_push(&Q, orc_owner0(seed, j, p), (int32_t)j);
    double *slot_free = slots > 0 ? (double *)calloc((size_t)p * (size_t)slots, sizeof(double)) : NULL;
    double *arrive = slots > 0 ? (double *)calloc((size_t)n + 1, sizeof(double)) : NULL;
    if (slots > 0 && (!slot_free || !arrive)) {
        free(slot_free); free(arrive); queues_free(&Q); free(nvisits); layout_free(&L); return ORC_ENOMEM;
    }
    while (applied < max_updates && Q.nne > 0) {
        int32_t q, j;
        if (slots <= 0) {
            q = Q.ne[orc_splitmix64(sched_seed + ctr++) % (uint64_t)Q.nne];
            j = q_pop(&Q, q);
        } else {
            double best = 0.0;
            int32_t best_slot = 0, best_j = -1;
            q = -1;
            for (int32_t x = 0; x < Q.nne; ++x) {
                int32_t qq = Q.ne[x], fs = 0, first = Q.head[qq];
                for (int32_t s2 = 1; s2 < slots; ++s2)
                    if (slot_free[(int64_t)qq * slots + s2] < slot_free[(int64_t)qq * slots + fs]) fs = s2;
                for (int32_t jj = Q.next[first]; jj >= 0; jj = Q.next[jj])
                    if (arrive[jj] < arrive[first] || (arrive[jj] == arrive[first] && jj < first)) first = jj;
                double ready = slot_free[(int64_t)qq * slots + fs];
                if (arrive[first] > ready) ready = arrive[first];
                if (q < 0 || ready < best || (ready == best && qq < q)) {
                    best = ready; q = qq; best_slot = fs; best_j = first;
                }
            }
            j = best_j;
            q_remove(&Q, q, j);
            int64_t v0 = find_visit(&L, j, q);
            double end = best + visit_cost + (v0 >= 0 ? (double)(L.visits[v0].end - L.visits[v0].begin) : 0.0);
            slot_free[(int64_t)q * slots + best_slot] = end;
            arrive[j] = end + hop_time;
        }
        int64_t vi = find_visit(&L, j, q);
        if (vi >= 0) {
            int32_t *t = &visit_count[(int64_t)q * n + j];
            apply_visit(&L, &L.visits[vi], k, W, H, lambda, orc_step(alpha, beta, gamma, (double)*t), 1, st);
            trace_put(trace, trace_cap, &tlen, q, j, *t, nvisits[j]++);
            applied += L.visits[vi].end - L.visits[vi].begin;
            (*t)++;
        }
        int32_t dst = (int32_t)(orc_splitmix64(sched_seed + ctr++) % (uint64_t)p);
        if (balance) {
            int32_t d2 = (int32_t)(orc_splitmix64(sched_seed + ctr++) % (uint64_t)p);
            dst = orc_balanced_pick(dst, q_len(&Q, Q.next, dst), d2, q_len(&Q, Q.next, d2));
        }
        if (st) st->hops++;
        q_push(&Q, dst, j);
        if (st) { int64_t len = q_len(&Q, Q.next, dst); if (len > st->max_queue) st->max_queue = len; }
    }
    queues_free(&Q);
    free(nvisits);
    free(slot_free);
    free(arrive);
    layout_free(&L);
    if (trace_len) *trace_len = tlen;
    return ORC_OK;
}

/* ------------------------------------------------------------------------------- */
/* Algorithm 1 on POSIX threads: the CPU throughput baseline.                        */
/* ------------------------------------------------------------------------------- */
/* One thread per worker.  Each worker's queue is a mutex-protected FIFO ring with room
 * for every item.  A worker pops an item (waiting while its queue is empty), applies its
 * ratings of the item in ascending row order with t = its earlier visits of the item,
 * and pushes the item to a worker drawn uniformly from all p (splitmix64 of a per-worker
 * counter).  Every item starts in the queue of owner0(j).  The run stops once at least
 * max_updates updates were applied (checked after each visit); items still queued stay
 * there.  Ownership holds by construction: an item is in one queue or held by one
 * worker, and a worker touches only its own rows.  With one worker the order is the ring
 * order, so the result is that of orc_train_ring bit for bit. */
typedef struct {
    pthread_mutex_t mu;
    int32_t *buf;
    int64_t head, size, cap;
} tqueue;

typedef struct {
    const layout *L;
    int32_t k, p;
    double lambda, alpha, beta, gamma;
    double *W, *H;
    tqueue *Q;
    int64_t *vmap;           /* p x n: visit index of (q, j), or -1 */
    int32_t *visit_count;    /* p x n: earlier visits of (q, j) */
    int64_t max_updates;
    uint64_t sched_seed;
    int64_t applied;         /* updates applied (atomic) */
    int32_t stop;            /* atomic */
    int64_t *hops;           /* per worker */
} tshared;

typedef struct {
    tshared *S;
    int32_t q;
} targ;

static void *worker_main(void *vp)
{
    targ *A = (targ *)vp;
    tshared *S = A->S;
    const int32_t q = A->q;
    const int64_t n = S->L->n;
    uint64_t ctr = 0;
    while (!__atomic_load_n(&S->stop, __ATOMIC_ACQUIRE)) {
        tqueue *mine = &S->Q[q];
        int32_t j = -1;
        pthread_mutex_lock(&mine->mu);
        if (mine->size > 0) {
            j = mine->buf[mine->head];
            mine->head = (mine->head + 1) % mine->cap;
            mine->size--;
        }
        pthread_mutex_unlock(&mine->mu);
        if (j < 0) { sched_yield(); continue; }
        int64_t vi = S->vmap[(int64_t)q * n + j];
        if (vi >= 0) {
            int32_t *t = &S->visit_count[(int64_t)q * n + j];
            const visit *V = &S->L->visits[vi];
            apply_visit(S->L, V, S->k, S->W, S->H, S->lambda, orc_step(S->alpha, S->beta, S->gamma, (double)*t),
                        1, NULL);
            (*t)++;
            int64_t done = __atomic_add_fetch(&S->applied, V->end - V->begin, __ATOMIC_ACQ_REL);
            if (done >= S->max_updates) __atomic_store_n(&S->stop, 1, __ATOMIC_RELEASE);
        }
        int32_t dst = (int32_t)(orc_splitmix64(S->sched_seed ^ ((uint64_t)q << 40) ^ ctr++) % (uint64_t)S->p);
        tqueue *to = &S->Q[dst];
        pthread_mutex_lock(&to->mu);
        to->buf[(to->head + to->size) % to->cap] = j;
        to->size++;
        pthread_mutex_unlock(&to->mu);
        S->hops[q]++;
    }
    return NULL;
}

int orc_train_threaded(int64_t m, int64_t n, int64_t nnz, const int32_t *row, const int32_t *col,
                       const float *val, int32_t k, double lambda, double alpha, double beta,
                       double gamma, int32_t p, uint64_t seed, int64_t max_updates, uint64_t sched_seed,
                       double *W, double *H, orc_stats *st, double *seconds)
{
    int rc = check_common(k, p, 0);
    if (rc) return rc;
    layout L;
    rc = layout_build(&L, m, n, nnz, row, col, val, p, seed);
    if (rc) return rc;
    if (st) memset(st, 0, sizeof(*st));
    tshared S;
    memset(&S, 0, sizeof(S));
    S.L = &L; S.k = k; S.p = p; S.lambda = lambda; S.alpha = alpha; S.beta = beta; S.gamma = gamma;
    S.W = W; S.H = H; S.max_updates = max_updates; S.sched_seed = sched_seed;
    S.Q = (tqueue *)calloc((size_t)p, sizeof(tqueue));
    S.vmap = (int64_t *)malloc(sizeof(int64_t) * (size_t)p * (size_t)(n > 0 ? n : 1));
    S.visit_count = (int32_t *)calloc((size_t)p * (size_t)(n > 0 ? n : 1), sizeof(int32_t));
    S.hops = (int64_t *)calloc((size_t)p, sizeof(int64_t));
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)p);
    targ *args = (targ *)malloc(sizeof(targ) * (size_t)p);
    int ok = S.Q && S.vmap && S.visit_count && S.hops && th && args;
    for (int32_t q = 0; ok && q < p; ++q) {
        S.Q[q].buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        S.Q[q].cap = n > 0 ? n : 1;
        if (!S.Q[q].buf) ok = 0;
        else pthread_mutex_init(&S.Q[q].mu, NULL);
    }
    if (!ok) {
        rc = ORC_ENOMEM;
        goto out;
    }
    for (int64_t x = 0; x < (int64_t)p * n; ++x) S.vmap[x] = -1;
    for (int64_t v = 0; v < L.nvisit; ++v) S.vmap[(int64_t)L.visits[v].q * n + L.visits[v].j] = v;
    if (max_updates > 0 && nnz > 0)
        for (int64_t j = 0; j < n; ++j) {
            tqueue *to = &S.Q[orc_owner0(seed, j, p)];
            to->buf[(to->head + to->size) % to->cap] = (int32_t)j;
            to->size++;
        }
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    if (max_updates > 0 && nnz > 0) {
        int32_t started = 0;
        for (int32_t q = 0; q < p; ++q) {
            args[q].S = &S;
            args[q].q = q;
            if (pthread_create(&th[q], NULL, worker_main, &args[q]) != 0) {
                __atomic_store_n(&S.stop, 1, __ATOMIC_RELEASE);
                rc = ORC_ENOMEM;
                break;
            }
            started++;
        }
        for (int32_t q = 0; q < started; ++q) pthread_join(th[q], NULL);
    }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    if (seconds) *seconds = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
    if (st) {
        st->updates = S.applied;
        for (int32_t q = 0; q < p; ++q) st->hops += S.hops[q];
    }
out:
    if (S.Q)
        for (int32_t q = 0; q < p; ++q)
            if (S.Q[q].buf) { free(S.Q[q].buf); pthread_mutex_destroy(&S.Q[q].mu); }
    free(S.Q); free(S.vmap); free(S.visit_count); free(S.hops); free(th); free(args);
    layout_free(&L);
    return rc;
}

/* Re-execute recorded visits.  Record x says: worker tq[x] applied its ratings of item
 * tj[x] with step index tt[x], as the tseq[x]-th visit of that item.  Records of one
 * worker are given in that worker's execution order.  A record runs once every earlier
 * record of its worker has run and the item has completed tseq[x] visits. */
int orc_replay_loss(int64_t m, int64_t n, int64_t nnz, const int32_t *row, const int32_t *col,
                    const float *val, int32_t k, double lambda, double alpha, double beta,
                    double gamma, int32_t p, uint64_t seed, int64_t nrec, const int32_t *tq,
                    const int32_t *tj, const int32_t *tt, const int32_t *tseq, double *W, double *H,
                    orc_stats *st, int32_t loss)
{
    int rc = check_common(k, p, 0);
    if (rc) return rc;
    if (loss != 0 && loss != 1) return ORC_EINVAL;
    layout L;
    rc = layout_build(&L, m, n, nnz, row, col, val, p, seed);
    if (rc) return rc;
    L.loss = loss;
    if (st) memset(st, 0, sizeof(*st));
    int64_t *wcount = (int64_t *)calloc((size_t)p + 1, sizeof(int64_t));
    int64_t *wptr = (int64_t *)calloc((size_t)p + 1, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nrec + 1));
    int64_t *fill = (int64_t *)calloc((size_t)p + 1, sizeof(int64_t));
    int64_t *ndone = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!wcount || !wptr || !order || !fill || !ndone) { rc = ORC_ENOMEM; goto out; }
    for (int64_t x = 0; x < nrec; ++x) {
        if (tq[x] < 0 || tq[x] >= p || tj[x] < 0 || tj[x] >= n) { rc = ORC_EINVAL; goto out; }
        wcount[tq[x] + 1]++;
    }
    for (int32_t q = 0; q < p; ++q) wcount[q + 1] += wcount[q];
    for (int64_t x = 0; x < nrec; ++x) order[wcount[tq[x]] + fill[tq[x]]++] = x;
    for (int32_t q = 0; q < p; ++q) wptr[q] = wcount[q];
    int64_t remaining = nrec;
    while (remaining > 0) {
        int64_t progressed = 0;
        for (int32_t q = 0; q < p; ++q) {
            while (wptr[q] < wcount[q + 1]) {
                int64_t x = order[wptr[q]];
                if (ndone[tj[x]] != tseq[x]) break;
                int64_t vi = find_visit(&L, tj[x], q);
                if (vi < 0) { rc = ORC_EINVAL; goto out; }
                apply_visit(&L, &L.visits[vi], k, W, H, lambda, orc_step(alpha, beta, gamma, (double)tt[x]), 1, st);
                ndone[tj[x]]++;
                wptr[q]++;
                progressed++;
            }
        }
        if (!progressed) { rc = ORC_EDEADLOCK; goto out; }
        remaining -= progressed;
    }
out:
    free(wcount); free(wptr); free(order); free(fill); free(ndone);
    layout_free(&L);
    return rc;
}

int orc_replay(int64_t m, int64_t n, int64_t nnz, const int32_t *row, const int32_t *col,
               const float *val, int32_t k, double lambda, double alpha, double beta,
               double gamma, int32_t p, uint64_t seed, int64_t nrec, const int32_t *tq,
               const int32_t *tj, const int32_t *tt, const int32_t *tseq, double *W, double *H,
               orc_stats *st)
{
    return orc_replay_loss(m, n, nnz, row, col, val, k, lambda, alpha, beta, gamma, p, seed, nrec, tq, tj, tt,
                           tseq, W, H, st, 0);
}

/* ------------------------------------------------------------------------------- */
/* Evaluation: FP64 dot products, Neumaier-compensated sums.                        */
/* ------------------------------------------------------------------------------- */
static void neumaier_add(double *sum, double *comp, double x)
{
    double t = *sum + x;
    if (fabs(*sum) >= fabs(x)) *comp += (*sum - t) + x;
    else *comp += (x - t) + *sum;
    *sum = t;
}

static double dot(const double *a, const double *b, int32_t k)
{
    double d = 0.0;
    for (int32_t l = 0; l < k; ++l) d += a[l] * b[l];
    return d;
}

/* sqrt( sum over test ratings of (A_ij - <w_i, h_j>)^2 / |test| ); NaN for an empty set. */
int orc_rmse(int64_t m, int64_t n, int64_t nnz, const int32_t *row, const int32_t *col,
             const float *val, int32_t k, const double *W, const double *H, double *out)
{
    if (k <= 0) return ORC_EINVAL;
    double sum = 0.0, comp = 0.0;
    for (int64_t e = 0; e < nnz; ++e) {
        if (row[e] < 0 || row[e] >= m || col[e] < 0 || col[e] >= n) return ORC_EINVAL;
        double err = (double)val[e] - dot(W + (int64_t)row[e] * k, H + (int64_t)col[e] * k, k);
        neumaier_add(&sum, &comp, err * err);
    }
    *out = nnz > 0 ? sqrt((sum + comp) / (double)nnz) : NAN;
    return ORC_OK;
}

/* J(W,H) = sum over ratings of [ loss(A_ij, <w_i,h_j>) + lambda/2 (|w_i|^2 + |h_j|^2) ];
 * with the square loss, 1/2 sum of [ (A_ij - <w_i,h_j>)^2 + lambda (|w_i|^2 + |h_j|^2) ]. */
int orc_objective_loss(int64_t m, int64_t n, int64_t nnz, const int32_t *row, const int32_t *col,
                       const float *val, int32_t k, double lambda, const double *W, const double *H,
                       double *out, int32_t loss)
{
    if (k <= 0 || (loss != 0 && loss != 1)) return ORC_EINVAL;
    double sum = 0.0, comp = 0.0;
    for (int64_t e = 0; e < nnz; ++e) {
        if (row[e] < 0 || row[e] >= m || col[e] < 0 || col[e] >= n) return ORC_EINVAL;
        const double *w = W + (int64_t)row[e] * k, *h = H + (int64_t)col[e] * k;
        double f = orc_loss((double)val[e], dot(w, h, k), loss);
        neumaier_add(&sum, &comp, f + 0.5 * lambda * (dot(w, w, k) + dot(h, h, k)));
    }
    *out = sum + comp;
    return ORC_OK;
}

int orc_objective(int64_t m, int64_t n, int64_t nnz, const int32_t *row, const int32_t *col,
                  const float *val, int32_t k, double lambda, const double *W, const double *H,
                  double *out)
{
    return orc_objective_loss(m, n, nnz, row, col, val, k, lambda, W, H, out, 0);
}
