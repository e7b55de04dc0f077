// Serving: resident sets, kernel rows of query batches, and the
// continuous-batching server.
//
// A resident set (e.g. an SVM's support vectors) is partitioned and sorted
// once per position set; its run entries and per-bucket group tables stay on
// the device together with K(sv, sv).  A query batch is extracted and
// partitioned like a Gram job (for its own K(q, q)), then every query g-mer
// is looked up in the resident tables.
//
// The server admits submitted queries into device batches whenever one of
// its workers is free: each worker owns a context (arena), a HIP stream and
// staging buffers, so up to n_streams batches are in flight at once (the
// kernels of batches large enough for the dense join in admission order, one
// batch after another, while the other workers prepare the next batches and
// copy results back) and requests arriving meanwhile wait only for the next
// free worker.  The
// batch size is bounded by max_batch and by the worker's share of the HBM
// budget.  Every query's result depends only on the query (integer counts
// exact, per-query fixed-order sums), so it is the same alone and in any mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>

#include "plan.h"

namespace gk {
void clear_error();
hipError_t init_kernel_attributes(size_t acc_lds);
}
using namespace gk;

struct gakco_resident {
    int device = 0;
    int n_sv = 0, sigma = 0, g = 0, k = 0, M = 0, b = 0, sb = 0;
    uint32_t maxng = 0;
    size_t bytes = 0;
    char *mem = nullptr;
    const void *rm = nullptr;   // device ResMask array
    const int32_t *lev_first = nullptr, *lev_count = nullptr;
    const int64_t *coef = nullptr, *hco = nullptr;
    const int64_t *Kd = nullptr;
    const double *alpha = nullptr;
    double bias = 0.0;
    // the top level joined on the matrix cores (dense_level < 0: none):
    // count rows of nsv_pad sequences x dense_stride columns (128-row tiles
    // of 8 KB column blocks), one 2^dense_w-column segment per position set
    // of the level (descriptors at dense_rm)
    int dense_level = -1, dense_w = 0, dense_nset = 0;
    size_t dense_stride = 0;
    const void *dense_rm = nullptr;
    int8_t *D = nullptr;
};

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Grow-only device scratch owned by a context for the rows path.
struct RowsScratch {
    char *p = nullptr;
    size_t cap = 0;
};
static std::mutex g_scratch_mu;
static std::map<const gakco_ctx *, RowsScratch> g_scratch;

static gakco_status rows_scratch(gakco_ctx *ctx, size_t bytes, char **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    RowsScratch &s = g_scratch[ctx];
    if (bytes > s.cap) {
        // the callers synchronise their stream before returning, so the old
        // buffer is idle; growth is geometric so that it stays rare
        if (s.p) {
            GK_HIP(hipFree(s.p));
            s.p = nullptr;
            s.cap = 0;
        }
        bytes = std::max(bytes, s.cap + s.cap / 2);
        GK_HIP(hipMalloc(&s.p, bytes));
        s.cap = bytes;
    }
    *out = s.p;
    return GAKCO_OK;
}

void rows_scratch_release(const gakco_ctx *ctx)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(ctx);
    if (it != g_scratch.end()) {
        if (it->second.p) (void)hipFree(it->second.p);
        g_scratch.erase(it);
    }
}

// The serving counters are uint32 summed over all position sets of a level:
// a query's own diagonal (at most C(g,m) * ng_q^2), its row entries (at most
// C(g,m) * ng_q * ng_sv) and the resident diagonal (C(g,m) * ng_sv^2).
static bool level_sum_fits(const gakco_resident *R, uint64_t ng_a, uint64_t ng_b)
{
    for (int m = 0; m <= R->M; ++m)
        if ((double)binom64(R->g, m) * (double)ng_a * (double)ng_b > 4294967295.0) return false;
    return true;
}

static gakco_status check_query_bounds(const gakco_resident *R, uint64_t ng_q)
{
    if (!level_sum_fits(R, ng_q, ng_q) || !level_sum_fits(R, ng_q, R->maxng)) {
        set_error("a query with %llu g-mers exceeds the 32-bit serving counters (C(g,m) * g-mers^2 and C(g,m) * "
                  "query g-mers * resident g-mers must stay below 2^32)", (unsigned long long)ng_q);
        return GAKCO_EUNSUPPORTED;
    }
    return GAKCO_OK;
}

// Rows of n_q queries (device symbols and lengths; host lengths when known)
// against a resident set, on stream st; synchronises st before returning.
// K_rows has row stride ldk (0: n_sv).
namespace gk {
hipError_t init_rows_attributes(size_t lds);
}

gakco_status gk::rows_run(gakco_ctx *ctx, const gakco_resident *R, const int8_t *q_seqs, const int32_t *q_lens,
                          const int32_t *q_lens_host, int32_t n_q, double *K_rows, int64_t ldk, int64_t *Nm_rows,
                          double *decision, hipStream_t st, const RowsGate *gate)
{
    if (!R || n_q < 1 || !q_seqs || !q_lens) { set_error("bad arguments"); return GAKCO_EINVAL; }
    Plan p;
    p.jobs.resize(1);
    JobPlan &jp = p.jobs[0];
    jp.seqs = q_seqs; jp.lens_dev = q_lens; jp.N = n_q; jp.sigma = R->sigma; jp.g = R->g; jp.k = R->k;
    jp.want_kernel = false;
    if (q_lens_host) jp.lens.assign(q_lens_host, q_lens_host + n_q);
    else GK_TRY(fetch_lens(jp, st));
    GK_TRY(plan_shape(ctx, jp, nullptr, 0));
    GK_TRY(check_query_bounds(R, jp.maxng));
    // The queries' diagonal counters come from per-query LDS histograms when
    // a query's g-mers fit a table of at most 4096 slots (twice as many as
    // g-mers) and no reduced g-mer is 64 bits wide; the plan then only
    // validates and extracts.  Otherwise the bucket sort of the queries'
    // g-mers sums them.
    int qd_bits = 8;
    while ((1u << qd_bits) < 2u * jp.maxng) ++qd_bits;
    const bool qdiag = qd_bits <= 12 && R->g * R->b < 64;
    if (qdiag) jp.masks.clear();
    const int M1 = R->M + 1;
    Layout l;
    const size_t o_diag = l.take((size_t)M1 * n_q * 4);
    const size_t o_kq = l.take((size_t)n_q * 8);
    const size_t o_C = l.take((size_t)M1 * n_q * R->n_sv * 4);
    const size_t o_part = l.take(rows_partial_count(n_q, R->n_sv) * 8);
    // a batch large enough joins the dense top level on the matrix cores:
    // the queries' count rows (padded to the product's query tile) and their
    // clipping flags
    const bool dense = R->D && n_q >= ctx->rows_dense_min_q;
    const size_t tq = (size_t)rows_gemm_tile_q(n_q);
    const size_t o_Q = dense ? l.take(((size_t)n_q + tq - 1) / tq * tq * R->dense_stride) : 0;
    const size_t o_qf = dense ? l.take((size_t)n_q * 4) : 0;
    char *scr = nullptr;
    GK_TRY(rows_scratch(ctx, l.size, &scr));
    uint32_t *diag = reinterpret_cast<uint32_t *>(scr + o_diag);
    for (int m = 0; m < M1; ++m) jp.ext_diag.push_back(diag + (size_t)m * n_q);
    GK_TRY(plan_layout(ctx, p));
    GK_TRY(plan_bind(ctx, p, st));
    GK_TRY(plan_upload(p, st));
    if (gate) gate->enter(gate->arg, st);
    GK_HIP(launch_fill_u32(diag, (size_t)M1 * n_q, 0u, st));
    GK_TRY(plan_launch(ctx, p, st));
    int nitems = 0;
    for (int m = 0; m <= R->M; ++m) nitems += (int)binom64(R->g, m);
    if (qdiag) GK_PHASE(PH_ROWS_QDIAG, launch_query_diag(jp.dev.key, jp.dev.gstart, n_q, nitems, qd_bits, R->rm, diag, st));
    int64_t *Kq = reinterpret_cast<int64_t *>(scr + o_kq);
    uint32_t *C = reinterpret_cast<uint32_t *>(scr + o_C);
    GK_PHASE(PH_ROWS_KDIAG, launch_kdiag_counts(diag, n_q, R->M, R->coef, R->hco, Kq, st));
    // grid: (level, position set) x query x SV slab, so that even one query
    // spreads over the whole device; one set per block measured faster at
    // every batch size (1..160 queries) than chunks of several sets, whose
    // partial rows are fewer but whose blocks run longer.  Slabs of about
    // half the SVs (4096..16384 of them: a 16..64 KB LDS row): every slab
    // repeats the group lookups of its query's g-mers and cuts each group at
    // its edges, so fewer slabs save lookups until the LDS row limits the
    // blocks per CU; for 20000 SVs two slabs measured 30.4 ms per 256-query
    // batch, three 32.3, four 35.7, one 80.4
    const size_t half = (R->n_sv + 1) / 2;
    int slab = (int)std::min<size_t>((size_t)R->n_sv, std::min<size_t>(16384, std::max<size_t>(4096, half)));
    if (ctx->rows_slabs > 0) slab = (int)std::max<size_t>(64, ((size_t)R->n_sv + ctx->rows_slabs - 1) / ctx->rows_slabs);
    if ((size_t)slab * 4 > ctx->lds_max) { set_error("SV slab of %d exceeds the LDS", slab); return GAKCO_EUNSUPPORTED; }
    if ((size_t)slab * 4 > 32768) GK_HIP(init_rows_attributes(ctx->lds_max));  // rows beyond the default LDS limit
    const int mchunk = 1;
    GK_HIP(launch_fill_u32(C, (size_t)M1 * n_q * R->n_sv, 0u, st));
    int8_t *Q = dense ? reinterpret_cast<int8_t *>(scr + o_Q) : nullptr;
    uint32_t *qflag = dense ? reinterpret_cast<uint32_t *>(scr + o_qf) : nullptr;
    if (dense) {
        GK_HIP(launch_fill_u32(qflag, (size_t)n_q, 0u, st));
        GK_PHASE(PH_ROWS_COUNT, launch_count_rows(jp.dev.key, jp.dev.gstart, n_q, R->dense_rm, R->dense_nset, R->dense_w, Q,
                                                  R->dense_stride, qflag, st));
    }
    unsigned long long *upd = ctx->prof_on && ctx->prof_stat ? ctx->prof_stat + kProfRowsFirst : nullptr;
    GK_PHASE(PH_ROWS, launch_rows(jp.dev.key, jp.dev.gstart, n_q, R->M, R->n_sv, slab, mchunk, nitems, R->rm, R->lev_first,
                                  R->lev_count, C, upd, dense ? R->dense_level : -1, qflag, st));
    if (dense) {
        // column splits chosen by the launcher (whole rounds of resident blocks)
        GK_PHASE(PH_ROWS_GEMM, launch_rows_gemm(Q, R->D, R->dense_stride, n_q, R->n_sv, 0, qflag,
                                                C + (size_t)R->dense_level * n_q * R->n_sv, st));
    }
    GK_PHASE(PH_ROWS_FINALIZE, launch_rows_finalize(C, n_q, R->n_sv, R->M, R->coef, R->hco, R->Kd, Kq, R->alpha, R->bias, K_rows,
                                           ldk, Nm_rows, decision,
                                                           reinterpret_cast<double *>(scr + o_part), st));
    if (gate) gate->leave(gate->arg, st);
    return plan_check_errors(ctx, p, st);
}

// ------------------------------------------------------------------ server --
struct SrvRequest {
    uint64_t tag;
    std::vector<int8_t> q;
    double t_submit;
};

struct SrvResult {
    gakco_result r;
    std::vector<double> row;
};

struct SrvWorker {
    gakco_ctx *ctx = nullptr;
    hipStream_t st = nullptr;
    int8_t *h_q = nullptr;     // pinned staging
    int32_t *h_lens = nullptr;
    size_t h_cap = 0, h_lcap = 0;
    char *d_buf = nullptr;     // device inputs and outputs
    size_t d_cap = 0;
    double *h_out = nullptr;   // pinned K rows + decisions
    size_t h_ocap = 0;
    hipEvent_t ev = nullptr;   // recorded once a batch's kernels are queued
    std::thread th;
};

struct gakco_server {
    const gakco_resident *res = nullptr;
    int device = 0, max_batch = 1, n_streams = 1;
    size_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_req, cv_done;
    std::deque<SrvRequest> queue;
    std::deque<SrvResult> done;
    std::vector<SrvResult> polled;  // results returned by the last poll (their rows stay valid)
    std::vector<SrvWorker> workers;
    bool stop = false;
    int running = 0;  // batches taken and not yet finished (under mu)
    // Batches that take the dense join take tickets in admission order; a
    // ticketed batch's kernels wait for the previous ticket's
    // (hipStreamWaitEvent on its worker's event), so such batches run on
    // the device one after another, each at full speed, while the workers'
    // host preparation and result copies overlap them.
    uint64_t next_ticket = 0;  // under mu
    std::mutex order_mu;
    std::condition_variable order_cv;
    uint64_t queued_ticket = 0;  // last ticket whose kernels are queued
    hipEvent_t queued_ev = nullptr;  // recorded after them (nullptr: none to wait for)
};

// One batch's place in the device order (ticket 0: unordered).
struct BatchTurn {
    gakco_server *S;
    SrvWorker *W;
    uint64_t ticket;
    bool entered = false, left = false;
    void wait_turn()
    {
        std::unique_lock<std::mutex> lk(S->order_mu);
        S->order_cv.wait(lk, [&] { return S->queued_ticket + 1 == ticket; });
    }
    static void enter(void *a, hipStream_t st)
    {
        auto *t = static_cast<BatchTurn *>(a);
        t->wait_turn();
        hipEvent_t e;
        {
            std::lock_guard<std::mutex> lk(t->S->order_mu);
            e = t->S->queued_ev;
        }
        if (e) (void)hipStreamWaitEvent(st, e, 0);
        t->entered = true;
    }
    static void leave(void *a, hipStream_t st)
    {
        auto *t = static_cast<BatchTurn *>(a);
        if (t->left) return;
        if (!t->entered) t->wait_turn();  // an early failure still passes its turn on
        const bool rec = t->entered && hipEventRecord(t->W->ev, st) == hipSuccess;
        {
            std::lock_guard<std::mutex> lk(t->S->order_mu);
            if (rec) t->S->queued_ev = t->W->ev;
            t->S->queued_ticket = t->ticket;
        }
        t->S->order_cv.notify_all();
        t->left = true;
    }
    ~BatchTurn()
    {
        if (ticket) leave(this, W->st);
    }
};

// Worker buffers grow geometrically (and are sized by a warm-up batch when
// the server starts), so that steady-state batches never reallocate.
static gakco_status grow_pinned(void **p, size_t *cap, size_t bytes)
{
    if (bytes <= *cap) return GAKCO_OK;
    bytes = std::max(bytes, *cap + *cap / 2);
    if (*p) GK_HIP(hipHostFree(*p));
    *p = nullptr;
    GK_HIP(hipHostMalloc(p, bytes, hipHostMallocDefault));
    *cap = bytes;
    return GAKCO_OK;
}

static gakco_status grow_device(char **p, size_t *cap, size_t bytes)
{
    if (bytes <= *cap) return GAKCO_OK;
    bytes = std::max(bytes, *cap + *cap / 2);
    if (*p) GK_HIP(hipFree(*p));
    *p = nullptr;
    GK_HIP(hipMalloc(p, bytes));
    *cap = bytes;
    return GAKCO_OK;
}

// Device bytes one query needs in a batch: its C_m rows, K row and decision,
// and its share of the partition buffers (36 bytes per g-mer and position
// set, the pool of one chunk).
static size_t query_bytes(const gakco_resident *R, size_t len, size_t npos)
{
    const size_t ng = len >= (size_t)R->g ? len - R->g + 1 : 0;
    return (size_t)(R->M + 1) * R->n_sv * 4 + (size_t)R->n_sv * 8 + 64 + len + ng * 48 * std::min<size_t>(npos, 64);
}

static gakco_status run_batch(gakco_server *S, SrvWorker &W, std::vector<SrvRequest> &batch, std::vector<SrvResult> &out,
                              uint64_t ticket)
{
    BatchTurn turn{S, &W, ticket};
    const RowsGate gate{&BatchTurn::enter, &BatchTurn::leave, &turn};
    const gakco_resident *R = S->res;
    const int nq = (int)batch.size();
    size_t tot = 0;
    for (auto &r : batch) tot += r.q.size();
    GK_TRY(grow_pinned(reinterpret_cast<void **>(&W.h_q), &W.h_cap, std::max<size_t>(tot, 1)));
    GK_TRY(grow_pinned(reinterpret_cast<void **>(&W.h_lens), &W.h_lcap, (size_t)nq * 4));
    size_t off = 0;
    for (int i = 0; i < nq; ++i) {
        memcpy(W.h_q + off, batch[(size_t)i].q.data(), batch[(size_t)i].q.size());
        W.h_lens[i] = (int32_t)batch[(size_t)i].q.size();
        off += batch[(size_t)i].q.size();
    }
    Layout l;
    const size_t o_q = l.take(std::max<size_t>(tot, 1));
    const size_t o_l = l.take((size_t)nq * 4);
    const size_t o_K = l.take((size_t)nq * R->n_sv * 8);
    const size_t o_d = l.take((size_t)nq * 8);
    GK_TRY(grow_device(&W.d_buf, &W.d_cap, l.size));
    GK_TRY(grow_pinned(reinterpret_cast<void **>(&W.h_out), &W.h_ocap, (size_t)nq * (R->n_sv + 1) * 8));
    GK_HIP(hipMemcpyAsync(W.d_buf + o_q, W.h_q, std::max<size_t>(tot, 1), hipMemcpyHostToDevice, W.st));
    GK_HIP(hipMemcpyAsync(W.d_buf + o_l, W.h_lens, (size_t)nq * 4, hipMemcpyHostToDevice, W.st));
    double *dK = reinterpret_cast<double *>(W.d_buf + o_K);
    double *dd = reinterpret_cast<double *>(W.d_buf + o_d);
    const gakco_status s = rows_run(W.ctx, R, reinterpret_cast<int8_t *>(W.d_buf + o_q),
                                    reinterpret_cast<int32_t *>(W.d_buf + o_l), W.h_lens, nq, dK, 0, nullptr, dd, W.st,
                                    ticket ? &gate : nullptr);
    if (s != GAKCO_OK && s != GAKCO_ERANGE) return s;
    GK_HIP(hipMemcpyAsync(W.h_out, dK, (size_t)nq * R->n_sv * 8, hipMemcpyDeviceToHost, W.st));
    GK_HIP(hipMemcpyAsync(W.h_out + (size_t)nq * R->n_sv, dd, (size_t)nq * 8, hipMemcpyDeviceToHost, W.st));
    GK_HIP(hipStreamSynchronize(W.st));
    out.resize((size_t)nq);
    for (int i = 0; i < nq; ++i) {
        SrvResult &r = out[(size_t)i];
        r.row.assign(W.h_out + (size_t)i * R->n_sv, W.h_out + (size_t)(i + 1) * R->n_sv);
        r.r.decision = W.h_out[(size_t)nq * R->n_sv + i];
        r.r.status = s;  // a batch with a bad symbol is reported on all its queries
    }
    return GAKCO_OK;
}

// Sizes a worker's context arena, rows scratch and staging buffers with one
// batch of as many 1024-symbol queries (pseudo-random codes) as max_batch and
// the worker's budget allow, so that batches of queries up to that length
// never reallocate (a reallocation frees device memory, which waits for the
// whole device and so for the other workers' batches).  Best effort: a
// failure leaves the buffers to grow on demand.
static void warm_worker(gakco_server *S, SrvWorker &W, size_t wbudget, size_t npos)
{
    const gakco_resident *R = S->res;
    const size_t len = 1024;
    const size_t per = query_bytes(R, len, npos);
    const int n = (int)std::min<size_t>((size_t)S->max_batch, per ? wbudget / per : 0);
    if (n < 1) return;
    std::vector<SrvRequest> batch((size_t)n);
    uint32_t x = 0x2545F491u;
    for (auto &r : batch) {
        r.q.resize(len);
        for (auto &c : r.q) {
            x = x * 1664525u + 1013904223u;  // a 32-bit LCG (Numerical Recipes constants)
            c = (int8_t)((x >> 16) % (uint32_t)R->sigma);
        }
    }
    std::vector<SrvResult> out;
    (void)run_batch(S, W, batch, out, 0);
    clear_error();
}

static void worker_loop(gakco_server *S, int wi)
{
    SrvWorker &W = S->workers[(size_t)wi];
    (void)hipSetDevice(S->device);
    const gakco_resident *R = S->res;
    const size_t wbudget = S->budget / (size_t)S->n_streams;
    size_t npos = 0;
    for (int m = 0; m <= R->M; ++m) npos += (size_t)binom64(R->g, m);
    while (true) {
        std::vector<SrvRequest> batch;
        std::vector<SrvResult> rejected;
        uint64_t ticket = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_req.wait(lk, [&] { return S->stop || !S->queue.empty(); });
            if (S->queue.empty()) return;  // stopping and nothing queued
            size_t used = 0;
            while (!S->queue.empty() && (int)batch.size() < S->max_batch) {
                const size_t need = query_bytes(R, S->queue.front().q.size(), npos);
                if (need > wbudget) {  // can never be admitted
                    SrvResult rr{};
                    rr.r.tag = S->queue.front().tag;
                    rr.r.status = GAKCO_EBUDGET;
                    rr.r.t_submit = S->queue.front().t_submit;
                    rr.r.t_start = rr.r.t_done = now_s();
                    rejected.push_back(std::move(rr));
                    S->queue.pop_front();
                    continue;
                }
                if (used + need > wbudget) break;  // admitted with the next free worker
                used += need;
                batch.push_back(std::move(S->queue.front()));
                S->queue.pop_front();
            }
            // batches large enough for the dense join fill the device alone
            // and go in order; smaller ones gain from running side by side
            if (!batch.empty() && R->D && (int)batch.size() >= W.ctx->rows_dense_min_q) ticket = ++S->next_ticket;
            if (!batch.empty()) ++S->running;
        }
        std::vector<SrvResult> out;
        const double t0 = now_s();
        gakco_status s = batch.empty() ? GAKCO_OK : run_batch(S, W, batch, out, ticket);
        const double t1 = now_s();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (auto &rr : rejected) S->done.push_back(std::move(rr));
            for (size_t i = 0; i < batch.size(); ++i) {
                SrvResult rr = (s == GAKCO_OK) ? std::move(out[i]) : SrvResult{};
                rr.r.tag = batch[i].tag;
                if (s != GAKCO_OK) rr.r.status = s;
                rr.r.t_submit = batch[i].t_submit;
                rr.r.t_start = t0;
                rr.r.t_done = t1;
                rr.r.batch_size = (int32_t)batch.size();
                S->done.push_back(std::move(rr));
            }
            if (!batch.empty()) --S->running;
        }
        S->cv_done.notify_all();
        S->cv_req.notify_all();
    }
}

extern "C" {

gakco_status gakco_resident_create(gakco_ctx *ctx, const int8_t *seqs, const int32_t *lens, int32_t n_sv, int32_t sigma,
                                   int32_t g, int32_t k, const double *dual_coef_host, double bias, gakco_resident **out)
{
    clear_error();
    if (!ctx || !out) { set_error("ctx/out is NULL"); return GAKCO_EINVAL; }
    *out = nullptr;
    GK_HIP(hipSetDevice(ctx->device));
    hipStream_t st = nullptr;
    GK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    auto *R = new gakco_resident();
    auto fail = [&](gakco_status s) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
        gakco_resident_destroy(R);
        return s;
    };
    Plan p;
    p.jobs.resize(1);
    JobPlan &jp = p.jobs[0];
    jp.seqs = seqs; jp.lens_dev = lens; jp.N = n_sv; jp.sigma = sigma; jp.g = g; jp.k = k;
    jp.want_kernel = false;
    if (n_sv < 1 || !seqs || !lens) { set_error("bad arguments"); return fail(GAKCO_EINVAL); }
    gakco_status s = fetch_lens(jp, st);
    if (s == GAKCO_OK) s = plan_shape(ctx, jp, nullptr, 0);
    if (s != GAKCO_OK) return fail(s);
    R->device = ctx->device;
    R->n_sv = n_sv; R->sigma = sigma; R->g = g; R->k = k; R->M = jp.M; R->b = jp.b; R->sb = jp.sb;
    R->maxng = jp.maxng;
    if (!level_sum_fits(R, jp.maxng, jp.maxng)) {
        set_error("a resident sequence with %u g-mers exceeds the 32-bit diagonal counters (C(g,m) * g-mers^2 < 2^32)",
                  jp.maxng);
        return fail(GAKCO_EUNSUPPORTED);
    }
    R->bias = bias;
    const int M1 = jp.M + 1;
    const size_t nm = jp.masks.size();
    // one allocation: descriptors, tables per position set, counters
    Layout l;
    const size_t o_rm = l.take(res_mask_size() * nm);
    const size_t o_lf = l.take((size_t)M1 * 4), o_lc = l.take((size_t)M1 * 4);
    const size_t o_coef = l.take((size_t)M1 * M1 * 8), o_hco = l.take((size_t)M1 * 8);
    const size_t o_kd = l.take((size_t)n_sv * 8);
    const size_t o_al = dual_coef_host ? l.take((size_t)n_sv * 8) : 0;
    const size_t o_dg = l.take((size_t)M1 * n_sv * 4);
    std::vector<size_t> o_boff(nm), o_bgrp(nm), o_E(nm), o_gtab(nm);
    for (size_t i = 0; i < nm; ++i) {
        const size_t nb = (size_t)1 << jp.level_B[(size_t)jp.masks[i].level];
        o_boff[i] = l.take((nb + 1) * 4);
        o_bgrp[i] = l.take(nb * 4);
        o_E[i] = l.take((size_t)jp.T * 4);
        o_gtab[i] = l.take((size_t)jp.T * 16);
    }
    if (l.size > ctx->budget) {
        set_error("the resident tables need %.3f GB; the budget is %.3f GB", l.size / 1e9, ctx->budget / 1e9);
        return fail(GAKCO_EBUDGET);
    }
    if (hipMalloc(&R->mem, l.size) != hipSuccess) { set_error("hipMalloc of %zu bytes failed", l.size); return fail(GAKCO_EHIP); }
    R->bytes = l.size;
    char *mem = R->mem;
    uint32_t *diag = reinterpret_cast<uint32_t *>(mem + o_dg);
    for (size_t i = 0; i < nm; ++i) {
        jp.ext_boff.push_back(reinterpret_cast<uint32_t *>(mem + o_boff[i]));
        jp.ext_bgrp.push_back(reinterpret_cast<uint32_t *>(mem + o_bgrp[i]));
        jp.ext_E.push_back(reinterpret_cast<uint32_t *>(mem + o_E[i]));
        jp.ext_gtab.push_back(reinterpret_cast<uint4 *>(mem + o_gtab[i]));
    }
    for (int m = 0; m < M1; ++m) jp.ext_diag.push_back(diag + (size_t)m * n_sv);
    // host tables
    std::vector<char> h(o_dg, 0);
    std::vector<int32_t> lf((size_t)M1, 0), lc((size_t)M1, 0);
    for (size_t i = 0; i < nm; ++i) {
        const MaskDesc &md = jp.masks[i];
        const int m = md.level;
        if (!lc[(size_t)m]) lf[(size_t)m] = (int32_t)i;
        lc[(size_t)m] += 1;
        const int w = (g - m) * jp.b, B = jp.level_B[(size_t)m];
        res_mask_fill(h.data() + o_rm + res_mask_size() * i, md, w, B, w - B, jp.sb, jp.ext_boff[i], jp.ext_bgrp[i],
                      jp.ext_E[i], jp.ext_gtab[i]);
    }
    memcpy(h.data() + o_lf, lf.data(), (size_t)M1 * 4);
    memcpy(h.data() + o_lc, lc.data(), (size_t)M1 * 4);
    int64_t *coef = reinterpret_cast<int64_t *>(h.data() + o_coef);
    int64_t *hco = reinterpret_cast<int64_t *>(h.data() + o_hco);
    for (int m = 0; m < M1; ++m) {
        hco[m] = binom64(g - m, k);                                              // Eq. 6
        for (int q = 0; q < m; ++q) coef[(size_t)m * M1 + q] = binom64(g - q, m - q);  // Eq. 9
    }
    if (dual_coef_host) memcpy(h.data() + o_al, dual_coef_host, (size_t)n_sv * 8);
    if (hipMemcpyAsync(mem, h.data(), h.size(), hipMemcpyHostToDevice, st) != hipSuccess) {
        set_error("upload of the resident descriptors failed");
        return fail(GAKCO_EHIP);
    }
    R->rm = mem + o_rm;
    R->lev_first = reinterpret_cast<const int32_t *>(mem + o_lf);
    R->lev_count = reinterpret_cast<const int32_t *>(mem + o_lc);
    R->coef = reinterpret_cast<const int64_t *>(mem + o_coef);
    R->hco = reinterpret_cast<const int64_t *>(mem + o_hco);
    R->Kd = reinterpret_cast<const int64_t *>(mem + o_kd);
    R->alpha = dual_coef_host ? reinterpret_cast<const double *>(mem + o_al) : nullptr;
    if (launch_fill_u32(diag, (size_t)M1 * n_sv, 0u, st) != hipSuccess) { set_error("fill failed"); return fail(GAKCO_EHIP); }
    if ((s = plan_layout(ctx, p)) != GAKCO_OK) return fail(s);
    if ((s = plan_bind(ctx, p, st)) != GAKCO_OK) return fail(s);
    if ((s = plan_upload(p, st)) != GAKCO_OK) return fail(s);
    if ((s = plan_launch(ctx, p, st)) != GAKCO_OK) return fail(s);
    if (launch_kdiag_counts(diag, n_sv, jp.M, R->coef, R->hco, const_cast<int64_t *>(R->Kd), st) != hipSuccess) {
        set_error("self-kernel launch failed");
        return fail(GAKCO_EHIP);
    }
    // The top level on the matrix cores when its reduced g-mers index at
    // most 4096 values per position set and the set is large enough: the
    // resident count rows, kept unless some count exceeds 127.
    const int L = jp.M, wL = (g - L) * jp.b;
    uint32_t *dflag = nullptr;
    if (ctx->rows_dense && wL >= 6 && wL <= 12 && n_sv >= ctx->rows_dense_min_sv) {
        const int nset = (int)binom64(g, L);
        const size_t stride = (size_t)nset << wL;
        const size_t tile = (size_t)rows_gemm_tile_sv();
        const size_t nsv_pad = ((size_t)n_sv + tile - 1) / tile * tile;
        if (l.size + nsv_pad * stride <= ctx->budget && hipMalloc(&R->D, nsv_pad * stride) == hipSuccess &&
            hipMalloc(&dflag, (size_t)n_sv * 4) == hipSuccess) {
            R->dense_level = L;
            R->dense_w = wL;
            R->dense_nset = nset;
            R->dense_stride = stride;
            R->dense_rm = mem + o_rm + res_mask_size() * (size_t)lf[(size_t)L];
            if (launch_fill_u32(dflag, (size_t)n_sv, 0u, st) != hipSuccess ||
                launch_count_rows(jp.dev.key, jp.dev.gstart, n_sv, R->dense_rm, nset, wL, R->D, stride, dflag, st) !=
                    hipSuccess) {
                (void)hipFree(dflag);
                set_error("count-row launch failed");
                return fail(GAKCO_EHIP);
            }
        } else {
            (void)hipGetLastError();  // no room: the level stays on the sparse walk
            if (R->D) (void)hipFree(R->D);
            R->D = nullptr;
        }
    }
    if ((s = plan_check_errors(ctx, p, st)) != GAKCO_OK) {
        if (dflag) (void)hipFree(dflag);
        return fail(s);
    }
    if (dflag) {
        std::vector<uint32_t> fl((size_t)n_sv);
        const hipError_t e = hipMemcpy(fl.data(), dflag, (size_t)n_sv * 4, hipMemcpyDeviceToHost);
        (void)hipFree(dflag);
        if (e != hipSuccess) { set_error("count-row flags: %s", hipGetErrorString(e)); return fail(GAKCO_EHIP); }
        bool over = false;
        for (uint32_t f : fl) over |= f != 0;
        if (over) {  // a count above 127: the level stays on the sparse walk
            (void)hipFree(R->D);
            R->D = nullptr;
            R->dense_level = -1;
        }
    }
    if (R->D) R->bytes += ((size_t)n_sv + rows_gemm_tile_sv() - 1) / rows_gemm_tile_sv() * rows_gemm_tile_sv() * R->dense_stride;
    (void)hipStreamDestroy(st);
    *out = R;
    return GAKCO_OK;
}

void gakco_resident_destroy(gakco_resident *R)
{
    if (!R) return;
    if (R->mem || R->D) {
        (void)hipSetDevice(R->device);
        (void)hipDeviceSynchronize();
        if (R->mem) (void)hipFree(R->mem);
        if (R->D) (void)hipFree(R->D);
    }
    delete R;
}

gakco_status gakco_resident_info(const gakco_resident *R, int32_t *n_sv, int32_t *sigma, int32_t *g, int32_t *k,
                                 size_t *device_bytes)
{
    clear_error();
    if (!R) { set_error("resident is NULL"); return GAKCO_EINVAL; }
    if (n_sv) *n_sv = R->n_sv;
    if (sigma) *sigma = R->sigma;
    if (g) *g = R->g;
    if (k) *k = R->k;
    if (device_bytes) *device_bytes = R->bytes;
    return GAKCO_OK;
}

gakco_status gakco_rows(gakco_ctx *ctx, const gakco_resident *res, const int8_t *q_seqs, const int32_t *q_lens, int32_t n_q,
                        double *K_rows, int64_t *Nm_rows, double *decision, void *hip_stream)
{
    clear_error();
    if (!ctx || !res) { set_error("ctx/resident is NULL"); return GAKCO_EINVAL; }
    if (res->device != ctx->device) { set_error("resident set and context are on different devices"); return GAKCO_EINVAL; }
    GK_HIP(hipSetDevice(ctx->device));
    if (init_rows_attributes(ctx->lds_max) != hipSuccess) { set_error("hipFuncSetAttribute failed"); return GAKCO_EHIP; }
    return rows_run(ctx, res, q_seqs, q_lens, nullptr, n_q, K_rows, 0, Nm_rows, decision, (hipStream_t)hip_stream);
}

gakco_status gakco_server_create(const gakco_resident *res, int32_t device, int32_t max_batch, int32_t n_streams,
                                 size_t hbm_budget, gakco_server **out)
{
    clear_error();
    if (!res || !out || max_batch < 1 || n_streams < 1 || n_streams > 8) {
        set_error("bad arguments (max_batch >= 1, 1 <= n_streams <= 8)");
        return GAKCO_EINVAL;
    }
    if (device != res->device) { set_error("resident set lives on device %d", res->device); return GAKCO_EINVAL; }
    *out = nullptr;
    GK_HIP(hipSetDevice(device));
    auto *S = new gakco_server();
    S->res = res;
    S->device = device;
    S->max_batch = max_batch;
    S->n_streams = n_streams;
    size_t total = 0;
    GK_HIP(hipDeviceTotalMem(&total, device));
    S->budget = hbm_budget ? hbm_budget : total / 4;
    S->workers.resize((size_t)n_streams);
    for (auto &W : S->workers) {
        gakco_status s = gakco_ctx_create(device, S->budget / (size_t)n_streams, nullptr, &W.ctx);
        if (s == GAKCO_OK && (hipStreamCreateWithFlags(&W.st, hipStreamNonBlocking) != hipSuccess ||
                              hipEventCreateWithFlags(&W.ev, hipEventDisableTiming) != hipSuccess)) {
            set_error("hipStreamCreate / hipEventCreate failed");
            s = GAKCO_EHIP;
        }
        if (s == GAKCO_OK && init_rows_attributes(W.ctx->lds_max) != hipSuccess) {
            set_error("hipFuncSetAttribute failed");
            s = GAKCO_EHIP;
        }
        if (s != GAKCO_OK) {
            gakco_server_destroy(S);
            return s;
        }
    }
    size_t npos = 0;
    for (int m = 0; m <= res->M; ++m) npos += (size_t)binom64(res->g, m);
    for (auto &W : S->workers) warm_worker(S, W, S->budget / (size_t)n_streams, npos);
    for (int i = 0; i < n_streams; ++i) S->workers[(size_t)i].th = std::thread(worker_loop, S, i);
    *out = S;
    return GAKCO_OK;
}

gakco_status gakco_server_submit(gakco_server *S, const int8_t *q_host, int32_t len, uint64_t tag)
{
    clear_error();
    if (!S || len < 0 || (len > 0 && !q_host)) { set_error("bad arguments"); return GAKCO_EINVAL; }
    for (int32_t i = 0; i < len; ++i)
        if (q_host[i] < 0 || q_host[i] >= S->res->sigma) { set_error("symbol %d at %d outside [0, sigma)", q_host[i], i); return GAKCO_ERANGE; }
    // screened alone, so that an oversized query never fails the batch it
    // would have joined
    GK_TRY(check_query_bounds(S->res, len >= S->res->g ? (uint64_t)(len - S->res->g + 1) : 0u));
    SrvRequest r;
    r.tag = tag;
    r.q.assign(q_host, q_host + len);
    r.t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) { set_error("server is stopping"); return GAKCO_EINVAL; }
        S->queue.push_back(std::move(r));
    }
    S->cv_req.notify_one();
    return GAKCO_OK;
}

gakco_status gakco_server_set_param(gakco_server *S, const char *name, int64_t value)
{
    clear_error();
    if (!S || !name) { set_error("bad arguments"); return GAKCO_EINVAL; }
    std::unique_lock<std::mutex> lk(S->mu);  // held: no batch is admitted meanwhile
    S->cv_done.wait(lk, [&] { return S->running == 0; });
    // the first worker's context validates it (an error changes nothing);
    // the others, alike, then take it
    GK_TRY(gakco_ctx_set_param(S->workers[0].ctx, name, value));
    for (size_t i = 1; i < S->workers.size(); ++i) GK_TRY(gakco_ctx_set_param(S->workers[i].ctx, name, value));
    return GAKCO_OK;
}

gakco_status gakco_server_cancel(gakco_server *S, uint64_t tag)
{
    clear_error();
    if (!S) { set_error("server is NULL"); return GAKCO_EINVAL; }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
            if (it->tag != tag) continue;
            SrvResult rr{};
            rr.r.tag = tag;
            rr.r.status = GAKCO_ECANCELLED;
            rr.r.t_submit = it->t_submit;
            rr.r.t_start = rr.r.t_done = now_s();
            S->queue.erase(it);
            S->done.push_back(std::move(rr));
            S->cv_done.notify_all();
            return GAKCO_OK;
        }
    }
    set_error("request %llu is not queued (running or finished)", (unsigned long long)tag);
    return GAKCO_EAGAIN;
}

gakco_status gakco_server_poll(gakco_server *S, gakco_result *out, int32_t max, int32_t *n_out, int32_t wait_us)
{
    clear_error();
    if (!S || !out || max < 1 || !n_out) { set_error("bad arguments"); return GAKCO_EINVAL; }
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->done.empty() && wait_us > 0)
        S->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), [&] { return !S->done.empty(); });
    S->polled.clear();
    int32_t n = 0;
    while (n < max && !S->done.empty()) {
        S->polled.push_back(std::move(S->done.front()));
        S->done.pop_front();
        ++n;
    }
    for (int32_t i = 0; i < n; ++i) {
        SrvResult &rr = S->polled[(size_t)i];
        out[i] = rr.r;
        out[i].K_row = rr.row.empty() ? nullptr : rr.row.data();
    }
    *n_out = n;
    return n ? GAKCO_OK : GAKCO_EAGAIN;
}

gakco_status gakco_server_destroy(gakco_server *S)
{
    if (!S) return GAKCO_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        // queued requests are cancelled; in-flight batches finish
        S->queue.clear();
    }
    S->cv_req.notify_all();
    for (auto &W : S->workers)
        if (W.th.joinable()) W.th.join();
    for (auto &W : S->workers) {
        if (W.st) {
            (void)hipStreamSynchronize(W.st);
            (void)hipStreamDestroy(W.st);
        }
        if (W.ev) (void)hipEventDestroy(W.ev);
        if (W.ctx) {
            rows_scratch_release(W.ctx);
            gakco_ctx_destroy(W.ctx);
        }
        if (W.h_q) (void)hipHostFree(W.h_q);
        if (W.h_lens) (void)hipHostFree(W.h_lens);
        if (W.h_out) (void)hipHostFree(W.h_out);
        if (W.d_buf) (void)hipFree(W.d_buf);
    }
    delete S;
    return GAKCO_OK;
}

}  // extern "C"
