// Batched Gram jobs, hipGraph-replayed batch plans, and the autotuner.
//
// All jobs of a batch are planned together: their position sets share the
// partition / sort / accumulation launches (work items of every job in one
// grid), so many small jobs fill the GPU that one of them alone would leave
// idle.  A batch plan captures that launch sequence once into a hipGraph on a
// private stream and owns its memory, so replays cost one graph launch.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>

#include "plan.h"

namespace gk {
void clear_error();
}
using namespace gk;

struct gakco_batch_plan {
    gakco_ctx own;  // private arena and count buffers, parameters copied from the creating context
    Plan p;
    std::vector<gakco_status *> status_out;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static int class_tau(const gakco_ctx *ctx, int b, int g)
{
    auto it = ctx->class_tau.find(b * 100 + g);
    return it == ctx->class_tau.end() ? -1 : it->second;
}

// Fills p.jobs from the job list; jobs that fail validation get their status
// and are left out of the plan (index map in `keep`).
static gakco_status prepare_jobs(gakco_ctx *ctx, const gakco_job *jobs, int n, hipStream_t st, Plan &p,
                                 std::vector<int> &keep, std::vector<gakco_status> &status)
{
    if (n < 1 || !jobs) { set_error("n_jobs must be >= 1 and jobs non-NULL"); return GAKCO_EINVAL; }
    status.assign((size_t)n, GAKCO_OK);
    std::vector<JobPlan> all((size_t)n);
    for (int i = 0; i < n; ++i) {
        JobPlan &jp = all[(size_t)i];
        jp.seqs = jobs[i].seqs;
        jp.lens_dev = jobs[i].lens;
        jp.N = jobs[i].N;
        jp.sigma = jobs[i].sigma;
        jp.g = jobs[i].g;
        jp.k = jobs[i].k;
        jp.K_out = jobs[i].K_out;
        jp.Nm_out = jobs[i].Nm_out;
        if (jp.N >= 1 && jp.lens_dev) {
            jp.lens.assign((size_t)jp.N, 0);
            GK_HIP(hipMemcpyAsync(jp.lens.data(), jp.lens_dev, sizeof(int32_t) * (size_t)jp.N, hipMemcpyDeviceToHost, st));
        }
    }
    GK_HIP(hipStreamSynchronize(st));
    gakco_status first = GAKCO_OK;
    for (int i = 0; i < n; ++i) {
        JobPlan &jp = all[(size_t)i];
        gakco_status s = plan_shape(ctx, jp, nullptr, 0);
        if (s == GAKCO_OK) {
            jp.tau = class_tau(ctx, jp.b, jp.g);
            keep.push_back(i);
            p.jobs.push_back(std::move(jp));
        } else {
            status[(size_t)i] = s;
            if (first == GAKCO_OK) first = s;
        }
    }
    return first;
}

static void write_status(const gakco_job *jobs, int n, const std::vector<gakco_status> &status)
{
    for (int i = 0; i < n; ++i)
        if (jobs[i].status_out) *jobs[i].status_out = status[(size_t)i];
}

extern "C" {

gakco_status gakco_gram_batch(gakco_ctx *ctx, const gakco_job *jobs_host, int32_t n_jobs, void *hip_stream)
{
    clear_error();
    if (!ctx) { set_error("ctx is NULL"); return GAKCO_EINVAL; }
    GK_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    Plan p;
    std::vector<int> keep;
    std::vector<gakco_status> status;
    gakco_status first = prepare_jobs(ctx, jobs_host, n_jobs, st, p, keep, status);
    if (status.empty()) return first;
    if (!p.jobs.empty()) {
        gakco_status s = run_single(ctx, p, st);
        for (size_t q = 0; q < keep.size(); ++q)
            status[(size_t)keep[q]] = (s == GAKCO_OK || s == GAKCO_ERANGE) ? p.jobs[q].status : s;
        if (first == GAKCO_OK) first = s;
    }
    write_status(jobs_host, n_jobs, status);
    return first;
}

gakco_status gakco_batch_plan_create(gakco_ctx *ctx, const gakco_job *jobs_host, int32_t n_jobs, void *hip_stream,
                                     gakco_batch_plan **out)
{
    clear_error();
    if (!ctx || !out) { set_error("ctx/out is NULL"); return GAKCO_EINVAL; }
    *out = nullptr;
    GK_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    auto *bp = new gakco_batch_plan();
    gakco_ctx &own = bp->own;
    own.device = ctx->device;
    own.budget = ctx->budget;
    own.dense_tau = ctx->dense_tau;
    own.bucket_avg = ctx->bucket_avg;
    own.acc_slab = ctx->acc_slab;
    own.acc_mstep = ctx->acc_mstep;
    own.direct_mode = ctx->direct_mode;
    own.excess_cap = ctx->excess_cap;
    own.chunk_masks = ctx->chunk_masks;
    own.info4 = ctx->info4;
    own.overlap = ctx->overlap;
    own.pool_cap = ctx->pool_cap;
    own.lds_max = ctx->lds_max;
    own.class_tau = ctx->class_tau;
    own.prof_on = false;
    auto fail = [&](gakco_status s) {
        gakco_batch_plan_destroy(bp);
        return s;
    };
    std::vector<int> keep;
    std::vector<gakco_status> status;
    gakco_status s = prepare_jobs(&own, jobs_host, n_jobs, st, bp->p, keep, status);
    if (s != GAKCO_OK) return fail(s);
    for (int i = 0; i < n_jobs; ++i) bp->status_out.push_back(jobs_host[i].status_out);
    if ((s = plan_layout(&own, bp->p)) != GAKCO_OK) return fail(s);
    if ((s = plan_bind(&own, bp->p, st)) != GAKCO_OK) return fail(s);
    if ((s = plan_upload(bp->p, st)) != GAKCO_OK) return fail(s);
    if (hipStreamSynchronize(st) != hipSuccess || hipStreamCreateWithFlags(&bp->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        set_error("stream setup for the batch graph failed");
        return fail(GAKCO_EHIP);
    }
    // the independent kernels of the plan (block beside wave sort, int8
    // products beside the last accumulation) fork onto a second stream that
    // joins the capture, so the graph keeps their overlap
    if (own.overlap) {
        bool ok = hipStreamCreateWithFlags(&own.side, hipStreamNonBlocking) == hipSuccess;
        for (int i = 0; i < 2 && ok; ++i)
            ok = hipEventCreateWithFlags(&own.fork_ev[i], hipEventDisableTiming) == hipSuccess &&
                 hipEventCreateWithFlags(&own.join_ev[i], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            set_error("side stream setup for the batch graph failed");
            return fail(GAKCO_EHIP);
        }
        own.capture_side = true;
    }
    if (hipStreamBeginCapture(bp->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        set_error("hipStreamBeginCapture failed");
        return fail(GAKCO_EHIP);
    }
    s = plan_launch(&own, bp->p, bp->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(bp->cap_stream, &g);
    bp->graph = g;
    if (s != GAKCO_OK) return fail(s);
    if (ec != hipSuccess || !g) { set_error("hipStreamEndCapture failed: %s", hipGetErrorString(ec)); return fail(GAKCO_EHIP); }
    if (hipGraphInstantiate(&bp->exec, bp->graph, nullptr, nullptr, 0) != hipSuccess) {
        set_error("hipGraphInstantiate failed");
        return fail(GAKCO_EHIP);
    }
    *out = bp;
    return GAKCO_OK;
}

gakco_status gakco_batch_run(gakco_batch_plan *bp, void *hip_stream)
{
    clear_error();
    if (!bp || !bp->exec) { set_error("plan is NULL or not instantiated"); return GAKCO_EINVAL; }
    GK_HIP(hipSetDevice(bp->own.device));
    hipStream_t st = (hipStream_t)hip_stream;
    GK_HIP(hipGraphLaunch(bp->exec, st));
    gakco_status s = plan_check_errors(&bp->own, bp->p, st);
    if (bp->p.excess_overflow) {
        // more counts above 127 in directly addressed position sets than the
        // captured list takes: redo the jobs once with those levels sorted, in
        // a temporary context (the plan's own memory stays as the graph uses it)
        gakco_ctx tmp;
        tmp.device = bp->own.device;
        tmp.budget = bp->own.budget;
        tmp.dense_tau = bp->own.dense_tau;
        tmp.bucket_avg = bp->own.bucket_avg;
        tmp.acc_slab = bp->own.acc_slab;
        tmp.acc_mstep = bp->own.acc_mstep;
        tmp.pool_cap = bp->own.pool_cap;
        tmp.lds_max = bp->own.lds_max;
        tmp.class_tau = bp->own.class_tau;
        tmp.direct_mode = 0;
        tmp.info4 = bp->own.info4;
        bp->own.direct_fallbacks += 1;
        Plan q;
        q.jobs = bp->p.jobs;
        clear_error();
        s = run_single(&tmp, q, st);
        if (tmp.arena) (void)hipFree(tmp.arena);
        if (tmp.dense_buf) (void)hipFree(tmp.dense_buf);
        for (size_t i = 0; i < q.jobs.size(); ++i) bp->p.jobs[i].status = q.jobs[i].status;
        bp->p.excess_overflow = false;
    }
    // a plan exists only when every job passed planning: job i is p.jobs[i]
    for (size_t i = 0; i < bp->status_out.size(); ++i)
        if (bp->status_out[i]) *bp->status_out[i] = bp->p.jobs[i].status;
    return s;
}

void gakco_batch_plan_destroy(gakco_batch_plan *bp)
{
    if (!bp) return;
    (void)hipSetDevice(bp->own.device);
    if (bp->cap_stream) (void)hipStreamSynchronize(bp->cap_stream);
    (void)hipDeviceSynchronize();
    if (bp->exec) (void)hipGraphExecDestroy(bp->exec);
    if (bp->graph) (void)hipGraphDestroy(bp->graph);
    if (bp->cap_stream) (void)hipStreamDestroy(bp->cap_stream);
    if (bp->own.side) (void)hipStreamDestroy(bp->own.side);
    for (int i = 0; i < 2; ++i) {
        if (bp->own.fork_ev[i]) (void)hipEventDestroy(bp->own.fork_ev[i]);
        if (bp->own.join_ev[i]) (void)hipEventDestroy(bp->own.join_ev[i]);
    }
    if (bp->own.arena) (void)hipFree(bp->own.arena);
    if (bp->own.dense_buf) (void)hipFree(bp->own.dense_buf);
    for (auto e : bp->own.ev_pool) (void)hipEventDestroy(e);
    delete bp;
}

// Autotuner: times candidate settings on the device (HIP events around a
// batch run, best of `reps`) and keeps the fastest.  The int8 matrix-core
// threshold tau is chosen per job class (symbol bits b, g): the jobs of each
// class are timed alone for every candidate tau.  The bucket size is chosen
// once for the whole batch afterwards.  The result is applied to the context
// and written to out_json (nullable) as a flat object usable as tune_json.
gakco_status gakco_autotune(gakco_ctx *ctx, const gakco_job *jobs_host, int32_t n_jobs, int32_t reps, void *hip_stream,
                            char *out_json, size_t out_cap)
{
    clear_error();
    if (!ctx || !jobs_host || n_jobs < 1) { set_error("bad arguments"); return GAKCO_EINVAL; }
    GK_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    reps = std::max(1, reps);
    hipEvent_t e0, e1;
    GK_HIP(hipEventCreate(&e0));
    GK_HIP(hipEventCreate(&e1));
    auto time_batch = [&](const std::vector<gakco_job> &js, double *ms_out) -> gakco_status {
        double best = 1e30;
        for (int r = 0; r <= reps; ++r) {  // first run warms the arena
            GK_HIP(hipEventRecord(e0, st));
            gakco_status s = gakco_gram_batch(ctx, js.data(), (int32_t)js.size(), st);
            if (s != GAKCO_OK) return s;
            GK_HIP(hipEventRecord(e1, st));
            GK_HIP(hipEventSynchronize(e1));
            float ms = 0;
            GK_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (r) best = std::min(best, (double)ms);
        }
        *ms_out = best;
        return GAKCO_OK;
    };
    // classes of jobs by (b, g)
    std::map<int, std::vector<gakco_job>> classes;
    for (int i = 0; i < n_jobs; ++i) {
        gakco_job j = jobs_host[i];
        j.status_out = nullptr;
        classes[symbol_bits(j.sigma) * 100 + j.g].push_back(j);
    }
    const int taus[] = {0, 32, 64, 128, 192, 256, 512};
    std::string js = "{";
    char buf[128];
    for (auto &kv : classes) {
        double best = 1e30;
        int best_tau = ctx->dense_tau;
        for (int t : taus) {
            ctx->class_tau[kv.first] = t;
            double ms = 0;
            gakco_status s = time_batch(kv.second, &ms);
            if (s != GAKCO_OK) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return s; }
            if (ms < best) { best = ms; best_tau = t; }
        }
        ctx->class_tau[kv.first] = best_tau;
        snprintf(buf, sizeof buf, "%s\"tau_b%d_g%d\": %d", js.size() > 1 ? ", " : "", kv.first / 100, kv.first % 100, best_tau);
        js += buf;
    }
    std::vector<gakco_job> all;
    for (int i = 0; i < n_jobs; ++i) { all.push_back(jobs_host[i]); all.back().status_out = nullptr; }
    const int avgs[] = {512, 768, 1024};
    double best = 1e30;
    int best_avg = ctx->bucket_avg;
    for (int a : avgs) {
        ctx->bucket_avg = a;
        double ms = 0;
        gakco_status s = time_batch(all, &ms);
        if (s != GAKCO_OK) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); return s; }
        if (ms < best) { best = ms; best_avg = a; }
    }
    ctx->bucket_avg = best_avg;
    snprintf(buf, sizeof buf, "%s\"bucket_avg\": %d}", js.size() > 1 ? ", " : "", best_avg);
    js += buf;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (out_json) {
        if (js.size() + 1 > out_cap) { set_error("out_json too small (%zu bytes needed)", js.size() + 1); return GAKCO_EINVAL; }
        memcpy(out_json, js.c_str(), js.size() + 1);
    }
    return GAKCO_OK;
}

}  // extern "C"
