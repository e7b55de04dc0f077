// C ABI of the library: context, Gram, stage entry points.
#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <vector>
#include <map>

#include "launch.h"
#include "plan.h"

namespace gk {
const char *last_error();
void clear_error();
hipError_t init_kernel_attributes(size_t acc_lds);
}  // namespace gk

using namespace gk;

void rows_scratch_release(const gakco_ctx *ctx);

static gakco_status apply_param(gakco_ctx *ctx, const char *name, int64_t v)
{
    if (!strcmp(name, "dense_tau")) {
        if (v < 0) { set_error("dense_tau must be >= 0"); return GAKCO_EINVAL; }
        ctx->dense_tau = (int)v;
    } else if (!strcmp(name, "profile")) {
        ctx->prof_on = v != 0;
        if (ctx->prof_on && !ctx->prof_stat) {
            GK_HIP(hipSetDevice(ctx->device));
            GK_HIP(hipMalloc(&ctx->prof_stat, kProfStatSlots * sizeof(unsigned long long)));
            GK_HIP(hipMemset(ctx->prof_stat, 0, kProfStatSlots * sizeof(unsigned long long)));
        }
    } else if (!strcmp(name, "pool_mb")) {
        if (v < 16) { set_error("pool_mb must be >= 16"); return GAKCO_EINVAL; }
        ctx->pool_cap = (size_t)v << 20;
    } else if (!strncmp(name, "tau_b", 5)) {
        int b = 0, g = 0;
        if (sscanf(name, "tau_b%d_g%d", &b, &g) != 2 || b < 1 || g < 1 || v < 0) {
            set_error("bad class parameter '%s'", name);
            return GAKCO_EINVAL;
        }
        ctx->class_tau[b * 100 + g] = (int)v;
    } else if (!strcmp(name, "direct")) {
        if (v < 0 || v > 2) { set_error("direct must be 0, 1 or 2"); return GAKCO_EINVAL; }
        ctx->direct_mode = (int)v;
    } else if (!strcmp(name, "excess_cap")) {
        if (v < 0 || v > (int64_t)kExcessCap) { set_error("excess_cap must be in 0..%u", kExcessCap); return GAKCO_EINVAL; }
        ctx->excess_cap = (uint32_t)v;
    } else if (!strcmp(name, "info4")) {
        if (v < 0 || v > 1) { set_error("info4 must be 0 or 1"); return GAKCO_EINVAL; }
        ctx->info4 = (int)v;
    } else if (!strcmp(name, "chunk_masks")) {
        if (v < 0 || v > (1 << 20)) { set_error("chunk_masks must be in 0..1048576"); return GAKCO_EINVAL; }
        ctx->chunk_masks = (int)v;
    } else if (!strcmp(name, "overlap")) {
        ctx->overlap = v != 0;
    } else if (!strcmp(name, "bucket_avg")) {
        if (v < 16 || v > 4096) { set_error("bucket_avg must be in 16..4096"); return GAKCO_EINVAL; }
        ctx->bucket_avg = (int)v;
    } else if (!strcmp(name, "rows_dense")) {
        if (v < 0 || v > 1) { set_error("rows_dense must be 0 or 1"); return GAKCO_EINVAL; }
        ctx->rows_dense = (int)v;
    } else if (!strcmp(name, "rows_dense_min_sv")) {
        if (v < 1 || v > (1 << 24)) { set_error("rows_dense_min_sv must be in 1..2^24"); return GAKCO_EINVAL; }
        ctx->rows_dense_min_sv = (int)v;
    } else if (!strcmp(name, "rows_dense_min_q")) {
        if (v < 1 || v > (1 << 24)) { set_error("rows_dense_min_q must be in 1..2^24"); return GAKCO_EINVAL; }
        ctx->rows_dense_min_q = (int)v;
    } else if (!strcmp(name, "rows_slabs")) {
        if (v < 0 || v > 64) { set_error("rows_slabs must be in 0..64"); return GAKCO_EINVAL; }
        ctx->rows_slabs = (int)v;
    } else if (!strcmp(name, "acc_mstep")) {
        if (v < 0 || v > (1 << 20)) { set_error("acc_mstep must be in 0..1048576"); return GAKCO_EINVAL; }
        ctx->acc_mstep = (int)v;
    } else if (!strcmp(name, "acc_slab")) {
        if (v != 0 && (v < 64 || v > (1 << 20) || v % 64)) {
            set_error("acc_slab must be 0 or a multiple of 64 in 64..1048576");
            return GAKCO_EINVAL;
        }
        ctx->acc_slab = (int)v;
    } else {
        set_error("unknown parameter '%s'", name);
        return GAKCO_EINVAL;
    }
    return GAKCO_OK;
}

// Minimal reader of a flat JSON object of integer values.
static gakco_status apply_json(gakco_ctx *ctx, const char *js)
{
    const char *p = js;
    while ((p = strchr(p, '"')) != nullptr) {
        const char *q = strchr(p + 1, '"');
        if (!q) break;
        std::string key(p + 1, (size_t)(q - p - 1));
        const char *c = strchr(q, ':');
        if (!c) break;
        char *end = nullptr;
        const long long v = strtoll(c + 1, &end, 10);
        if (end == c + 1) { set_error("tune json: value of '%s' is not an integer", key.c_str()); return GAKCO_EINVAL; }
        GK_TRY(apply_param(ctx, key.c_str(), v));
        p = end;
    }
    return GAKCO_OK;
}

namespace gk {
// Lays out, binds, launches and checks a planned call.  When the directly
// addressed position sets hold more counts above 127 than the call's list
// takes, the call is redone with those levels sorted instead (same result).
gakco_status run_single(gakco_ctx *ctx, Plan &p, hipStream_t st)
{
    GK_TRY(plan_layout(ctx, p));
    GK_TRY(plan_bind(ctx, p, st));
    GK_TRY(plan_upload(p, st));
    GK_TRY(plan_launch(ctx, p, st));
    gakco_status s = plan_check_errors(ctx, p, st);
    if (p.excess_overflow && ctx->direct_mode != 0) {
        clear_error();
        const int saved = ctx->direct_mode;
        ctx->direct_mode = 0;
        ctx->direct_fallbacks += 1;
        p.excess_overflow = false;
        s = run_single(ctx, p, st);
        ctx->direct_mode = saved;
    }
    return s;
}
}  // namespace gk

extern "C" {

const char *gakco_last_error(void) { return last_error(); }
const char *gakco_version(void) { return "gakco-mi355x 0.1 (gfx950)"; }

gakco_status gakco_ctx_create(int device, size_t hbm_budget, const char *tune_json, gakco_ctx **out)
{
    clear_error();
    if (!out) { set_error("out is NULL"); return GAKCO_EINVAL; }
    *out = nullptr;
    int ndev = 0;
    GK_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) { set_error("device %d out of range (%d devices)", device, ndev); return GAKCO_EINVAL; }
    GK_HIP(hipSetDevice(device));
    size_t total = 0;
    GK_HIP(hipDeviceTotalMem(&total, device));
    int lds = 0;
    GK_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    auto *ctx = new gakco_ctx();
    ctx->device = device;
    ctx->budget = hbm_budget ? hbm_budget : total / 2;
    ctx->dense_tau = 192;  // measured best of 48..1024 on the protein workload
    // the row accumulation keeps ~5 KB of static LDS next to its rows
    ctx->lds_max = (size_t)lds > 8192 ? (size_t)lds - 8192 : 0;
    if (tune_json) {
        gakco_status s = apply_json(ctx, tune_json);
        if (s != GAKCO_OK) { delete ctx; return s; }
    }
    if (init_kernel_attributes(ctx->lds_max) != hipSuccess) {
        set_error("hipFuncSetAttribute failed");
        delete ctx;
        return GAKCO_EHIP;
    }
    bool ok = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; i < 2 && ok; ++i)
        ok = hipEventCreateWithFlags(&ctx->fork_ev[i], hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&ctx->join_ev[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        set_error("creating the side stream failed");
        gakco_ctx_destroy(ctx);
        return GAKCO_EHIP;
    }
    *out = ctx;
    return GAKCO_OK;
}

void gakco_ctx_destroy(gakco_ctx *ctx)
{
    if (!ctx) return;
    rows_scratch_release(ctx);
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->side) {
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->side);
        (void)hipStreamDestroy(ctx->side);
    }
    for (int i = 0; i < 2; ++i) {
        if (ctx->fork_ev[i]) (void)hipEventDestroy(ctx->fork_ev[i]);
        if (ctx->join_ev[i]) (void)hipEventDestroy(ctx->join_ev[i]);
    }
    if (ctx->prof_stat) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->prof_stat);
    }
    if (ctx->dense_buf) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->dense_buf);
    }
    if (ctx->arena) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->arena);
    }
    if (ctx->small) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->small);
    }
    delete ctx;
}

gakco_status gakco_ctx_set_param(gakco_ctx *ctx, const char *name, int64_t value)
{
    clear_error();
    if (!ctx || !name) { set_error("ctx/name is NULL"); return GAKCO_EINVAL; }
    return apply_param(ctx, name, value);
}

gakco_status gakco_count_gmers(const int32_t *lens_host, int32_t N, int32_t g, int64_t *T_out)
{
    clear_error();
    if (!T_out || N < 0 || g < 1 || (N > 0 && !lens_host)) { set_error("bad arguments"); return GAKCO_EINVAL; }
    int64_t T = 0;
    for (int i = 0; i < N; ++i) {
        if (lens_host[i] < 0) { set_error("lens[%d] is negative", i); return GAKCO_EINVAL; }
        T += lens_host[i] >= g ? lens_host[i] - g + 1 : 0;
    }
    *T_out = T;
    return GAKCO_OK;
}

gakco_status gakco_gram(gakco_ctx *ctx, const int8_t *seqs, const int32_t *lens, int32_t N, int32_t sigma, int32_t g,
                        int32_t k, double *K_out, int64_t *Nm_out, int64_t *Cm_out, void *hip_stream)
{
    clear_error();
    if (!ctx) { set_error("ctx is NULL"); return GAKCO_EINVAL; }
    GK_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    Plan p;
    p.jobs.resize(1);
    JobPlan &jp = p.jobs[0];
    jp.seqs = seqs; jp.lens_dev = lens; jp.N = N; jp.sigma = sigma; jp.g = g; jp.k = k;
    jp.K_out = K_out; jp.Nm_out = Nm_out; jp.Cm_out = Cm_out;
    if (N < 1) { set_error("N must be >= 1 (got %d)", N); return GAKCO_EINVAL; }
    if (!seqs || !lens) { set_error("seqs and lens must not be NULL"); return GAKCO_EINVAL; }
    GK_TRY(fetch_lens(jp, st));
    GK_TRY(plan_shape(ctx, jp, nullptr, 0));
    return run_single(ctx, p, st);
}

gakco_status gakco_extract(gakco_ctx *ctx, const int8_t *seqs, const int32_t *lens, int32_t N, int32_t sigma, int32_t g,
                           uint64_t *keys_out, int32_t *sid_out, void *hip_stream)
{
    clear_error();
    if (!ctx) { set_error("ctx is NULL"); return GAKCO_EINVAL; }
    GK_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    Plan p;
    p.jobs.resize(1);
    JobPlan &jp = p.jobs[0];
    jp.seqs = seqs; jp.lens_dev = lens; jp.N = N; jp.sigma = sigma; jp.g = g; jp.k = g;
    jp.want_kernel = false;
    if (N < 1 || !seqs || !lens) { set_error("bad arguments"); return GAKCO_EINVAL; }
    GK_TRY(fetch_lens(jp, st));
    GK_TRY(plan_shape(ctx, jp, nullptr, 0));
    jp.masks.clear();  // extraction only
    if (jp.T && (!keys_out || !sid_out)) { set_error("keys_out/sid_out must not be NULL"); return GAKCO_EINVAL; }
    jp.key_override = keys_out;
    jp.sid_override = reinterpret_cast<uint32_t *>(sid_out);
    GK_TRY(plan_layout(ctx, p));
    GK_TRY(plan_bind(ctx, p, st));
    GK_TRY(plan_upload(p, st));
    GK_TRY(plan_launch(ctx, p, st));
    return plan_check_errors(ctx, p, st);
}

gakco_status gakco_mask_groups(gakco_ctx *ctx, const int8_t *seqs, const int32_t *lens, int32_t N, int32_t sigma,
                               int32_t g, const int32_t *removed_host, int32_t m, int32_t *grp_off, int32_t *grp_rep,
                               int32_t *ent_sid, int32_t *ent_cnt, int64_t cap, int64_t *n_groups_out, void *hip_stream)
{
    clear_error();
    if (!ctx) { set_error("ctx is NULL"); return GAKCO_EINVAL; }
    if (m < 0 || m > g || (m > 0 && !removed_host) || !grp_off || !grp_rep || !ent_sid || !ent_cnt || !n_groups_out) {
        set_error("bad arguments");
        return GAKCO_EINVAL;
    }
    GK_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    Plan p;
    p.jobs.resize(1);
    JobPlan &jp = p.jobs[0];
    jp.seqs = seqs; jp.lens_dev = lens; jp.N = N; jp.sigma = sigma; jp.g = g; jp.k = g - m;
    jp.want_kernel = false;
    if (N < 1 || !seqs || !lens) { set_error("bad arguments"); return GAKCO_EINVAL; }
    GK_TRY(fetch_lens(jp, st));
    static const int32_t none[1] = {0};
    GK_TRY(plan_shape(ctx, jp, m ? removed_host : none, m));
    GK_TRY(plan_layout(ctx, p));
    GK_TRY(plan_bind(ctx, p, st));
    GK_TRY(plan_upload(p, st));
    GK_TRY(plan_launch(ctx, p, st));
    GK_TRY(plan_check_errors(ctx, p, st));
    const MaskWork &W = p.mw[0];
    const uint32_t T = jp.T;
    std::vector<uint32_t> E(T);
    std::vector<uint2> info(T);
    if (T) {
        GK_HIP(hipMemcpyAsync(E.data(), W.E, (size_t)T * 4, hipMemcpyDeviceToHost, st));
        GK_HIP(hipMemcpyAsync(info.data(), W.info, (size_t)T * 8, hipMemcpyDeviceToHost, st));
        GK_HIP(hipStreamSynchronize(st));
    }
    // a group is [first entry, end): its first entry's leader has the
    // longest tail; every leader of the group shares the same end
    std::map<uint32_t, std::pair<uint32_t, uint32_t>> groups;  // end -> (first entry, rep g-mer)
    for (uint32_t t = 0; t < T; ++t) {
        const uint32_t len = info[t].y & (uint32_t)((2ull << jp.sb) - 1);
        if (!len) continue;
        const uint32_t end = info[t].x + len;
        auto it = groups.find(end);
        if (it == groups.end() || info[t].x < it->second.first) groups[end] = {info[t].x, t};
    }
    const uint32_t sidmask = (uint32_t)((1ull << jp.sb) - 1);
    int64_t ng = 0, ne = 0;
    grp_off[0] = 0;
    for (auto &kv : groups) {
        const uint32_t a = kv.second.first, b = kv.first;
        if (ng + 1 > cap || ne + (int64_t)(b - a) > cap) { set_error("cap %lld too small", (long long)cap); return GAKCO_EINVAL; }
        grp_rep[ng] = (int32_t)kv.second.second;
        for (uint32_t e = a; e < b; ++e, ++ne) {
            ent_sid[ne] = (int32_t)(E[e] & sidmask);
            ent_cnt[ne] = (int32_t)(E[e] >> jp.sb);
        }
        ++ng;
        grp_off[ng] = (int32_t)ne;
    }
    *n_groups_out = ng;
    return GAKCO_OK;
}

gakco_status gakco_ctx_stat(const gakco_ctx *ctx, const char *name, int64_t *value)
{
    clear_error();
    if (!ctx || !name || !value) { set_error("bad arguments"); return GAKCO_EINVAL; }
    if (!strcmp(name, "dense_rows")) *value = ctx->last_dense_rows;
    else if (!strcmp(name, "chunks")) *value = ctx->last_chunks;
    else if (!strcmp(name, "excess")) *value = ctx->last_excess;
    else if (!strcmp(name, "direct")) *value = ctx->direct_mode;
    else if (!strcmp(name, "direct_levels")) *value = ctx->last_direct_levels;
    else if (!strcmp(name, "direct_fallbacks")) *value = ctx->direct_fallbacks;
    else if (!strcmp(name, "dense_tau")) *value = ctx->dense_tau;
    else if (!strcmp(name, "bucket_avg")) *value = ctx->bucket_avg;
    else if (!strcmp(name, "arena_bytes")) *value = (int64_t)ctx->arena_cap;
    else if (!strcmp(name, "dense_bytes")) *value = (int64_t)ctx->dense_cap;
    else if (!strncmp(name, "sort_gmers_", 11) || !strcmp(name, "acc_updates") || !strcmp(name, "rows_updates")) {
        // g-mers handled by each sort kernel, or pair updates of the row
        // accumulation, since the last profile reset.  Slots: the six sort
        // kinds, then kProfUpdSlots slots of pair updates (block b adds to
        // slot b % kProfUpdSlots)
        static const char *kinds[6] = {"wave", "wave_wide", "block", "block_wide", "global", "global_wide"};
        int k = -1, nk = 1;
        if (!strcmp(name, "acc_updates")) {
            k = kProfUpdFirst;
            nk = kProfUpdSlots;
        } else if (!strcmp(name, "rows_updates")) {
            k = kProfRowsFirst;
            nk = kProfUpdSlots;
        }
        for (int i = 0; i < 6 && k < 0; ++i)
            if (!strcmp(name + 11, kinds[i])) k = i;
        if (k < 0) { set_error("unknown statistic '%s'", name); return GAKCO_EINVAL; }
        std::vector<unsigned long long> v((size_t)nk, 0ull);
        if (ctx->prof_stat) {
            if (hipSetDevice(ctx->device) != hipSuccess ||
                hipMemcpy(v.data(), ctx->prof_stat + k, sizeof(unsigned long long) * v.size(), hipMemcpyDeviceToHost) !=
                    hipSuccess) {
                set_error("reading the profiling counters failed");
                return GAKCO_EHIP;
            }
        }
        unsigned long long sum = 0;
        for (auto x : v) sum += x;
        *value = (int64_t)sum;
    }
    else { set_error("unknown statistic '%s'", name); return GAKCO_EINVAL; }
    return GAKCO_OK;
}

int32_t gakco_profile_phases(void) { return PH_COUNT; }

gakco_status gakco_profile_get(const gakco_ctx *ctx, int32_t phase, const char **name, double *total_ms,
                               int64_t *launches)
{
    clear_error();
    if (!ctx || phase < 0 || phase >= PH_COUNT) { set_error("bad arguments"); return GAKCO_EINVAL; }
    if (name) *name = phase_name(phase);
    if (total_ms) *total_ms = ctx->prof_ms[phase];
    if (launches) *launches = ctx->prof_n[phase];
    return GAKCO_OK;
}

gakco_status gakco_probe_lds_atomics(gakco_ctx *ctx, int32_t row_words, double *updates_per_s)
{
    clear_error();
    if (!ctx || !updates_per_s || row_words < 64 || row_words > 8192 || (row_words & (row_words - 1))) {
        set_error("row_words must be a power of two in 64..8192");
        return GAKCO_EINVAL;
    }
    GK_HIP(hipSetDevice(ctx->device));
    GK_HIP(probe_lds_atomics(row_words, updates_per_s));
    return GAKCO_OK;
}

void gakco_profile_reset(gakco_ctx *ctx)
{
    if (!ctx) return;
    for (int i = 0; i < PH_COUNT; ++i) {
        ctx->prof_ms[i] = 0;
        ctx->prof_n[i] = 0;
    }
    if (ctx->prof_stat && hipSetDevice(ctx->device) == hipSuccess)
        (void)hipMemset(ctx->prof_stat, 0, kProfStatSlots * sizeof(unsigned long long));
}

}  // extern "C"
